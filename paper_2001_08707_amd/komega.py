"""ctypes binding of libkomega_hip.so (include/komega_hip.h).

Argument marshalling only: every step of the solver runs in the HIP library.
PyTorch provides device memory (torch tensors on the GPU) and the stream.
If the library is not built, importing this module raises at once; there is
no CPU fallback.
"""
import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libkomega_hip.so")

OK, CONVERGED = 0, 1
E_INVALID, E_BREAKDOWN, E_SHIFT_BREAKDOWN, E_MAXITER = -1, -2, -3, -4
E_HIP, E_STATE, E_NONFINITE, E_NOMEM = -5, -6, -7, -8
CG_R, CG_C, COCG, BICG = 0, 1, 2, 3
METHODS = {"cg_r": CG_R, "cg_c": CG_C, "cocg": COCG, "bicg": BICG}
F_NO_SWITCH, F_HISTORY, F_GRAPH, F_X32 = 1, 2, 4, 8
K_SPMV, K_SEED, K_SHIFT, K_DOT = 0, 1, 2, 3
T_SHIFT_BLOCK, T_SHIFT_NT, T_SPMV_BLOCKS, T_SHIFT_ORDER, T_SHIFT_STEPS = 0, 1, 2, 3, 4
MAX_NL = 8
NOALLOC_MAX_VECTORS = 4096   # KOMEGA_NOALLOC_MAX_VECTORS


class KomegaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"komega status {status}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [
        ("method", C.c_int32), ("nz", C.c_int32), ("ndim", C.c_int64),
        ("nl", C.c_int32), ("nrhs", C.c_int32), ("itermax", C.c_int32), ("flags", C.c_uint32),
        ("tol", C.c_double), ("freeze_tol", C.c_double), ("stream", C.c_void_p),
    ]


class Iter(C.Structure):
    _fields_ = [("status", C.c_int32), ("iter", C.c_int32), ("seed", C.c_int32),
                ("nswitch", C.c_int32), ("maxres", C.c_double)]


APPLY_FN = C.CFUNCTYPE(C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p)

_vp = C.c_void_p
_pd = C.POINTER(C.c_double)
_SIGS = {
    "komega_create": [C.POINTER(_vp), C.POINTER(Params), _pd],
    "komega_create_batched": [C.POINTER(_vp), C.POINTER(Params), _pd, C.POINTER(C.c_int64)],
    "komega_init": [_vp, _vp, _vp, _vp, _vp],
    "komega_update": [_vp, _vp, _vp, _vp, _vp, C.POINTER(Iter)],
    "komega_iterate": [_vp, _vp, C.c_int32],
    "komega_solve": [_vp, _vp, C.c_int32, C.POINTER(Iter)],
    "komega_getstate": [_vp, C.POINTER(Iter)],
    "komega_getresidual": [_vp, _pd],
    "komega_getcoef": [_vp, C.c_int32, _pd, _pd, _pd, C.POINTER(C.c_int32), _pd, _pd, C.POINTER(C.c_int32)],
    "komega_finalize": [_vp],
    "komega_recalc": [_vp, C.c_int32, C.c_int32, _pd, _vp, _pd],
    "komega_state_size": [_vp, C.POINTER(C.c_int64)],
    "komega_save_state": [_vp, _vp, C.c_int64],
    "komega_restore_state": [_vp, _vp, C.c_int64, _vp, _vp],
    "komega_op_stencil3d": [C.POINTER(_vp), C.c_int32, C.c_int32, C.c_int32, C.c_double, _pd],
    "komega_op_stencil3d_batch": [C.POINTER(_vp), C.c_int32, C.POINTER(C.c_int32), C.c_double, _pd],
    "komega_op_csr": [C.POINTER(_vp), C.c_int64, C.POINTER(C.c_int64), C.POINTER(C.c_int32), _pd, C.c_int32],
    "komega_op_heisenberg": [C.POINTER(_vp), C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                             C.POINTER(C.c_int32), _pd],
    "komega_op_callback": [C.POINTER(_vp), C.c_int64, APPLY_FN, _vp],
    "komega_op_dim": [_vp, C.POINTER(C.c_int64)],
    "komega_op_apply": [_vp, _vp, _vp, C.c_int32, C.c_int32, _vp],
    "komega_op_heisenberg_states": [_vp, _vp, _vp],
    "komega_op_heisenberg_lookup": [_vp, _vp, _vp, C.c_int64, _vp],
    "komega_op_heisenberg_szq": [_vp, _pd, _vp, _vp, _vp],
    "komega_op_set_variant": [_vp, C.c_int32],
    "komega_op_heisenberg_bond_grad": [_vp, _vp, C.c_int64, _vp, C.c_int64, C.c_int32, _vp, _vp],
    "komega_dotc": [_vp, C.c_int64, _vp, C.c_int64, C.c_int64, C.c_int32, _vp, _vp],
    "komega_dotc_c64": [_vp, C.c_int64, _vp, C.c_int64, C.c_int64, C.c_int32, _vp, _vp],
    "komega_dotc_noalloc": [_vp, C.c_int64, _vp, C.c_int64, C.c_int64, C.c_int32, _vp, _vp],
    "komega_onsite_grad": [_vp, _vp, C.c_int64, _vp, C.c_int64, C.c_int64, C.c_int32, _vp, _vp],
    "komega_stream_probe": [_vp, _vp, C.c_int64, C.c_int32, _vp],
    "komega_stream_probe_groups": [],
    "komega_contour_moments": [_vp, C.c_int32, C.c_int64, C.c_int32, C.c_int32, _pd, _vp, _vp],
    "komega_op_destroy": [_vp],
    "komega_set_timing": [_vp, C.c_uint32],
    "komega_get_timing": [_vp, C.c_int32, _pd, C.POINTER(C.c_int64), C.c_int32],
    "komega_launch_info": [_vp, _vp, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64)],
    "komega_set_tuning": [_vp, C.c_int32, C.c_int32],
    "komega_get_tuning": [_vp, C.c_int32, C.POINTER(C.c_int32)],
}
EXPORTS = sorted(list(_SIGS) + ["komega_strerror", "komega_last_error"])


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2001_08707_amd.build` "
                          "(there is no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    for name, args in _SIGS.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int32
    lib.komega_strerror.argtypes = [C.c_int32]
    lib.komega_strerror.restype = C.c_char_p
    lib.komega_last_error.argtypes = []
    lib.komega_last_error.restype = C.c_char_p
    return lib


_lib = _load()


def _check(rc, ok=(OK,)):
    if rc in ok:
        return rc
    raise KomegaError(rc, f"{_lib.komega_strerror(rc).decode()}: {_lib.komega_last_error().decode()}")


def _ptr(t):
    """Raw device pointer.  Conjugate / negative views are lazy in PyTorch (the
    memory is not conjugated), so they are refused here: resolve them first."""
    if t is None:
        return None
    if t.is_conj() or t.is_neg():
        raise ValueError("tensor is a lazy conjugate/negative view; call .resolve_conj()/.resolve_neg()")
    return C.c_void_p(t.data_ptr())


def _resolved(t):
    return t.resolve_conj().resolve_neg().contiguous()


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_tensor(a, dtype, device):
    if isinstance(a, torch.Tensor):
        return _resolved(a.to(device=device, dtype=dtype))
    return torch.as_tensor(np.asarray(a), dtype=dtype, device=device).contiguous()


# ----------------------------------------------------------------------------
class Operator:
    """A built-in (or callback) operator H owned by the library."""

    def __init__(self, handle, M, kind, keep=None):
        self._h = handle
        self.M = int(M)
        self.kind = kind
        self._keep = keep

    @property
    def handle(self):
        return self._h

    @staticmethod
    def stencil3d(Lx, Ly, Lz, eps, hop=1.0):
        eps = np.ascontiguousarray(eps, dtype=np.float64)
        if eps.size != Lx * Ly * Lz:
            raise ValueError("eps must have Lx*Ly*Lz entries")
        h = C.c_void_p()
        _check(_lib.komega_op_stencil3d(C.byref(h), Lx, Ly, Lz, float(hop), eps.ctypes.data_as(_pd)))
        return Operator(h, eps.size, "stencil3d")

    @staticmethod
    def stencil3d_batch(L, eps, hop=1.0):
        """Independent cubes as one block-diagonal operator: L is [nsys, 3]
        edges, eps the concatenated on-site energies (or a list per cube)."""
        L = np.ascontiguousarray(np.asarray(L, dtype=np.int32).reshape(-1, 3))
        if isinstance(eps, (list, tuple)):
            eps = np.concatenate([np.asarray(e, dtype=np.float64).ravel() for e in eps])
        eps = np.ascontiguousarray(eps, dtype=np.float64)
        rows = np.prod(L.astype(np.int64), axis=1)
        if eps.size != rows.sum():
            raise ValueError("eps must have sum(Lx*Ly*Lz) entries")
        h = C.c_void_p()
        _check(_lib.komega_op_stencil3d_batch(C.byref(h), L.shape[0], L.ctypes.data_as(C.POINTER(C.c_int32)),
                                              float(hop), eps.ctypes.data_as(_pd)))
        op = Operator(h, eps.size, "stencil3d_batch")
        op.rows = rows
        return op

    @staticmethod
    def csr(rowptr, col, val):
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        val = np.asarray(val)
        cplx = np.iscomplexobj(val)
        val = np.ascontiguousarray(val, dtype=np.complex128 if cplx else np.float64)
        h = C.c_void_p()
        _check(_lib.komega_op_csr(C.byref(h), rowptr.size - 1, rowptr.ctypes.data_as(C.POINTER(C.c_int64)),
                                  col.ctypes.data_as(C.POINTER(C.c_int32)), val.ctypes.data_as(_pd),
                                  1 if cplx else 0))
        return Operator(h, rowptr.size - 1, "csr")

    @staticmethod
    def heisenberg(L, nup, bonds, J):
        bonds = np.asarray(bonds, dtype=np.int32).reshape(-1, 2)
        bi = np.ascontiguousarray(bonds[:, 0])
        bj = np.ascontiguousarray(bonds[:, 1])
        J = np.ascontiguousarray(np.broadcast_to(np.asarray(J, dtype=np.float64), (len(bonds),)))
        h = C.c_void_p()
        _check(_lib.komega_op_heisenberg(C.byref(h), L, nup, len(bonds), bi.ctypes.data_as(C.POINTER(C.c_int32)),
                                         bj.ctypes.data_as(C.POINTER(C.c_int32)), J.ctypes.data_as(_pd)))
        M = C.c_int64()
        _check(_lib.komega_op_dim(h, C.byref(M)))
        op = Operator(h, M.value, "heisenberg")
        op.L = L
        op.nb = len(bonds)
        return op

    @staticmethod
    def callback(M, fn):
        """fn(v, out, nvec, is_complex) with torch tensors; must enqueue out = H v
        on the current stream."""
        def tramp(user, v, out, nvec, is_complex, stream):
            try:
                dt = torch.complex128 if is_complex else torch.float64
                es = 16 if is_complex else 8
                vt = _wrap_device(v, nvec * M, dt, es)
                ot = _wrap_device(out, nvec * M, dt, es)
                fn(vt.view(nvec, M), ot.view(nvec, M), nvec, bool(is_complex))
                return 0
            except Exception:  # noqa: BLE001 -- reported to the library as failure
                return 1
        cb = APPLY_FN(tramp)
        h = C.c_void_p()
        _check(_lib.komega_op_callback(C.byref(h), int(M), cb, None))
        return Operator(h, M, "callback", keep=cb)

    def apply(self, v, out=None):
        v = _resolved(v)
        nvec = 1 if v.dim() == 1 else v.shape[0]
        if out is None:
            out = torch.empty_like(v)
        _check(_lib.komega_op_apply(self._h, _ptr(v), _ptr(out), nvec, 1 if v.is_complex() else 0, _stream()))
        return out

    def states(self, device="cuda"):
        out = torch.empty(self.M, dtype=torch.int32, device=device)
        _check(_lib.komega_op_heisenberg_states(self._h, _ptr(out), _stream()))
        return out  # uint32 bit patterns held in int32 (view as uint32 on the host)

    def lookup(self, states):
        states = _resolved(states)
        idx = torch.empty(states.numel(), dtype=torch.int64, device=states.device)
        _check(_lib.komega_op_heisenberg_lookup(self._h, _ptr(states), _ptr(idx), states.numel(), _stream()))
        return idx

    def szq(self, w, v):
        w = np.ascontiguousarray(np.asarray(w, dtype=np.complex128))
        v = _resolved(v.to(torch.complex128))
        out = torch.empty_like(v)
        _check(_lib.komega_op_heisenberg_szq(self._h, w.view(np.float64).ctypes.data_as(_pd), _ptr(v),
                                             _ptr(out), _stream()))
        return out

    def bond_grad(self, w, x):
        """out[k, b] = w_k^H (S_i . S_j)_b x_k for vector sets w, x [n, M] (device complex128)."""
        w = _resolved(w)
        x = _resolved(x)
        n = x.shape[0]
        out = torch.empty((n, self.nb), dtype=torch.complex128, device=x.device)
        _check(_lib.komega_op_heisenberg_bond_grad(self._h, _ptr(w), w.stride(0), _ptr(x), x.stride(0), n,
                                                   _ptr(out), _stream()))
        return out

    def set_variant(self, variant):
        """Heisenberg product kernel: 0 auto, 1 row kernel, 2 group kernel."""
        _check(_lib.komega_op_set_variant(self._h, int(variant)))

    def close(self):
        if self._h:
            _lib.komega_op_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass


def _wrap_device(ptr, n, dtype, es):
    """A torch view of n elements of device memory at ptr (no copy)."""
    class _Arr:
        __cuda_array_interface__ = {
            "shape": (n,), "typestr": "<c16" if es == 16 else "<f8", "data": (ptr, False), "version": 2,
        }
    return torch.as_tensor(_Arr(), device="cuda")


# ----------------------------------------------------------------------------
class Solver:
    """Shifted Krylov solver handle.

    method: 'cocg' | 'bicg' | 'cg_c' | 'cg_r';  z: shifts;  ndim: M;
    nl: 0 keeps every x^(k), else the number of projection rows.
    rows: sizes of independent batched systems (ndim = their sum; vectors are
    concatenated and whole-x output is flat, see system_x).
    x32: keep x^(k), p^(k) as complex64 (whole-x mode).
    """

    def __init__(self, method, z, ndim=None, nl=0, nrhs=1, tol=1e-10, itermax=10000, freeze_tol=-1.0,
                 switch=True, history=False, graph=False, stream=None, rows=None, x32=False):
        z = np.ascontiguousarray(np.asarray(z, dtype=np.complex128).ravel())
        self.method = METHODS[method] if isinstance(method, str) else int(method)
        self.rows = None
        if rows is not None:
            self.rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64).ravel())
            self.offsets = np.concatenate([[0], np.cumsum(self.rows)]).astype(np.int64)
            if ndim is not None and int(ndim) != int(self.rows.sum()):
                raise ValueError("ndim must equal sum(rows)")
            ndim, nrhs = int(self.rows.sum()), self.rows.size
        self.nz, self.ndim, self.nl, self.nrhs = z.size, int(ndim), int(nl), int(nrhs)
        self.itermax = int(itermax)
        self.z = z
        self.x32 = bool(x32)
        p = Params()
        p.method, p.nz, p.ndim, p.nl, p.nrhs, p.itermax = self.method, self.nz, self.ndim, self.nl, self.nrhs, self.itermax
        p.flags = ((0 if switch else F_NO_SWITCH) | (F_HISTORY if history else 0) | (F_GRAPH if graph else 0)
                   | (F_X32 if x32 else 0))
        p.tol, p.freeze_tol = float(tol), float(freeze_tol)
        self._stream_obj = stream if stream is not None else torch.cuda.current_stream()
        p.stream = C.c_void_p(self._stream_obj.cuda_stream)
        h = C.c_void_p()
        zp = z.view(np.float64).ctypes.data_as(_pd)
        if self.rows is not None:
            _check(_lib.komega_create_batched(C.byref(h), C.byref(p), zp,
                                              self.rows.ctypes.data_as(C.POINTER(C.c_int64))))
        else:
            _check(_lib.komega_create(C.byref(h), C.byref(p), zp))
        self._h = h
        self.dtype = torch.float64 if self.method == CG_R else torch.complex128
        self.x = None
        self._keep = []

    def _vec_shape(self):
        return (self.ndim,) if self.rows is not None else (self.nrhs, self.ndim)

    def _out_shape(self):
        """Output buffer shape and dtype for the current mode."""
        if self.nl > 0:
            return (self.nrhs, self.nz, self.nl), torch.complex128
        xdt = torch.complex64 if self.x32 else self.dtype
        if self.rows is not None:
            return (self.nz * self.ndim,), xdt
        return (self.nrhs, self.nz, self.ndim), xdt

    def system_x(self, r, x=None):
        """Kept solutions [nz, M_r] of batched system r (a view of x)."""
        x = self.x if x is None else x
        o, m = int(self.offsets[r]), int(self.rows[r])
        return x[self.nz * o: self.nz * (o + m)].view(self.nz, m)

    def system_rows(self, v, r):
        """Rows of batched system r in a concatenated vector v."""
        o, m = int(self.offsets[r]), int(self.rows[r])
        return v[o: o + m]

    @property
    def handle(self):
        return self._h

    def init(self, b, P=None, bshadow=None, x=None):
        dev = "cuda"
        b = _dev_tensor(b, self.dtype, dev).reshape(self._vec_shape())
        if self.nl > 0:
            if P is None:
                raise ValueError("projected mode needs P")
            P = _dev_tensor(P, self.dtype, dev).reshape(self.nl, self.ndim)
        else:
            P = None
        shape, xdt = self._out_shape()
        if x is None:
            x = torch.empty(shape, dtype=xdt, device=dev)
        elif x.dtype != xdt or x.numel() != int(np.prod(shape)) or not x.is_contiguous():
            raise ValueError(f"x must be a contiguous {xdt} tensor of {int(np.prod(shape))} elements")
        bs = _dev_tensor(bshadow, self.dtype, dev).reshape(self._vec_shape()) if bshadow is not None else None
        self._keep = [b, P, bs]
        _check(_lib.komega_init(self._h, _ptr(b), _ptr(bs), _ptr(P), _ptr(x)))
        self.x = x
        return x

    def update(self, q, r, qs=None, rs=None, wait=True):
        it = (Iter * self.nrhs)() if wait else None
        rc = _lib.komega_update(self._h, _ptr(q), _ptr(r), _ptr(qs), _ptr(rs), it)
        _check(rc, ok=(OK, CONVERGED, E_MAXITER, E_BREAKDOWN, E_SHIFT_BREAKDOWN, E_NONFINITE))
        return rc

    def iterate(self, op, n):
        _check(_lib.komega_iterate(self._h, op.handle, int(n)))

    def solve(self, op, poll=16):
        it = (Iter * self.nrhs)()
        rc = _lib.komega_solve(self._h, op.handle, int(poll), it)
        _check(rc, ok=(OK, CONVERGED, E_MAXITER, E_BREAKDOWN, E_SHIFT_BREAKDOWN, E_NONFINITE))
        return rc

    def state(self):
        it = (Iter * self.nrhs)()
        _check(_lib.komega_getstate(self._h, it))
        return [dict(status=i.status, iter=i.iter, seed=i.seed, nswitch=i.nswitch, maxres=i.maxres) for i in it]

    def residual(self):
        res = np.zeros((self.nrhs, self.nz))
        _check(_lib.komega_getresidual(self._h, res.ctypes.data_as(_pd)))
        return res

    def coef(self, rhs=0):
        cap = self.itermax
        a = np.zeros(cap, np.complex128)
        b = np.zeros(cap, np.complex128)
        zs = np.zeros(cap, np.complex128)
        seed = np.zeros(cap, np.int32)
        sw = np.zeros((cap, 2), np.complex128)
        pr = np.zeros((cap, max(self.nl, 1)), np.complex128)
        n = C.c_int32()
        f = lambda arr: arr.view(np.float64).ctypes.data_as(_pd)
        _check(_lib.komega_getcoef(self._h, rhs, f(a), f(b), f(zs), seed.ctypes.data_as(C.POINTER(C.c_int32)),
                                   f(sw), f(pr), C.byref(n)))
        k = n.value
        return dict(alpha=a[:k], beta=b[:k], zseed=zs[:k], seed=seed[:k], sw=sw[:k], Pr=pr[:k, : self.nl])

    def recalc(self, znew, rhs=0):
        """Projected solution at new shifts from the recorded history (no
        operator products).  Returns (y [nzn, nl] device, residual [nzn])."""
        znew = np.ascontiguousarray(np.asarray(znew, dtype=np.complex128).ravel())
        y = torch.empty((znew.size, self.nl), dtype=torch.complex128, device="cuda")
        res = np.zeros(znew.size)
        _check(_lib.komega_recalc(self._h, int(rhs), znew.size, znew.view(np.float64).ctypes.data_as(_pd), _ptr(y),
                                  res.ctypes.data_as(_pd)))
        return y, res

    def save_state(self):
        """Snapshot of the whole solver state (host bytes)."""
        n = C.c_int64()
        _check(_lib.komega_state_size(self._h, C.byref(n)))
        buf = np.empty(n.value, dtype=np.uint8)
        _check(_lib.komega_save_state(self._h, buf.ctypes.data_as(C.c_void_p), n.value))
        return buf

    def restore_state(self, buf, P=None, x=None):
        """Load a snapshot; P as for init; x is the output buffer (allocated
        when None; whole-x mode: must hold the saved solutions)."""
        if self.nl > 0:
            P = _dev_tensor(P, self.dtype, "cuda").reshape(self.nl, self.ndim)
        else:
            P = None
        shape, xdt = self._out_shape()
        if x is None:
            x = torch.zeros(shape, dtype=xdt, device="cuda")
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._keep = [P]
        _check(_lib.komega_restore_state(self._h, buf.ctypes.data_as(C.c_void_p), buf.size, _ptr(P), _ptr(x)))
        self.x = x
        return x

    def set_timing(self, mask):
        _check(_lib.komega_set_timing(self._h, int(mask)))

    def get_timing(self, cls, reset=True):
        ms = C.c_double()
        n = C.c_int64()
        _check(_lib.komega_get_timing(self._h, int(cls), C.byref(ms), C.byref(n), 1 if reset else 0))
        return ms.value, n.value

    def launch_info(self, cls, op=None):
        b = C.c_int64()
        t = C.c_int64()
        _check(_lib.komega_launch_info(self._h, op.handle if op is not None else None, int(cls), C.byref(b), C.byref(t)))
        return b.value, t.value

    def set_tuning(self, knob, value):
        _check(_lib.komega_set_tuning(self._h, int(knob), int(value)))

    def get_tuning(self, knob):
        v = C.c_int32()
        _check(_lib.komega_get_tuning(self._h, int(knob), C.byref(v)))
        return v.value

    def close(self):
        if self._h:
            _lib.komega_finalize(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass


def dotc_noalloc(a, x, out):
    """komega_dotc_noalloc: out[k] = a^H x_k into the caller's `out` (device
    complex128 [n]); the library allocates nothing (its partial sums live in
    a static device array shared by every call on the device)."""
    x = _resolved(x)
    n, M = x.shape
    a = _resolved(a)
    if a.dtype != torch.complex128 or x.dtype != torch.complex128 or out.dtype != torch.complex128:
        raise ValueError("a, x and out must be complex128")
    if out.numel() < n or not out.is_contiguous():
        raise ValueError("out must be a contiguous complex128 tensor of at least n elements")
    lda = 0 if a.dim() == 1 else a.stride(0)
    _check(_lib.komega_dotc_noalloc(_ptr(a), lda, _ptr(x), x.stride(0), M, n, _ptr(out), _stream()))
    return out


def dotc(a, x):
    """out[k] = a^H x_k (a: [M] or [n, M] device complex128; x: [n, M] device
    complex128, or complex64 with the products and sums formed in double)."""
    x = _resolved(x)
    n, M = x.shape
    a = _resolved(a)
    if a.dtype != torch.complex128:
        raise ValueError("a must be complex128")
    lda = 0 if a.dim() == 1 else a.stride(0)
    out = torch.empty(n, dtype=torch.complex128, device=x.device)
    if x.dtype == torch.complex64:
        _check(_lib.komega_dotc_c64(_ptr(a), lda, _ptr(x), x.stride(0), M, n, _ptr(out), _stream()))
    elif x.dtype == torch.complex128:
        _check(_lib.komega_dotc(_ptr(a), lda, _ptr(x), x.stride(0), M, n, _ptr(out), _stream()))
    else:
        raise ValueError("x must be complex128 or complex64")
    return out


def onsite_grad(g, w, x):
    """out[i] = sum_k g[k] w[k, i] conj(x[k, i]) (device complex128; g [n], w, x [n, M])."""
    g = _resolved(g.to(torch.complex128))
    w = _resolved(w)
    x = _resolved(x)
    n, M = x.shape
    if w.shape != x.shape or g.numel() != n:
        raise ValueError("g [n], w and x [n, M] expected")
    out = torch.empty(M, dtype=torch.complex128, device=x.device)
    _check(_lib.komega_onsite_grad(_ptr(g), _ptr(w), w.stride(0), _ptr(x), x.stride(0), M, n, _ptr(out), _stream()))
    return out


def stream_probe(src, dst, kind):
    """Bandwidth probe: kind 0 copies src to dst, kind 1 only reads src (dst
    receives per-work-group partial sums, stream_probe_groups() complex
    values).  Device tensors; enqueued on the current stream."""
    _check(_lib.komega_stream_probe(_ptr(src), _ptr(dst), src.numel() * src.element_size(), int(kind), _stream()))


def stream_probe_groups():
    return int(_lib.komega_stream_probe_groups())


def contour_moments(x, weights):
    """s[l, k] = sum_j weights[k, j] x[l, j] for kept solutions x [nrhs, nz, M]."""
    x = _resolved(x)
    nrhs, nz, M = x.shape
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.complex128))
    nk = w.shape[0]
    assert w.shape == (nk, nz)
    s = torch.empty((nrhs, nk, M), dtype=torch.complex128, device=x.device)
    _check(_lib.komega_contour_moments(_ptr(x), nz, M, nrhs, nk, w.view(np.float64).ctypes.data_as(_pd), _ptr(s),
                                       _stream()))
    return s


def greens_function(op, a, b, z, method="cocg", tol=1e-10, itermax=10000, switch=True, poll=16):
    """F_k = a^H (z_k I - H)^-1 b for every shift (projected mode, M_left = 1).
    Returns (F [nz] complex128 torch tensor on the GPU, final state)."""
    s = Solver(method, z, op.M, nl=1, tol=tol, itermax=itermax, switch=switch)
    a = _dev_tensor(a, torch.complex128, "cuda")
    y = s.init(b, P=torch.conj(a).resolve_conj().reshape(1, -1))
    s.solve(op, poll=poll)
    st = s.state()[0]
    out = y[0, :, 0].clone()
    s.close()
    return out, st
