"""ctypes front end of the C oracle (komega_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the library.  Everything here is
argument marshalling; the arithmetic lives in komega_oracle.c.
"""
import contextlib
import ctypes as C
import os

import numpy as np

from . import build as _build

CG_R, CG_C, COCG, BICG = 0, 1, 2, 3
METHODS = {"cg_r": CG_R, "cg_c": CG_C, "cocg": COCG, "bicg": BICG}

OK, CONVERGED = 0, 1
E_INVALID, E_BREAKDOWN, E_SHIFT_BREAKDOWN, E_MAXITER, E_NONFINITE = -1, -2, -3, -4, -7

STENCIL3D, CSR, HEISENBERG = 1, 2, 3

_pd = C.POINTER(C.c_double)
_pi32 = C.POINTER(C.c_int32)
_pi64 = C.POINTER(C.c_int64)
_pu32 = C.POINTER(C.c_uint32)


class _Op(C.Structure):
    _fields_ = [
        ("kind", C.c_int32), ("pad0", C.c_int32), ("M", C.c_int64),
        ("Lx", C.c_int32), ("Ly", C.c_int32), ("Lz", C.c_int32), ("pad1", C.c_int32),
        ("hop", C.c_double), ("eps", _pd),
        ("rowptr", _pi64), ("col", _pi32), ("val", _pd),
        ("L", C.c_int32), ("nup", C.c_int32), ("nb", C.c_int32), ("pad2", C.c_int32),
        ("bi", _pi32), ("bj", _pi32), ("J", _pd), ("states", _pu32),
    ]


class _Args(C.Structure):
    _fields_ = [
        ("method", C.c_int32), ("nz", C.c_int32), ("z", _pd),
        ("nl", C.c_int32), ("itermax", C.c_int32), ("P", _pd),
        ("tol", C.c_double), ("freeze_tol", C.c_double),
        ("seed_switch", C.c_int32), ("pad", C.c_int32),
        ("out", _pd), ("res", _pd),
        ("iters", C.c_int32), ("status", C.c_int32), ("seed", C.c_int32), ("nswitch", C.c_int32),
        ("hist_alpha", _pd), ("hist_beta", _pd), ("hist_zseed", _pd), ("hist_seed", _pi32),
    ]


_lib = None
_lib_path = None
_default_path = _build.LIB


@contextlib.contextmanager
def using(path):
    """Route every call through another build of the oracle (the mutation
    tests use this to run the pins against deliberately broken copies)."""
    global _default_path
    old = _default_path
    _default_path = path
    try:
        load(path)
        yield
    finally:
        _default_path = old


def load(path=None):
    """Load (building first if absent) the oracle shared library."""
    global _lib, _lib_path
    path = path or _default_path
    if _lib is not None and _lib_path == path:
        return _lib
    if not os.path.exists(path):
        _build.build(out=path)
    lib = C.CDLL(path)
    lib.orc_heis_basis.restype = C.c_int64
    lib.orc_heis_basis.argtypes = [C.c_int32, C.c_int32, _pu32]
    lib.orc_heis_index.restype = C.c_int64
    lib.orc_heis_index.argtypes = [_pu32, C.c_int64, C.c_uint32]
    lib.orc_apply.restype = C.c_int
    lib.orc_apply.argtypes = [C.POINTER(_Op), _pd, _pd]
    lib.orc_heis_szq.restype = None
    lib.orc_heis_szq.argtypes = [_pu32, C.c_int64, C.c_int32, _pd, _pd, _pd]
    lib.orc_solve.restype = C.c_int
    lib.orc_solve.argtypes = [C.POINTER(_Op), C.c_int64, _pd, _pd, C.POINTER(_Args)]
    lib.orc_threads.restype = C.c_int
    lib.orc_threads.argtypes = []
    lib.orc_lanczos.restype = C.c_int
    lib.orc_lanczos.argtypes = [C.POINTER(_Op), C.c_int64, _pd, C.c_int, _pd, _pd]
    _lib, _lib_path = lib, path
    return lib


def _ptr(a, t=_pd):
    return a.ctypes.data_as(t) if a is not None else None


def _c128(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


class Operator:
    """Oracle-side operator.  Keeps its arrays alive for the C struct."""

    def __init__(self, kind, M, **arrays):
        self.kind, self.M = kind, int(M)
        self._keep = arrays
        self.st = _Op()
        self.st.kind = kind
        self.st.M = self.M

    @staticmethod
    def stencil3d(Lx, Ly, Lz, eps, hop=1.0):
        eps = np.ascontiguousarray(eps, dtype=np.float64)
        if min(Lx, Ly, Lz) < 3 or eps.size != Lx * Ly * Lz:
            raise ValueError("stencil3d needs edges >= 3 and eps of size Lx*Ly*Lz")
        op = Operator(STENCIL3D, eps.size, eps=eps)
        op.st.Lx, op.st.Ly, op.st.Lz, op.st.hop = Lx, Ly, Lz, float(hop)
        op.st.eps = _ptr(eps)
        return op

    @staticmethod
    def csr(rowptr, col, val):
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        val = _c128(val)
        op = Operator(CSR, rowptr.size - 1, rowptr=rowptr, col=col, val=val)
        op.st.rowptr, op.st.col, op.st.val = _ptr(rowptr, _pi64), _ptr(col, _pi32), _ptr(val)
        return op

    @staticmethod
    def heisenberg(L, nup, bonds, J):
        bonds = np.asarray(bonds, dtype=np.int32).reshape(-1, 2)
        J = np.ascontiguousarray(np.broadcast_to(np.asarray(J, dtype=np.float64), (len(bonds),)))
        states = basis(L, nup)
        bi = np.ascontiguousarray(bonds[:, 0])
        bj = np.ascontiguousarray(bonds[:, 1])
        op = Operator(HEISENBERG, states.size, states=states, bi=bi, bj=bj, J=J)
        op.st.L, op.st.nup, op.st.nb = L, nup, len(bonds)
        op.st.bi, op.st.bj, op.st.J = _ptr(bi, _pi32), _ptr(bj, _pi32), _ptr(J)
        op.st.states = _ptr(states, _pu32)
        op.states = states
        return op

    def apply(self, v):
        v = _c128(v)
        out = np.empty_like(v)
        rc = load().orc_apply(C.byref(self.st), _ptr(v.view(np.float64)), _ptr(out.view(np.float64)))
        if rc != 0:
            raise RuntimeError("oracle operator application failed")
        return out


def threads():
    """Threads the oracle's row loops run on."""
    return int(load().orc_threads())


def basis(L, nup):
    lib = load()
    n = lib.orc_heis_basis(L, nup, None)
    if n < 0:
        raise ValueError("bad (L, nup)")
    out = np.empty(n, dtype=np.uint32)
    lib.orc_heis_basis(L, nup, _ptr(out, _pu32))
    return out


def index(states, s):
    states = np.ascontiguousarray(states, dtype=np.uint32)
    return int(load().orc_heis_index(_ptr(states, _pu32), states.size, int(s)))


def szq(states, L, w, v):
    states = np.ascontiguousarray(states, dtype=np.uint32)
    w, v = _c128(w), _c128(v)
    out = np.empty_like(v)
    load().orc_heis_szq(_ptr(states, _pu32), states.size, L, _ptr(w.view(np.float64)),
                        _ptr(v.view(np.float64)), _ptr(out.view(np.float64)))
    return out


class Result:
    def __init__(self, **kw):
        self.__dict__.update(kw)


def solve(op, b, z, method="cocg", P=None, tol=1e-10, itermax=10000, freeze_tol=None,
          seed_switch=True, bshadow=None, history=False, lib_path=None):
    """Shifted solve.  P=None keeps the whole x (returns x[nz, M]); otherwise
    returns y[nz, nl] = P x.  freeze_tol=None means 1e-3*tol; 0 disables."""
    lib = load(lib_path)
    b = _c128(b)
    z = _c128(z).ravel()
    M = b.size
    nz = z.size
    a = _Args()
    a.method = METHODS[method] if isinstance(method, str) else int(method)
    a.nz = nz
    a.z = _ptr(z.view(np.float64))
    if P is not None:
        P = _c128(P).reshape(-1, M)
        nl = P.shape[0]
        out = np.zeros((nz, nl), dtype=np.complex128)
        a.P = _ptr(P.view(np.float64))
    else:
        nl = 0
        out = np.zeros((nz, M), dtype=np.complex128)
        a.P = None
    a.nl = nl
    a.itermax = int(itermax)
    a.tol = float(tol)
    a.freeze_tol = 1e-3 * tol if freeze_tol is None else float(freeze_tol)
    a.seed_switch = 1 if seed_switch else 0
    res = np.zeros(nz, dtype=np.float64)
    a.out = _ptr(out.view(np.float64))
    a.res = _ptr(res)
    h = {}
    if history:
        h["alpha"] = np.zeros(max(itermax, 1), dtype=np.complex128)
        h["beta"] = np.zeros(max(itermax, 1), dtype=np.complex128)
        h["zseed"] = np.zeros(max(itermax, 1), dtype=np.complex128)
        h["seed"] = np.zeros(max(itermax, 1), dtype=np.int32)
        a.hist_alpha = _ptr(h["alpha"].view(np.float64))
        a.hist_beta = _ptr(h["beta"].view(np.float64))
        a.hist_zseed = _ptr(h["zseed"].view(np.float64))
        a.hist_seed = _ptr(h["seed"], _pi32)
    bs = _c128(bshadow) if bshadow is not None else None
    lib.orc_solve(C.byref(op.st), M, _ptr(b.view(np.float64)),
                  _ptr(bs.view(np.float64)) if bs is not None else None, C.byref(a))
    if history:
        for k in h:
            h[k] = h[k][: a.iters]
    return Result(out=out, res=res, iters=a.iters, status=a.status, seed=a.seed,
                  nswitch=a.nswitch, history=h if history else None)


def lanczos(op, b, nsteps):
    b = _c128(b)
    a = np.zeros(nsteps)
    bb = np.zeros(max(nsteps - 1, 1))
    made = load().orc_lanczos(C.byref(op.st), b.size, _ptr(b.view(np.float64)), nsteps,
                              _ptr(a), _ptr(bb))
    return a[:made], bb[: max(made - 1, 0)]
