"""Differentiable spectra with respect to Hamiltonian parameters.

F_k(theta) = a^H G(z_k) b,  G(z) = (z I - H(theta))^-1  (Kawamura et al., Sec. 1
Eq. EQ-GREEN-ELEM).  H is linear in its parameters and dG = G dH G, so

    dF_k / dtheta = a^H G(z_k) (dH/dtheta) G(z_k) b = w_k^H (dH/dtheta) x_k,
    x_k = G(z_k) b,   w_k = G(z_k)^H a = G(conj z_k) a   (H Hermitian).

Two parameter families:
  HeisenbergSpectrum  bond couplings J_b of H = sum_b J_b S_{i_b} . S_{j_b}
                      (Sec. 4.2, Eq. eq:heisenberg with a coupling per bond):
                      dH/dJ_b = S_i . S_j, contracted by the library's bond kernel;
  AndersonSpectrum    on-site energies eps_i of the 3D Anderson stencil:
                      dH/deps_i = e_i e_i^T, so dF_k/deps_i = conj(w_k[i]) x_k[i],
                      contracted over the shifts by komega_onsite_grad.

Forward: one shifted solve keeping the whole x over the augmented shift set
{z_k} U {conj z_k}; with a = b the same Krylov sequence yields both x_k and
w_k, so the adjoint costs shift updates but no extra operator products (for
a != b a second solve with right-hand side a over {conj z_k}).  Backward: the
library's bond contraction (komega_op_heisenberg_bond_grad), combined with the
upstream gradient as grad_J = Re sum_k g_k conj(dF_k/dJ) (PyTorch's complex
convention).  All solver and contraction arithmetic runs in the HIP library.
"""
import numpy as np
import torch

from . import komega as K


class HeisenbergSpectrum:
    """F(J) for fixed (L, nup, bonds, a, b, z); call with a float64 tensor J."""

    def __init__(self, L, nup, bonds, a, b, z, tol=1e-12, itermax=20000, method="cocg"):
        self.L, self.nup = int(L), int(nup)
        self.bonds = np.asarray(bonds, dtype=np.int32).reshape(-1, 2)
        self.z = np.asarray(z, dtype=np.complex128).ravel()
        self.a = torch.as_tensor(a, dtype=torch.complex128, device="cuda").contiguous()
        self.b = torch.as_tensor(b, dtype=torch.complex128, device="cuda").contiguous()
        self.same = bool(torch.equal(self.a, self.b))
        self.tol, self.itermax, self.method = tol, itermax, method
        self.last = {}

    def _op(self, J):
        return K.Operator.heisenberg(self.L, self.nup, self.bonds, J.detach().cpu().numpy())

    def _solve(self, op, rhs, shifts):
        s = K.Solver(self.method, shifts, op.M, nl=0, tol=self.tol, itermax=self.itermax)
        X = s.init(rhs)
        rc = s.solve(op)
        st = s.state()[0]
        s.close()
        if rc != K.CONVERGED:
            raise RuntimeError(f"shifted solve did not converge: {st}")
        return X[0], st

    def forward_only(self, J):
        """F(J) keeping x over the N_z shifts only (no adjoint vectors)."""
        op = self._op(J)
        x, st = self._solve(op, self.b, self.z)
        self.last = {"fwd_iters": st["iter"]}
        return K.dotc(self.a, x)

    def __call__(self, J):
        return _SpectrumFn.apply(J, self)


def _augmented_solve(op, a, b, z, same, tol, itermax, method):
    """x_k = G(z_k) b and w_k = G(conj z_k) a, whole vectors kept: one Krylov
    sequence over {z} U {conj z} when a = b, else two solves."""
    nz = z.size

    def solve(rhs, shifts):
        s = K.Solver(method, shifts, op.M, nl=0, tol=tol, itermax=itermax)
        X = s.init(rhs)
        rc = s.solve(op)
        st = s.state()[0]
        s.close()
        if rc != K.CONVERGED:
            raise RuntimeError(f"shifted solve did not converge: {st}")
        return X[0], st

    if same:
        X, st = solve(b, np.concatenate([z, z.conj()]))
        return X[:nz], X[nz:], {"iters": st["iter"]}
    x, st1 = solve(b, z)
    w, st2 = solve(a, z.conj())
    return x, w, {"iters": st1["iter"], "adjoint_iters": st2["iter"]}


class AndersonSpectrum:
    """F(eps) for the periodic Lx x Ly x Lz Anderson cube (hopping -hop) with
    fixed (a, b, z); call with a float64 tensor eps of Lx*Ly*Lz on-site energies."""

    def __init__(self, shape, a, b, z, hop=1.0, tol=1e-12, itermax=20000, method="cocg"):
        self.shape = tuple(int(v) for v in shape)
        self.M = int(np.prod(self.shape))
        self.hop = float(hop)
        self.z = np.asarray(z, dtype=np.complex128).ravel()
        self.a = torch.as_tensor(a, dtype=torch.complex128, device="cuda").contiguous()
        self.b = torch.as_tensor(b, dtype=torch.complex128, device="cuda").contiguous()
        self.same = bool(torch.equal(self.a, self.b))
        self.tol, self.itermax, self.method = tol, itermax, method
        self.last = {}

    def _op(self, eps):
        return K.Operator.stencil3d(*self.shape, eps.detach().cpu().numpy(), hop=self.hop)

    def __call__(self, eps):
        return _OnsiteFn.apply(eps, self)


class _OnsiteFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eps, model):
        op = model._op(eps)
        x, w, model.last = _augmented_solve(op, model.a, model.b, model.z, model.same, model.tol,
                                            model.itermax, model.method)
        op.close()
        ctx.x, ctx.w = x, w
        ctx.eps_device = eps.device
        return K.dotc(model.a, x)

    @staticmethod
    def backward(ctx, gF):
        # grad_eps_i = Re sum_k g_k conj(dF_k/deps_i) = Re sum_k g_k w_k[i] conj(x_k[i])
        out = K.onsite_grad(gF.to(device=ctx.x.device), ctx.w, ctx.x)
        return out.real.to(device=ctx.eps_device, dtype=torch.float64), None


class _SpectrumFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, J, model):
        op = model._op(J)
        nz = model.z.size
        if model.same:
            X, st = model._solve(op, model.b, np.concatenate([model.z, model.z.conj()]))
            x, w = X[:nz], X[nz:]
            model.last = {"iters": st["iter"]}
        else:
            x, st1 = model._solve(op, model.b, model.z)
            w, st2 = model._solve(op, model.a, model.z.conj())
            model.last = {"iters": st1["iter"], "adjoint_iters": st2["iter"]}
        F = K.dotc(model.a, x)
        ctx.op, ctx.x, ctx.w = op, x, w
        ctx.J_device = J.device
        return F

    @staticmethod
    def backward(ctx, gF):
        dF = ctx.op.bond_grad(ctx.w, ctx.x)          # [nz, nb] = dF_k / dJ_b
        gJ = (gF.to(dF.dtype)[:, None] * dF.conj()).real.sum(0)
        # the saved operator and vectors live until the graph is released
        # (backward may run more than once with retain_graph)
        return gJ.to(device=ctx.J_device, dtype=torch.float64), None
