"""Contour-integral (Sakurai-Sugiura) eigenvalues inside a circle, driven by
the shifted solver (Sec. 4.1).

P_Gamma = (1/2 pi i) \\oint (zI - H)^-1 dz projects onto the eigenvectors
inside the contour; the moments s_{k,l} = (1/2 pi i) \\oint (z - gamma)^k
(zI - H)^-1 phi_l dz span them.  On the circle z = gamma + rho e^{i theta}
the trapezoid rule with N nodes z_j = gamma + rho e^{2 pi i (j+1/2)/N} gives
s_{k,l} = (1/N) sum_j (z_j - gamma)^{k+1} G(z_j) phi_l.

GPU: one shifted solve per random vector phi_l keeping x at the N nodes (all
right-hand sides batched), and the moment kernel.  Host: the small dense
steps of the paper's sample code -- SVD of S, Rayleigh-Ritz with
H~ = U~^H H U~ (the products H U~ on the GPU), eigenvalues of H~ -- via
LAPACK (numpy), as in the paper.
"""
import numpy as np
import torch

from . import komega as K


def nodes(gamma, rho, n):
    j = np.arange(n)
    return gamma + rho * np.exp(2j * np.pi * (j + 0.5) / n)


def weights(gamma, rho, n, nk):
    z = nodes(gamma, rho, n)
    return np.array([(z - gamma) ** (k + 1) / n for k in range(nk)])


def ss_eigenvalues(op, gamma, rho, n_nodes=100, n_moments=10, n_vectors=2, seed=0, tol=1e-12,
                   sv_cut=1e-3, itermax=20000):
    """Eigenvalues of H (operator `op`) inside |z - gamma| < rho.  Singular
    values of S below sv_cut * max are discarded (the paper discards those
    below 1e-3).  Returns (eigenvalues ascending, singular values)."""
    M = op.M
    rng = np.random.default_rng(seed)
    phi = rng.standard_normal((n_vectors, M)) + 1j * rng.standard_normal((n_vectors, M))
    phi /= np.linalg.norm(phi, axis=1, keepdims=True)
    z = nodes(gamma, rho, n_nodes)
    s = K.Solver("cocg", z, M, nl=0, nrhs=n_vectors, tol=tol, itermax=itermax)
    X = s.init(torch.as_tensor(phi, device="cuda"))
    rc = s.solve(op)
    s.close()
    if rc != K.CONVERGED:
        raise RuntimeError("contour solves did not converge")
    S = K.contour_moments(X, weights(gamma, rho, n_nodes, n_moments))       # [nl, nk, M]
    S = S.reshape(n_vectors * n_moments, M).T.contiguous()                  # columns s_{k,l}
    Sh = S.cpu().numpy()
    U, sv, _ = np.linalg.svd(Sh, full_matrices=False)
    keep = sv > sv_cut * sv[0]
    Ut = np.ascontiguousarray(U[:, keep])
    HU = op.apply(torch.as_tensor(Ut.T.copy(), device="cuda")).cpu().numpy().T
    Ht = Ut.conj().T @ HU
    lam = np.linalg.eigvalsh((Ht + Ht.conj().T) / 2)
    inside = np.abs(lam - gamma) < rho
    return np.sort(lam[inside]), sv
