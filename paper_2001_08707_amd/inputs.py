"""Seeded synthetic inputs for the shifted Krylov solver.

This module only draws random numbers and lays out problem descriptions
(lattice sizes, disorder, bond lists, shift grids, start vectors).  It holds
none of the solver's arithmetic, so both the GPU library's tests and the CPU
oracle can take their inputs from it.

Every generator uses numpy.random.default_rng(seed) (PCG64) in FP64, with the
draw order written in its docstring.  Shift grids on the real axis use
numpy.linspace (end points included).
"""
import math

import numpy as np


class Workload(dict):
    """A plain dict with attribute access."""

    __getattr__ = dict.__getitem__


def unit(v):
    return v / np.linalg.norm(v)


# --------------------------------------------------------------------------
# 3D Anderson tight-binding cube: H_ii = eps_i ~ U[-W/2, W/2], H_ij = -t for
# the 6 periodic neighbours, site i = x + L*(y + L*z).
def anderson(L, W, seed_eps, seed_vec, z, t=1.0, complex_vec=False, nrhs=1, rhs_seeds=None):
    """eps = rng(seed_eps).uniform(-W/2, W/2, L^3).
    Real start vector: unit(rng(seed_vec).standard_normal(M)).
    Complex start vectors (one generator per right-hand side, seeds rhs_seeds):
    g = rng(s); unit(g.standard_normal(M) + 1j * g.standard_normal(M))."""
    M = L ** 3
    eps = np.random.default_rng(seed_eps).uniform(-W / 2, W / 2, M)
    if complex_vec:
        seeds = rhs_seeds if rhs_seeds is not None else [seed_vec + i for i in range(nrhs)]
        bs = []
        for s in seeds:
            g = np.random.default_rng(s)
            re = g.standard_normal(M)
            im = g.standard_normal(M)
            bs.append(unit(re + 1j * im))
        b = np.array(bs)
    else:
        b = unit(np.random.default_rng(seed_vec).standard_normal(M)).astype(np.complex128)[None, :]
    return Workload(kind="stencil3d", L=L, M=M, W=W, t=t, eps=eps, b=b,
                    z=np.asarray(z, dtype=np.complex128))


def real_axis(lo, hi, n, delta):
    """z_k = omega_k + i delta with omega_k = linspace(lo, hi, n)."""
    return np.linspace(lo, hi, n) + 1j * delta


def contour(gamma, rho, n):
    """Contour nodes z_j = gamma + rho exp(2 pi i (j + 1/2) / n) (Sec. 4.1)."""
    j = np.arange(n)
    return gamma + rho * np.exp(2j * np.pi * (j + 0.5) / n)


# --------------------------------------------------------------------------
# Spin-1/2 chains.
def ring_bonds(L, d=1):
    """Bonds (j, j+d mod L) for j = 0..L-1."""
    return np.array([(j, (j + d) % L) for j in range(L)], dtype=np.int32)


def sector_dim(L, nup):
    return math.comb(L, nup)


def phases(L, q_quarter):
    """w_j = exp(i q j) for q = q_quarter * pi/2, taken from the exact table
    {1, i, -1, -i} so that no cosine rounding enters."""
    table = np.array([1.0, 1j, -1.0, -1j])
    return table[(np.arange(L) * q_quarter) % 4].astype(np.complex128)


def heisenberg_chain(L, seed_vec, z, J=1.0, q_quarter=2):
    """Uniform periodic chain, S^z = 0 sector.  v = unit(rng(seed_vec)
    .standard_normal(M)); the start vector is b = S^z(q) v with q = q_quarter*pi/2,
    applied by whoever consumes the workload (phases w_j given)."""
    M = sector_dim(L, L // 2)
    v = unit(np.random.default_rng(seed_vec).standard_normal(M))
    bonds = ring_bonds(L)
    return Workload(kind="heisenberg", L=L, nup=L // 2, M=M, bonds=bonds,
                    J=np.full(len(bonds), float(J)), v=v, w=phases(L, q_quarter),
                    z=np.asarray(z, dtype=np.complex128))


def j1j2_chain(L, seed, z, q_quarter=1, seed_target=5):
    """J1-J2 ring with per-bond couplings, r = rng(seed):
    J1 = 1 + 0.1 r.standard_normal(L) on (j, j+1); J2 = 0.3 + 0.05
    r.standard_normal(L) on (j, j+2); then v = unit(r.standard_normal(M)).
    Perturbed couplings for targets: theta + 0.05 rng(seed_target)
    .standard_normal(2L)."""
    r = np.random.default_rng(seed)
    J1 = 1.0 + 0.1 * r.standard_normal(L)
    J2 = 0.3 + 0.05 * r.standard_normal(L)
    M = sector_dim(L, L // 2)
    v = unit(r.standard_normal(M))
    bonds = np.concatenate([ring_bonds(L, 1), ring_bonds(L, 2)])
    theta = np.concatenate([J1, J2])
    theta_star = theta + 0.05 * np.random.default_rng(seed_target).standard_normal(2 * L)
    return Workload(kind="heisenberg", L=L, nup=L // 2, M=M, bonds=bonds, J=theta,
                    J_target=theta_star, v=v, w=phases(L, q_quarter),
                    z=np.asarray(z, dtype=np.complex128))


# --------------------------------------------------------------------------
# The five benchmark configurations at full size.
def config1():
    """3D Anderson 16^3 (M=4096), W=4, eps seed 0, a = b unit real (seed 1),
    64 shifts on [-8, 8] + 0.05i, tolerance 1e-10."""
    return anderson(16, 4.0, 0, 1, real_axis(-8, 8, 64, 0.05))


def config2(L=24):
    """Heisenberg ring L=24, J=1, S^z=0 (M=2,704,156), b = a = S^z(pi) v with
    v unit random (seed 2), 1024 shifts on [-1, 8] + 0.02i, projected."""
    return heisenberg_chain(L, 2, real_axis(-1, 8, 1024, 0.02), q_quarter=2)


def config3(L=64, nrhs=16, nz=32):
    """3D Anderson 64^3 (M=262,144), W=16.5, eps seed 3, 16 complex Gaussian
    right-hand sides (seeds 10..25), 32 nodes on |z| = 0.5, whole x kept."""
    return anderson(L, 16.5, 3, 10, contour(0.0, 0.5, nz), complex_vec=True,
                    nrhs=nrhs, rhs_seeds=list(range(10, 10 + nrhs)))


def config4(L=20):
    """J1-J2 ring L=20 (M=184,756), per-bond couplings (seed 4), b = a =
    S^z(pi/2) v, 256 shifts on [-2, 6] + 0.05i."""
    return j1j2_chain(L, 4, real_axis(-2, 6, 256, 0.05), q_quarter=1, seed_target=5)


def config5(n=64):
    """64 Anderson instances: r = rng(5), edges = r.integers(8, 41, n),
    W = r.uniform(2, 20, n); instance i: eps = rng(1000+i).uniform(-W/2, W/2,
    edge^3), a = b = unit(rng(2000+i).standard_normal(edge^3)); 256 shifts on
    [-10, 10] + 0.02i."""
    r = np.random.default_rng(5)
    edges = r.integers(8, 41, n)
    Ws = r.uniform(2, 20, n)
    z = real_axis(-10, 10, 256, 0.02)
    inst = [anderson(int(e), float(W), 1000 + i, 2000 + i, z) for i, (e, W) in enumerate(zip(edges, Ws))]
    return Workload(kind="batch", instances=inst, z=z)
