"""Plain dense definitions for small problems (numpy, FP64).

TEST INFRASTRUCTURE ONLY.

  G(z) = (z I - H)^-1                         (Sec. 1, Eq. EQ-GREEN-FN)
  F_k  = a^H G(z_k) b = a^H x^(k)             (Sec. 1, Eqs. EQ-GREEN-ELEM,
                                               EQ-SOLUTION-VECTOR)
  G(z) = sum_j y_j y_j^H / (z - lambda_j)     (Sec. 1, spectral decomposition)

The dense Hamiltonians are built here from their definitions, independently
of the C oracle's operator code, so the two can be checked against each other.
"""
import numpy as np


def stencil3d_dense(Lx, Ly, Lz, eps, hop=1.0):
    """Anderson cube: H_ii = eps_i, H_ij = -hop for the 6 periodic neighbours,
    site i = x + Lx*(y + Ly*z).  Edges must be >= 3 so the neighbours are
    distinct."""
    M = Lx * Ly * Lz
    H = np.zeros((M, M))
    for z in range(Lz):
        for y in range(Ly):
            for x in range(Lx):
                i = x + Lx * (y + Ly * z)
                H[i, i] = eps[i]
                for (dx, dy, dz) in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    j = (x + dx) % Lx + Lx * (((y + dy) % Ly) + Ly * ((z + dz) % Lz))
                    H[i, j] += -hop
    return H


def spin_basis(L, nup):
    """Ascending list of the L-bit integers with nup set bits."""
    return np.array([s for s in range(1 << L) if bin(s).count("1") == nup], dtype=np.int64)


def heisenberg_dense(L, nup, bonds, J):
    """H = sum_b J_b S_i . S_j (spin 1/2, site j = bit j, up = 1) on the
    sector with nup up spins, built from the matrix elements
    <s|S^z_i S^z_j|s> = +-1/4 and <s'|(S^+_i S^-_j + S^-_i S^+_j)/2|s> = 1/2."""
    states = spin_basis(L, nup)
    pos = {int(s): n for n, s in enumerate(states)}
    J = np.broadcast_to(np.asarray(J, dtype=np.float64), (len(bonds),))
    M = len(states)
    H = np.zeros((M, M))
    for n, s in enumerate(states):
        s = int(s)
        for (i, j), Jb in zip(bonds, J):
            si, sj = (s >> i) & 1, (s >> j) & 1
            if si == sj:
                H[n, n] += 0.25 * Jb
            else:
                H[n, n] -= 0.25 * Jb
                t = s ^ ((1 << i) | (1 << j))
                H[pos[t], n] += 0.5 * Jb
    return H


def csr_to_dense(rowptr, col, val):
    M = len(rowptr) - 1
    H = np.zeros((M, M), dtype=np.complex128)
    for i in range(M):
        for p in range(rowptr[i], rowptr[i + 1]):
            H[i, col[p]] += val[p]
    return H


def greens_solve(H, b, z):
    """x^(k) = (z_k I - H)^-1 b for every k, by LU; returns x[nz, M]."""
    H = np.asarray(H)
    M = H.shape[0]
    I = np.eye(M)
    return np.array([np.linalg.solve(zk * I - H, b) for zk in np.atleast_1d(z)])


def greens_element(H, a, b, z):
    """F_k = a^H (z_k I - H)^-1 b by LU."""
    x = greens_solve(H, b, z)
    return x @ np.conj(a)


def greens_element_eigh(H, a, b, z):
    """F_k = sum_j (a^H y_j)(y_j^H b) / (z_k - lambda_j) from one eigh."""
    lam, Y = np.linalg.eigh(H)
    wa = Y.conj().T @ a
    wb = Y.conj().T @ b
    return np.array([np.sum(np.conj(wa) * wb / (zk - lam)) for zk in np.atleast_1d(z)])


def continued_fraction(a, bet, nb2, z):
    """||b||^2 [(z - T_n)^-1]_{11} for the Lanczos tridiagonal T_n
    (diagonal a[0..n-1], off-diagonal bet[0..n-2]), evaluated bottom-up."""
    z = np.atleast_1d(np.asarray(z, dtype=np.complex128))
    n = len(a)
    g = np.zeros_like(z)
    for j in range(n - 1, -1, -1):
        tail = bet[j] ** 2 * g if j < n - 1 else 0.0
        g = 1.0 / (z - a[j] - tail)
    return nb2 * g


def heisenberg_bond_operators(L, nup, bonds):
    """O_b = S_i . S_j (dense, sector nup) for every bond: H = sum_b J_b O_b."""
    return [heisenberg_dense(L, nup, [bd], [1.0]) for bd in bonds]


def onsite_gradient(H, a, b, z):
    """dF_k/deps_i for F_k = a^H (z_k - H)^-1 b and on-site energies eps_i on
    the diagonal of H: a^H G e_i e_i^T G b = (a^H G)_i (G b)_i (dG = G dH G).
    Returns (F [nz], dF [nz, M])."""
    H = np.asarray(H)
    M = H.shape[0]
    F, dF = [], []
    for zk in np.atleast_1d(z):
        G = np.linalg.inv(zk * np.eye(M) - H)
        x = G @ b
        aG = np.conj(a) @ G
        F.append(aG @ b)
        dF.append(aG * x)
    return np.array(F), np.array(dF)


def heisenberg_coupling_gradient(L, nup, bonds, J, a, b, z):
    """dF_k/dJ_b for F_k = a^H (z_k - H)^-1 b with H = sum_b J_b O_b:
    a^H G O_b G b with G = (z_k - H)^-1 (dG = G dH G).  Returns (F [nz],
    dF [nz, nb])."""
    Ob = heisenberg_bond_operators(L, nup, bonds)
    H = sum(Jb * O for Jb, O in zip(J, Ob))
    M = H.shape[0]
    F, dF = [], []
    for zk in np.atleast_1d(z):
        G = np.linalg.inv(zk * np.eye(M) - H)
        x = G @ b
        wH = np.conj(a) @ G
        F.append(np.conj(a) @ x)
        dF.append([wH @ (O @ x) for O in Ob])
    return np.array(F), np.array(dF)


def contour_moments(X, z, gamma, nk):
    """Trapezoid moments of the contour rule (Sec. 4.1): on the circle
    z_j = gamma + rho exp(2 pi i (j+1/2)/N), j < N,
        s_k = (1/2 pi i) oint (z - gamma)^k G(z) phi dz
            ~ (1/N) sum_j (z_j - gamma)^(k+1) G(z_j) phi,
    since dz = i (z - gamma) d(theta).  X[j] holds G(z_j) phi (or any linear
    image of it, such as its projections); returns s[k] for k < nk."""
    X = np.asarray(X)
    z = np.asarray(z)
    N = z.size
    return np.array([sum((z[j] - gamma) ** (k + 1) * X[j] for j in range(N)) / N for k in range(nk)])
