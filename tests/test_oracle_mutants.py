"""The pins must catch plausible mistakes in the oracle.

Each case plants one mistake in a private copy of komega_oracle.c (text
substitution, on the CPU, in a temporary directory), builds it, and runs a
quick battery of the pins from test_oracle_pins against the broken build.  At
least one pin must fail.  The committed oracle is never modified.
"""
import os

import numpy as np
import pytest

from oracle import build as B
from oracle import dense as D
from oracle import oracle as O
from paper_2001_08707_amd import inputs as I

SRC = open(B.SRC).read()

MUTANTS = {
    "drop_three_term_gamma": ("r_new[i] = c_r * r[i] + alpha * q[i] - gamma * r_old[i];",
                              "r_new[i] = c_r * r[i] + alpha * q[i];"),
    "alpha_denominator_sign": ("cplx rAr = zs * rho - t;", "cplx rAr = zs * rho + t;"),
    "start_ratio_not_zero": ("cplx ba = 0.0;", "cplx ba = 1.0;"),
    "sigma_sign": ("cplx sigma = a->z[k] - zs;", "cplx sigma = zs - a->z[k];"),
    "beta_k_not_squared": ("cplx bk = ratio * ratio * beta;", "cplx bk = ratio * beta;"),
    "u_update_old_pi": ("*uk = Pr[l] / pn + bk * *uk;", "*uk = Pr[l] / pi[k] + bk * *uk;"),
    "p_update_old_pi": ("pk[i] = r_new[i] / pn + bk * pk[i];", "pk[i] = r_new[i] / pi[k] + bk * pk[i];"),
    "x_update_alpha_seed": ("xk[i] += ak * pk[i];", "xk[i] += alpha * pk[i];"),
    "cocg_uses_conjugate": ("return method == ORC_COCG ? dot_bilinear(n, x, y) : dot_sesq(n, x, y);",
                            "return dot_sesq(n, x, y);"),
    "switch_keeps_rho": ("rho_new /= c1 * c1;", ";"),
    "switch_keeps_alpha": ("alpha *= c0 / c1;", ";"),
    "switch_keeps_old_residual": ("{ r_new[i] /= c1; r[i] /= c0; }", "{ r_new[i] /= c1; }"),
    "switch_keeps_old_pi": ("pi_old[k] /= c0;", ";"),
    "residual_ignores_pi": ("a->res[k] = sqrt(nu) / (cabs(pi[k]) * bnorm);", "a->res[k] = sqrt(nu) / bnorm;"),
    "bicg_shadow_not_conjugated": ("cplx c_rs = conj(c_r), ca = conj(alpha), cg = conj(gamma);",
                                   "cplx c_rs = c_r, ca = alpha, cg = gamma;"),
    "heisenberg_diag_sign": ("diag -= 0.25 * op->J[b];", "diag += 0.25 * op->J[b];"),
    "heisenberg_flip_weight": ("off += 0.5 * op->J[b] * v[j];", "off += op->J[b] * v[j];"),
    "stencil_hop_sign": ("out[i] = op->eps[i] * v[i] - op->hop * nb;", "out[i] = op->eps[i] * v[i] + op->hop * nb;"),
    "stencil_wrap_axis": ("int64_t zm = (z + Lz - 1) % Lz, zp = (z + 1) % Lz;",
                          "int64_t zm = (z + Lz - 1) % Lz, zp = (z + 2) % Lz;"),
    "basis_order_reversed": ("if (v < s) lo = mid + 1; else hi = mid - 1;", "if (v > s) lo = mid + 1; else hi = mid - 1;"),
}


def _csr(H):
    H = np.asarray(H, dtype=np.complex128)
    rows, cols = np.nonzero(H)
    rowptr = np.cumsum(np.r_[0, np.bincount(rows, minlength=H.shape[0])]).astype(np.int64)
    return O.Operator.csr(rowptr, cols.astype(np.int32), H[rows, cols])


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - b) / np.maximum(np.abs(b), 1e-300)))


def _battery():
    """Quick pins; returns the names of those that fail."""
    failed = []

    def check(name, fn):
        try:
            ok = fn()
        except Exception:
            ok = False
        if not ok:
            failed.append(name)

    w = I.anderson(5, 4.0, 0, 1, I.real_axis(-8, 8, 12, 0.1))
    sop = O.Operator.stencil3d(5, 5, 5, w.eps)
    Hs = D.stencil3d_dense(5, 5, 5, w.eps)
    b = w.b[0]

    def anderson_dense():
        r = O.solve(sop, b, w.z, P=b.conj()[None, :], tol=1e-11)
        return r.status == O.CONVERGED and _rel(r.out[:, 0], D.greens_element(Hs, b, b, w.z)) < 1e-9
    check("anderson_dense", anderson_dense)

    def full_x_dense():
        bc = b + 0.3j * np.roll(b, 1)
        r = O.solve(sop, bc, w.z, tol=1e-12)
        X = D.greens_solve(Hs, bc, w.z)
        return r.status == O.CONVERGED and np.max(np.linalg.norm(r.out - X, axis=1) / np.linalg.norm(X, axis=1)) < 1e-9
    check("full_x_dense", full_x_dense)

    def residual_true():
        r = O.solve(sop, b, w.z, tol=0.0, itermax=15)
        R = np.array([b - (zk * np.eye(b.size) - Hs) @ x for zk, x in zip(w.z, r.out)])
        return _rel(np.linalg.norm(R, axis=1), r.res) < 1e-8
    check("residual_true", residual_true)

    def heis_dense():
        bonds = I.ring_bonds(8)
        hop = O.Operator.heisenberg(8, 4, bonds, 1.0)
        H = D.heisenberg_dense(8, 4, bonds, 1.0)
        v = np.random.default_rng(0).standard_normal(hop.M)
        return np.max(np.abs(hop.apply(v) - H @ v)) < 1e-12
    check("heis_dense", heis_dense)

    def lanczos_cf():
        hw = I.heisenberg_chain(10, 2, I.real_axis(-1, 4, 16, 0.05))
        hop = O.Operator.heisenberg(10, 5, hw.bonds, hw.J)
        hb = O.szq(hop.states, 10, hw.w, hw.v)
        a_, b_ = O.lanczos(hop, hb, 12)
        cf = D.continued_fraction(a_, b_, np.vdot(hb, hb).real, hw.z)
        r = O.solve(hop, hb, hw.z, P=hb.conj()[None, :], tol=0.0, itermax=12)
        return _rel(r.out[:, 0], cf) < 1e-10
    check("lanczos_cf", lanczos_cf)

    def complex_offdiag():
        rng = np.random.default_rng(11)
        A = rng.standard_normal((20, 20))
        H = (A + A.T) / 4
        a = rng.standard_normal(20) + 1j * rng.standard_normal(20)
        bb = rng.standard_normal(20) + 1j * rng.standard_normal(20)
        z = I.contour(0.3, 1.5, 8)
        r = O.solve(_csr(H), bb, z, P=a.conj()[None, :], tol=1e-13)
        return _rel(r.out[:, 0], D.greens_element(H, a, bb, z)) < 1e-9
    check("complex_offdiag", complex_offdiag)

    def hermitian_bicg():
        rng = np.random.default_rng(12)
        A = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
        H = (A + A.conj().T) / 4
        bb = rng.standard_normal(16) + 1j * rng.standard_normal(16)
        z = I.real_axis(-3, 3, 6, 0.2)
        r = O.solve(_csr(H), bb, z, method="bicg", P=bb.conj()[None, :], tol=1e-13)
        return _rel(r.out[:, 0], D.greens_element(H, bb, bb, z)) < 1e-9
    check("hermitian_bicg", hermitian_bicg)

    def two_by_two():
        zs = 0.3 + 0.7j
        z = np.array([zs, 2.0 + 0.5j])
        r = O.solve(_csr([[0, 1], [1, 0]]), [1.0, 0.0], z, P=np.array([[1.0, 0.0]]), tol=1e-14,
                    itermax=5, seed_switch=False)
        return r.iters == 2 and _rel(r.out[:, 0], z / (z ** 2 - 1)) < 1e-13
    check("two_by_two", two_by_two)

    return failed


@pytest.fixture(scope="module")
def battery_on_good_oracle():
    return _battery()


def test_battery_passes_on_the_committed_oracle(battery_on_good_oracle):
    assert battery_on_good_oracle == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name, battery_on_good_oracle):
    old, new = MUTANTS[name]
    assert SRC.count(old) == 1, "mutation target text not found exactly once"
    src = tmp_path / "komega_oracle.c"
    src.write_text(SRC.replace(old, new))
    lib = str(tmp_path / "libmutant.so")
    import subprocess
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    "-w", "-o", lib, str(src), "-lm"], check=True)
    with O.using(lib):
        failed = _battery()
    assert failed, f"mutant {name} passed every pin"
