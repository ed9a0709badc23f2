"""The bench's fixed parts, checked without a GPU: it refuses more than one
GPU (the solver has no multi-GPU path), and its algorithmic bytes per launch
are the per-row figures the method must move."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    for args, env in ((["--gpus", "2"], {}), ([], {"WORLD_SIZE": "4"})):
        p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, capture_output=True,
                           text=True, env={**os.environ, **env}, timeout=120)
        assert p.returncode == 2
        assert "exactly one GPU" in p.stderr
        assert p.stdout == ""


def test_algorithmic_bytes_per_launch():
    # Heisenberg ring L=24, projected: product = state 4 B + r 16 B + q 16 B
    # per row; seed update = r_n, q, r_{n-1} read + r_{n+1} written (64 B)
    # + the projection row (16 B) per row.
    h = bench.make_workload("heis24")
    M = 2704156
    assert h["M"] == M and h["nl"] == 1 and h["nrhs"] == 1
    assert bench.algorithmic_bytes(h, 0) == 36 * M
    assert bench.algorithmic_bytes(h, 1) == 80 * M
    # Anderson 64^3, 16 right-hand sides x 32 shifts, whole x: the shift update
    # reads and writes x and p (64 B per shift.row) and reads r_{n+1} once.
    a = bench.make_workload("anderson64")
    Ma = 64 ** 3
    assert a["M"] == Ma and a["nrhs"] == 16 and a["nz"] == 32
    assert bench.algorithmic_bytes(a, 2) == 16 * 32 * Ma * 64 + 16 * Ma * 16
    assert bench.algorithmic_bytes(a, 0) == 8 * Ma + 16 * Ma * 32
    assert bench.algorithmic_bytes({**a, "x32": True}, 2) == 16 * 32 * Ma * 32 + 16 * Ma * 16


def test_iteration_algorithmic_bytes():
    # Table 2's count per iteration: Heisenberg L=24 projected = 68 B per row
    # (state 4 + r_n, r_{n-1}, projection row read and r_{n+1} written, 16 B
    # each); the 64^3 contour workload = 8 + 16 x (64 + 32 x 64) B per row
    # (the on-site energies read once for the 16 right-hand sides).
    h = bench.make_workload("heis24")
    assert bench.iteration_algorithmic_bytes(h) == 68 * 2704156
    assert bench.design_bytes_per_row(h) == 116
    a = bench.make_workload("anderson64")
    assert bench.iteration_algorithmic_bytes(a) == (8 + 16 * (64 + 32 * 64)) * 64 ** 3
    assert abs(bench.iteration_algorithmic_bytes(a) - 8.86e9) < 0.01e9


def test_host_cpu_description():
    h = bench.host_cpu()
    assert h["nproc"] >= 1 and h["logical_cpus"] >= h["nproc"]


def test_stencil_csr_workload():
    # The CSR copy of the periodic stencil that the CSR workload runs applies
    # like the oracle's stencil operator (a 5^3 cube: every row wraps in some
    # direction at the faces), and its product moves the CSR rows once (row
    # pointer 8 B, 7 x (column 4 B + value 8 B)) plus r and q per right-hand side.
    import numpy as np
    from oracle import oracle as O
    L = 5
    rng = np.random.default_rng(11)
    eps = rng.uniform(-2.0, 2.0, L ** 3)
    v = rng.standard_normal(L ** 3) + 1j * rng.standard_normal(L ** 3)
    rowptr, col, val = bench.stencil_csr(L, eps)
    assert rowptr[-1] == col.size == val.size == 7 * L ** 3
    assert np.all(np.diff(col.reshape(-1, 7), axis=1) > 0)
    q_csr = O.Operator.csr(rowptr, col, val).apply(v)
    q_st = O.Operator.stencil3d(L, L, L, eps).apply(v)
    assert np.max(np.abs(q_csr - q_st)) <= 1e-13 * np.max(np.abs(q_st))
    c = bench.make_workload("anderson64csr")
    Ma = 64 ** 3
    assert c["kind"] == "csr" and c["nrhs"] == 16 and c["nz"] == 32
    assert bench.algorithmic_bytes(c, 0) == (8 + 7 * 12) * Ma + 16 * Ma * 32
