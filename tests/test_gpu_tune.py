"""Launch-configuration knobs and the autotuner: no knob changes a result bit,
and the autotuner leaves the solver freshly initialised with its choice."""
import json

import numpy as np
import pytest

from paper_2001_08707_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def K():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2001_08707_amd import komega
    return komega


@pytest.mark.parametrize("method,x32", [("cocg", False), ("cocg", True), ("cg_r", False)])
def test_shift_knobs_do_not_change_results(K, method, x32):
    w = I.anderson(7, 5.0, 3, 4, I.real_axis(-7, 7, 21, 0.05))   # 21 shifts: ragged shift blocks
    op = K.Operator.stencil3d(7, 7, 7, w.eps)
    b = torch.as_tensor(w.b[0], device="cuda")
    z = w.z
    if method == "cg_r":   # real vectors, real shifts below the spectrum
        b = b.real.contiguous()
        z = np.linspace(-16.0, -10.0, 21) + 0j
    # the per-step update (steps = 1) and the blocked update (16 and 32
    # steps): for each, every launch shape gives the same bits
    for steps in (1, 16, 32):
        ref = None
        for sb in (1, 2, 4, 8, 16):
            for nt in (0, 1):
                for order in (0, 1):
                    s = K.Solver(method, z, op.M, tol=1e-11, x32=x32)
                    s.set_tuning(K.T_SHIFT_STEPS, steps)
                    s.set_tuning(K.T_SHIFT_BLOCK, sb)
                    s.set_tuning(K.T_SHIFT_NT, nt)
                    s.set_tuning(K.T_SHIFT_ORDER, order)
                    assert (s.get_tuning(K.T_SHIFT_STEPS), s.get_tuning(K.T_SHIFT_BLOCK), s.get_tuning(K.T_SHIFT_NT),
                            s.get_tuning(K.T_SHIFT_ORDER)) == (steps, sb, nt, order)
                    x = s.init(b)
                    s.solve(op)
                    if ref is None:
                        ref = x.clone()
                    assert torch.equal(x, ref), (steps, sb, nt, order)
                    s.close()
    s = K.Solver("cocg", w.z, op.M)
    with pytest.raises(K.KomegaError):
        s.set_tuning(K.T_SHIFT_BLOCK, 3)
    with pytest.raises(K.KomegaError):
        s.set_tuning(K.T_SHIFT_NT, 2)
    with pytest.raises(K.KomegaError):
        s.set_tuning(K.T_SHIFT_STEPS, 0)
    with pytest.raises(K.KomegaError):
        s.set_tuning(K.T_SHIFT_STEPS, 33)
    with pytest.raises(K.KomegaError):
        s.set_tuning(99, 1)


def test_autotune_batched_and_cache(K, tmp_path):
    from paper_2001_08707_amd import tune as T
    r = np.random.default_rng(1)
    L = np.array([[6, 6, 6], [5, 4, 7], [3, 3, 3]], dtype=np.int32)
    eps = [r.uniform(-3, 3, int(np.prod(l))) for l in L]
    op = K.Operator.stencil3d_batch(L, eps)
    b = torch.as_tensor(r.standard_normal(op.M) + 0j, device="cuda")
    z = I.real_axis(-6, 6, 24, 0.1)
    ref = K.Solver("cocg", z, rows=op.rows, tol=1e-11)
    ref.set_tuning(K.T_SHIFT_STEPS, 1)   # graph replay applies every step at once
    ref.init(b)
    ref.solve(op)
    s = K.Solver("cocg", z, rows=op.rows, tol=1e-11, graph=True)
    s.init(b)
    path = str(tmp_path / "tune.json")
    chosen, timings = T.autotune(s, op, b, path=path)
    assert set(chosen) == {"shift_steps", "shift_block", "shift_nt", "shift_order"}
    assert len(timings) == len(T.SHIFT_CANDIDATES) and all(t > 0 for t in timings.values())
    assert s.state()[0]["iter"] == 0           # freshly initialised
    s.solve(op, poll=10)
    assert torch.equal(s.x, ref.x)
    table = json.load(open(path))
    assert len(table) == 1
    # a second solver of the same bucket takes the cached choice without timing
    s2 = K.Solver("cocg", z, rows=op.rows, tol=1e-11)
    s2.init(b)
    chosen2, timings2 = T.autotune(s2, op, b, path=path)
    assert chosen2 == chosen and timings2 == {}
    for h in (ref, s, s2):
        h.close()


def test_autotune_heisenberg_variant(K, tmp_path):
    from paper_2001_08707_amd import tune as T
    w = I.heisenberg_chain(16, 2, I.real_axis(-1, 5, 32, 0.05))
    op = K.Operator.heisenberg(16, 8, w.bonds, w.J)
    b = op.szq(w.w, torch.as_tensor(w.v, device="cuda"))
    P = torch.conj(b).resolve_conj()[None, :]
    s = K.Solver("cocg", w.z, op.M, nl=1, tol=1e-10)
    s.init(b, P=P)
    chosen, timings = T.autotune(s, op, b, P=P, path=str(tmp_path / "t.json"))
    assert chosen["heis_variant"] in T.HEIS_VARIANTS and chosen["spmv_blocks"] in T.SPMV_BLOCKS
    assert len(timings) == len(T.HEIS_VARIANTS) * len(T.SPMV_BLOCKS)
    s.solve(op)
    F = s.x[0, :, 0].clone()
    ref = K.Solver("cocg", w.z, op.M, nl=1, tol=1e-10)
    op.set_variant(1)
    y = ref.init(b, P=P)
    ref.solve(op)
    # the two product kernels sum the bonds in different orders: rounding-level agreement
    assert float(((F - y[0, :, 0]).abs() / y[0, :, 0].abs()).max()) < 1e-10
