"""The blocked whole-x update against the per-step update.

With KOMEGA_T_SHIFT_STEPS = s > 1 the library composes up to s steps of
x^k += alpha^k p^k, p^k = r_{n+1}/pi^k_{n+1} + beta^k p^k (Sec. 2.2.2, Eqs.
EQ-SHIFTEDCG-x/p) into one linear map per shift and applies it with one pass
over x^k, p^k.  The seed recurrence never reads x or p, so residuals,
iteration counts and seed switches are identical bit for bit; x^k differs
from the per-step update only by the rounding of the two association orders,
bounded here normwise by 1e-12 (FP64) relative to x^k.  Uneven iterate()
batches check that a partial block is applied whenever a call returns."""
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


def nrel(a, b):
    a = a.to(torch.complex128) if a.is_complex() else a
    b = b.to(torch.complex128) if b.is_complex() else b
    return (torch.linalg.vector_norm(a - b, dim=-1) / torch.linalg.vector_norm(b, dim=-1)).max().item()


def _problem(method):
    w = I.anderson(9, 5.0, 11, 12, I.real_axis(-7, 7, 21, 0.05), complex_vec=method != "cg_r",
                   rhs_seeds=[13])
    z = np.linspace(-16.0, -10.0, 21) + 0j if method.startswith("cg") else w.z
    b = w.b[0].real.copy() if method == "cg_r" else w.b[0]
    return w, z, b


@pytest.mark.parametrize("method,x32", [("cocg", False), ("bicg", False), ("cg_c", False), ("cg_r", False),
                                        ("cocg", True)])
@pytest.mark.parametrize("steps", [32, 16, 5, 2])
def test_blocked_equals_per_step(K, method, x32, steps):
    w, z, b = _problem(method)
    op = K.Operator.stencil3d(9, 9, 9, w.eps)
    bd = torch.as_tensor(b, device="cuda")
    out = {}
    for s_ in (1, steps):
        s = K.Solver(method, z, op.M, tol=1e-11, x32=x32)
        s.set_tuning(K.T_SHIFT_STEPS, s_)
        x = s.init(bd)
        snaps = []
        for n in (7, 16, 3, 40, 1):   # partial blocks at every return
            s.iterate(op, n)
            snaps.append((s.state()[0], s.residual().copy(), x.clone()))
        assert s.solve(op) == K.CONVERGED
        snaps.append((s.state()[0], s.residual().copy(), x.clone()))
        out[s_] = snaps
        s.close()
    tol = 1e-5 if x32 else 1e-12
    for (st1, r1, x1), (stb, rb, xb) in zip(out[1], out[steps]):
        assert st1 == stb
        assert np.array_equal(r1, rb)
        assert nrel(xb, x1) < tol, (method, steps, st1["iter"])


def test_blocked_batched_systems(K):
    # uneven systems in one launch, blocked vs per-step; systems stop at
    # different iterations, inside a block
    r = np.random.default_rng(4)
    L = np.array([[6, 6, 6], [5, 4, 7], [3, 3, 3], [8, 8, 8]], dtype=np.int32)
    eps = [r.uniform(-3, 3, int(np.prod(l))) for l in L]
    op = K.Operator.stencil3d_batch(L, eps)
    b = torch.as_tensor(r.standard_normal(op.M) + 1j * r.standard_normal(op.M), device="cuda")
    z = I.real_axis(-6, 6, 24, 0.1)
    sol = {}
    for steps in (1, 16):
        s = K.Solver("cocg", z, rows=op.rows, tol=1e-11)
        s.set_tuning(K.T_SHIFT_STEPS, steps)
        s.init(b)
        assert s.solve(op, poll=10) == K.CONVERGED
        sol[steps] = (s.state(), s.x.clone())
        s.close()
    assert [st["iter"] for st in sol[1][0]] == [st["iter"] for st in sol[16][0]]
    assert len({st["iter"] for st in sol[16][0]}) > 1     # the systems stop at different steps
    s1 = K.Solver("cocg", z, rows=op.rows)
    for k in range(len(L)):
        assert nrel(s1.system_x(k, sol[16][1]), s1.system_x(k, sol[1][1])) < 1e-12
    s1.close()


def test_knob_changes_between_calls(K):
    w, z, b = _problem("cocg")
    op = K.Operator.stencil3d(9, 9, 9, w.eps)
    s = K.Solver("cocg", z, op.M, tol=1e-11)
    s.init(torch.as_tensor(b, device="cuda"))
    s.iterate(op, 5)
    # every iterate() applies its partial block before it returns
    s.set_tuning(K.T_SHIFT_STEPS, 8)
    s.iterate(op, 9)
    s.set_tuning(K.T_SHIFT_STEPS, 1)
    s.iterate(op, 3)
    assert s.get_tuning(K.T_SHIFT_STEPS) == 1
    s.close()


@pytest.mark.parametrize("poll", [5, 16, 40])
def test_solve_keeps_blocks_across_polls(K, poll):
    # komega_solve checks convergence every `poll` steps but applies the
    # whole-x block only when it is full or when the solve returns: one
    # update launch per 32 steps, whatever the poll interval, and the same
    # x^k as the per-step update to rounding
    w, z, b = _problem("cocg")
    op = K.Operator.stencil3d(9, 9, 9, w.eps)
    bd = torch.as_tensor(b, device="cuda")
    out = {}
    for steps in (1, 32):
        s = K.Solver("cocg", z, op.M, tol=1e-11)
        s.set_tuning(K.T_SHIFT_STEPS, steps)
        x = s.init(bd)
        s.set_timing(1 << K.K_SHIFT)
        assert s.solve(op, poll=poll) == K.CONVERGED
        _, launches = s.get_timing(K.K_SHIFT)
        out[steps] = (s.state()[0], s.residual().copy(), x.clone(), launches)
        s.close()
    (st1, r1, x1, n1), (st32, r32, x32, n32) = out[1], out[32]
    assert st1 == st32
    assert np.array_equal(r1, r32)
    assert nrel(x32, x1) < 1e-12
    # the last poll may run up to poll - 1 steps past convergence (launches
    # that a stopped system skips), so up to one more block than the steps
    # taken
    it = st32["iter"]
    assert -(-it // 32) <= n32 <= -(-(it + poll) // 32), (it, n32)
    assert n1 >= it
