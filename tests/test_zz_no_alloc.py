"""The allocation-free projection (komega_dotc_noalloc) against komega_dotc.

Both go through the C interface with the same kernels; the only difference
is where the partial sums live (a static device array instead of
stream-ordered scratch), so the results must be identical bit for bit.  Two
calls in a row, the second smaller, check that the shared array's previous
contents never leak into a result."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def K():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2001_08707_amd import komega
    return komega


def _case(seed, n, M, shared_a):
    g = np.random.default_rng(seed)
    x = g.standard_normal((n, M)) + 1j * g.standard_normal((n, M))
    a = g.standard_normal(M if shared_a else (n, M)) + 1j * g.standard_normal(M if shared_a else (n, M))
    return a, x


@pytest.mark.parametrize("shared_a", [True, False])
def test_noalloc_matches_dotc_twice(K, shared_a):
    # first call: 300 vectors of 70,001 rows (64 work-groups, ragged tail);
    # second call: 7 vectors of 1,000 rows (4 work-groups) into the same array
    for seed, n, M in ((1, 300, 70001), (2, 7, 1000)):
        print(f"noalloc: seed {seed} n {n} M {M} shared_a {shared_a}", flush=True)
        a, x = _case(seed, n, M, shared_a)
        ad = torch.as_tensor(a, device="cuda")
        xd = torch.as_tensor(x, device="cuda")
        ref = K.dotc(ad, xd)
        out = torch.full((n,), complex("nan"), dtype=torch.complex128, device="cuda")
        K.dotc_noalloc(ad, xd, out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (seed, n, M)
        want = (np.conj(a) * x).sum(axis=1) if not shared_a else x @ np.conj(a)
        err = np.max(np.abs(out.cpu().numpy() - want) / np.linalg.norm(x, axis=1) / np.linalg.norm(a, axis=-1))
        assert err < 1e-14, err


def test_noalloc_limits(K):
    M = 512
    x = torch.zeros((K.NOALLOC_MAX_VECTORS + 1, M), dtype=torch.complex128, device="cuda")
    a = torch.zeros(M, dtype=torch.complex128, device="cuda")
    out = torch.zeros(K.NOALLOC_MAX_VECTORS + 1, dtype=torch.complex128, device="cuda")
    with pytest.raises(K.KomegaError, match="static scratch limit"):
        K.dotc_noalloc(a, x, out)
    # at the limit it runs, in a single launch pair
    y = K.dotc_noalloc(a, x[: K.NOALLOC_MAX_VECTORS], out)
    torch.cuda.synchronize()
    assert torch.count_nonzero(y[: K.NOALLOC_MAX_VECTORS]).item() == 0
