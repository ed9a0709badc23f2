"""The bandwidth probe (a diagnostic kernel pair) moves the data it claims:
the copy is exact and the read pass's per-group partial sums add up to the
sum of the elements' real parts, including a ragged tail."""
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def K():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2001_08707_amd import komega
    return komega


@pytest.mark.parametrize("n", [1, 777, 4096 * 256 * 4 + 13, 3 * 10 ** 6])
def test_probe_copy_and_read(K, n):
    g = torch.Generator(device="cuda").manual_seed(n)
    src = torch.randn(n, dtype=torch.complex128, device="cuda", generator=g)
    dst = torch.zeros_like(src)
    K.stream_probe(src, dst, 0)
    assert torch.equal(dst, src)
    part = torch.zeros(K.stream_probe_groups(), dtype=torch.complex128, device="cuda")
    K.stream_probe(src, part, 1)
    tot = float(part.real.sum())
    ref = float(src.real.sum())
    assert abs(tot - ref) <= 1e-12 * float(src.real.abs().sum())
    with pytest.raises(K.KomegaError):
        K.stream_probe(src[:0], dst, 0)
