"""The stored oracle values parse, come from the current oracle source, and
have the shapes the full-size parity tests read (CPU only)."""
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _load():
    import importlib.util
    spec = importlib.util.spec_from_file_location("fullsize", os.path.join(HERE, "test_gpu_fullsize.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.fixture(scope="module")
def F():
    return _load()


def _have(name):
    return os.path.exists(os.path.join(HERE, "golden", name))


@pytest.mark.skipif(not _have("config5_oracle.txt"), reason="not generated yet")
def test_config5_golden(F):
    Fo, it = F._config5_golden()
    assert sorted(Fo) == sorted(it) and len(Fo) == 4
    for r in Fo:
        assert Fo[r].shape == (256,) and np.all(np.isfinite(Fo[r])) and np.all(Fo[r].imag < 0)
        assert it[r] > 0


@pytest.mark.skipif(not _have("config3_oracle.txt"), reason="not generated yet")
def test_config3_golden(F):
    from paper_2001_08707_amd import inputs as I
    meta, vals = F.golden("config3_oracle.txt")
    assert len(vals["F"]) == 16 * 32 and len(vals["MU"]) == 16 * 10 * 16
    it = [m.split()[1:] for m in meta if m.startswith("iters")][0]
    assert len(it) == 16 and all(int(t) > 0 for t in it)
    # Herglotz: Im phi^H G(z) phi = -Im z sum |y^H phi|^2 / |z - lam|^2
    z = I.contour(0.0, 0.5, 32)
    for (l, j), v in vals["F"].items():
        assert np.sign(v.imag) == -np.sign(z[j].imag)


@pytest.mark.skipif(not _have("config2_oracle.txt"), reason="not generated yet")
def test_config2_golden(F):
    meta, vals = F.golden("config2_oracle.txt")
    Fo = np.array([vals["F"][(k,)] for k in range(1024)])
    assert np.all(Fo.imag < 0)          # Herglotz: Im a^H G(w + i d) a < 0 for d > 0
    assert int(F.meta_field(meta, "iters")) > 0
