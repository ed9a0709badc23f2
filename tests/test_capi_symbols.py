"""The C interface library loads and exports every symbol the header declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "komega_hip.h")
LIB = os.path.join(ROOT, "paper_2001_08707_amd", "_lib", "libkomega_hip.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(komega_[a-z_0-9]+)\s*\(", src))
    names.discard("komega_apply_fn")
    return sorted(names)


def test_header_declares_the_paper_flow():
    names = declared()
    for n in ("komega_create", "komega_init", "komega_update", "komega_getresidual", "komega_getcoef",
              "komega_finalize", "komega_solve", "komega_iterate"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="HIP library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="HIP library not built")
def test_strerror_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.komega_strerror.restype = ctypes.c_char_p
    assert lib.komega_strerror(1) == b"converged"
    assert b"breakdown" in lib.komega_strerror(-3)


def test_binding_signatures_cover_the_header():
    # the Python binding declares a signature for every exported function
    src = open(os.path.join(ROOT, "paper_2001_08707_amd", "komega.py")).read()
    for n in declared():
        assert f'"{n}"' in src, n
