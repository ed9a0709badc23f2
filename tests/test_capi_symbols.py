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


C_CALLER = r"""
#include <stdio.h>
#include <string.h>
#include "komega_hip.h"
int main(void) {
  komega_params p;
  komega_solver* s = NULL;
  double z[2] = {0.0, 0.1};
  memset(&p, 0, sizeof p);
  p.method = KOMEGA_COCG;
  p.nz = 0;              /* invalid: rejected on the host, before any device call */
  p.ndim = 8;
  p.nrhs = 1;
  if (komega_create(&s, &p, z) != KOMEGA_E_INVALID || s != NULL) return 1;
  printf("%s|%s\n", komega_strerror(KOMEGA_CONVERGED), komega_last_error());
  return 0;
}
"""


@pytest.mark.skipif(not os.path.exists(LIB), reason="HIP library not built")
def test_plain_c_caller(tmp_path):
    # the header is plain C: a C99 program compiles against it, links the
    # library and gets a host-side error without touching a GPU
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    src = tmp_path / "caller.c"
    src.write_text(C_CALLER)
    exe = tmp_path / "caller"
    libdir = os.path.dirname(LIB)
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", os.path.join(ROOT, "include"),
                    str(src), "-o", str(exe), "-L", libdir, "-lkomega_hip", "-Wl,-rpath," + libdir],
                   check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stderr
    first, last = out.stdout.strip().split("|", 1)
    assert first == "converged" and last
