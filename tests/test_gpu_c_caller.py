"""A plain C99 program drives the library through the C ABI alone (no Python
binding): a stencil operator, a projected COCG solve with the built-in loop,
and the same solve by reverse communication with the caller's own product
(komega_op_apply then komega_update, Algorithm 1).  Python only writes the
inputs and checks the outputs against the oracle."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from paper_2001_08707_amd import inputs as I

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_2001_08707_amd", "_lib")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

PROGRAM = r"""
#define __HIP_PLATFORM_AMD__ 1
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>
#include "komega_hip.h"

#define CK(x) do { komega_status rc_ = (x); if (rc_ < 0) { \
  fprintf(stderr, "%s: %s (%s)\n", #x, komega_strerror(rc_), komega_last_error()); return 2; } } while (0)
#define HK(x) do { if ((x) != hipSuccess) { fprintf(stderr, "%s failed\n", #x); return 3; } } while (0)

static int rd(FILE* f, void* p, size_t n) { return fread(p, 1, n, f) == n; }

int main(int argc, char** argv) {
  if (argc != 3) return 1;
  FILE* f = fopen(argv[1], "rb");
  int32_t hdr[2];
  if (!f || !rd(f, hdr, sizeof hdr)) return 1;
  const int L = hdr[0], nz = hdr[1];
  const size_t M = (size_t)L * L * L;
  double* eps = malloc(M * sizeof(double));
  double* b = malloc(2 * M * sizeof(double));
  double* Pc = malloc(2 * M * sizeof(double));
  double* z = malloc(2 * (size_t)nz * sizeof(double));
  double* y = malloc(4 * (size_t)nz * sizeof(double));
  if (!eps || !b || !Pc || !z || !y) return 1;
  if (!rd(f, eps, M * 8) || !rd(f, b, 2 * M * 8) || !rd(f, z, 2 * (size_t)nz * 8)) return 1;
  fclose(f);
  for (size_t i = 0; i < M; ++i) { Pc[2 * i] = b[2 * i]; Pc[2 * i + 1] = -b[2 * i + 1]; }  /* conj(b) */

  komega_op* op = NULL;
  CK(komega_op_stencil3d(&op, L, L, L, 1.0, eps));
  void *db, *dP, *dy1, *dy2, *dr, *dq;
  HK(hipMalloc(&db, 16 * M));
  HK(hipMalloc(&dP, 16 * M));
  HK(hipMalloc(&dr, 16 * M));
  HK(hipMalloc(&dq, 16 * M));
  HK(hipMalloc(&dy1, 16 * (size_t)nz));
  HK(hipMalloc(&dy2, 16 * (size_t)nz));
  HK(hipMemcpy(db, b, 16 * M, hipMemcpyHostToDevice));
  HK(hipMemcpy(dP, Pc, 16 * M, hipMemcpyHostToDevice));

  komega_params p = {0};
  p.method = KOMEGA_COCG; p.nz = nz; p.ndim = (int64_t)M; p.nl = 1; p.nrhs = 1;
  p.itermax = 100000; p.tol = 1e-10; p.freeze_tol = -1.0; p.stream = NULL;

  /* built-in loop */
  komega_solver* s1 = NULL;
  komega_iter st1;
  CK(komega_create(&s1, &p, z));
  CK(komega_init(s1, db, NULL, dP, dy1));
  CK(komega_solve(s1, op, 16, &st1));

  /* reverse communication: the caller applies H to r, the library updates */
  komega_solver* s2 = NULL;
  komega_iter st2;
  CK(komega_create(&s2, &p, z));
  CK(komega_init(s2, db, NULL, dP, dy2));
  HK(hipMemcpy(dr, db, 16 * M, hipMemcpyDeviceToDevice));
  komega_status rc = KOMEGA_OK;
  for (int n = 0; n < 100000 && rc == KOMEGA_OK; ++n) {
    CK(komega_op_apply(op, dr, dq, 1, 1, NULL));
    rc = komega_update(s2, dq, dr, NULL, NULL, &st2);
    CK(rc);
  }
  HK(hipMemcpy(y, dy1, 16 * (size_t)nz, hipMemcpyDeviceToHost));
  HK(hipMemcpy(y + 2 * nz, dy2, 16 * (size_t)nz, hipMemcpyDeviceToHost));

  FILE* o = fopen(argv[2], "wb");
  int32_t res[4] = {st1.status, st1.iter, st2.status, st2.iter};
  if (!o || fwrite(res, sizeof res, 1, o) != 1 || fwrite(y, 16, 2 * (size_t)nz, o) != 2 * (size_t)nz) return 1;
  fclose(o);
  CK(komega_finalize(s1));
  CK(komega_finalize(s2));
  CK(komega_op_destroy(op));
  hipFree(db); hipFree(dP); hipFree(dr); hipFree(dq); hipFree(dy1); hipFree(dy2);
  free(eps); free(b); free(Pc); free(z); free(y);
  return 0;
}
"""


def test_c_program_solves_through_the_abi(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    if not os.path.exists(os.path.join(LIBDIR, "libkomega_hip.so")):
        pytest.skip("HIP library not built")
    src = tmp_path / "caller.c"
    src.write_text(PROGRAM)
    exe = tmp_path / "caller"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROCM, "include"), str(src), "-o", str(exe),
                    "-L", LIBDIR, "-lkomega_hip", "-Wl,-rpath," + LIBDIR,
                    "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib")],
                   check=True, capture_output=True, text=True)
    w = I.anderson(8, 5.0, 21, 22, I.real_axis(-7, 7, 24, 0.05), complex_vec=True, rhs_seeds=[31])
    b = w.b[0].astype(np.complex128)
    inp = tmp_path / "in.bin"
    with open(inp, "wb") as f:
        np.array([8, w.z.size], dtype=np.int32).tofile(f)
        np.ascontiguousarray(w.eps, dtype=np.float64).tofile(f)
        b.tofile(f)
        np.ascontiguousarray(w.z, dtype=np.complex128).tofile(f)
    out = tmp_path / "out.bin"
    p = subprocess.run([str(exe), str(inp), str(out)], capture_output=True, text=True, timeout=120)
    assert p.returncode == 0, p.stderr
    raw = out.read_bytes()
    st = np.frombuffer(raw[:16], dtype=np.int32)
    y = np.frombuffer(raw[16:], dtype=np.complex128).reshape(2, -1)
    assert st[0] == 1 and st[2] == 1          # KOMEGA_CONVERGED for both
    ref = O.solve(O.Operator.stencil3d(8, 8, 8, w.eps), b, w.z, P=b.conj()[None, :], tol=1e-10)
    F = ref.out[:, 0]
    print(f"C caller: built-in {st[1]} iterations, reverse communication {st[3]}, oracle {ref.iters}")
    assert np.max(np.abs(y[0] - F) / np.abs(F)) < 1e-10
    assert np.max(np.abs(y[1] - F) / np.abs(F)) < 1e-10
    assert abs(int(st[1]) - ref.iters) <= max(3, 0.05 * ref.iters)
