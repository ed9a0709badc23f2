"""Independent FP64 CPU oracle of the shifted Krylov solver.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check in __graft_entry__ and
the CPU-baseline leg of bench.py may import this package.  The GPU library
never imports it, and it never imports the GPU library.

  komega_oracle.c : the shifted CG / COCG / BiCG solver, its operators, the
                    brute-force spin basis and Lanczos (plain C, FP64)
  oracle.py       : ctypes front end
  dense.py        : the plain definitions for small matrices (dense H,
                    a^H (zI - H)^-1 b by LU, spectra by eigh)
"""
