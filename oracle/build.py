"""Build the C oracle into oracle/_build/libkomega_oracle.so.

TEST INFRASTRUCTURE ONLY (see komega_oracle.c).  Plain gcc; no HIP headers.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "komega_oracle.c")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libkomega_oracle.so")


def build(extra_defines=(), out=None, verbose=False):
    """Compile the oracle.  `extra_defines` are -D flags (used only by the
    mutation tests, which plant mistakes into private copies of the oracle)."""
    out = out or LIB
    os.makedirs(os.path.dirname(out), exist_ok=True)
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unused-variable"]
    cmd += ["-D" + d for d in extra_defines]
    cmd += ["-o", out, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
