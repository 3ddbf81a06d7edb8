"""Build the FP64 CPU oracle (test infrastructure only) into oracle/liboracle.so.

Plain C, gcc, no fast-math and no floating-point contraction, so every
operation rounds exactly as written.  OpenMP is used only over independent
rows; no reduction is parallelised, so results do not depend on the thread
count.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["lbb_oracle.c", "lbb_oracle_adjoint.c", "lbb_oracle3d.c"]
TARGET = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter",
           "-o", TARGET + ".tmp"] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(TARGET + ".tmp", TARGET)
    return TARGET


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
