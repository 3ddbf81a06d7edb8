"""Build the gfx950 HIP library liblbboil.so in-tree with hipcc.

Every HIP source is compiled with packed FP32 instructions disabled (the
compiler otherwise forms v_pk_* FP32 operations from scalar or float2 code),
and with multiply-add contraction limited to single expressions
(-ffp-contract=on): HIP's default lets the compiler fuse across statements
wherever the schedule allows, so two instantiations of one kernel (two tile
shapes) could round the same arithmetic differently.  With contraction tied
to the source, every tile shape gives bitwise the same state.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "csrc", "lbb_host.hip")]
DEPS = [os.path.join(HERE, "csrc", n) for n in os.listdir(os.path.join(HERE, "csrc"))]
TARGET = os.path.join(HERE, "liblbboil.so")
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=on",
    "-Wall", "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc] + FLAGS + ["-o", TARGET + ".tmp"] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(TARGET + ".tmp", TARGET)
    return TARGET


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
