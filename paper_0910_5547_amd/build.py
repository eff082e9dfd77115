"""Build the gfx950 HIP library ``libamrhydro.so`` in-tree with hipcc.

Flags: ``-O3 -ffp-contract=off`` (no FMA contraction: the FP64 path performs
exactly the operations written), packed FP32 instructions disabled, position
independent shared object exporting the C ABI of ``include/amr_hydro.h``.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libamrhydro.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("amr_kernels.hip", "amr_refine.hip", "amr_regrid.hip",
                                                       "amr_api.hip", "amr_cluster.cpp")]
ARCH = os.environ.get("AMR_OFFLOAD_ARCH", "gfx950")


def build(verbose: bool = False, extra=()) -> str:
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include"),
           "-o", LIB + ".tmp", *SOURCES, *extra]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
