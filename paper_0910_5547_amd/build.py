"""Build the gfx950 HIP library ``libamrhydro.so`` in-tree with hipcc.

Flags: ``-O3 -ffp-contract=off`` (no FMA contraction: the FP64 path performs
exactly the operations written), packed FP32 instructions disabled, position
independent shared object exporting the C ABI of ``include/amr_hydro.h``.

Each source compiles to its own object in parallel (the stage kernel's
instantiations are spread over several translation units, ``amr_stage_*.hip``),
then one hipcc line links them.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libamrhydro.so")
OBJDIR = os.path.join(HERE, "_build")
SOURCES = [os.path.join(HERE, "csrc", f) for f in (
    "amr_stage_hydro_f32.hip", "amr_stage_hydro_f64.hip", "amr_stage_mhd.hip", "amr_stage_glm.hip",
    "amr_kernels.hip", "amr_refine.hip", "amr_regrid.hip", "amr_api.hip", "amr_noalloc.hip", "amr_stream.hip", "amr_cluster.cpp")]
ARCH = os.environ.get("AMR_OFFLOAD_ARCH", "gfx950")


def _flags():
    return ["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-result",
            "-I", os.path.join(ROOT, "include")]


def build(verbose: bool = False, extra=(), jobs: int = 0) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    objs = [os.path.join(OBJDIR, os.path.basename(s) + ".o") for s in SOURCES]
    cmds = [[*_flags(), "-c", "-o", o, s, *extra] for s, o in zip(SOURCES, objs)]
    jobs = jobs or min(len(cmds), os.cpu_count() or 1, 16)

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        return subprocess.run(cmd, capture_output=True, text=True)

    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(run, cmds))
    failed = [(c, r) for c, r in zip(cmds, results) if r.returncode != 0]
    for c, r in zip(cmds, results):
        if r.stderr and (verbose or r.returncode != 0):
            sys.stderr.write(r.stderr)
    if failed:
        raise subprocess.CalledProcessError(failed[0][1].returncode, failed[0][0])
    link = [*_flags(), "-shared", "-o", LIB + ".tmp", *objs]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
