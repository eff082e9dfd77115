"""Build the FP64 CPU oracle (test infrastructure) into ``oracle/liboracle.so``.

Compiled with plain gcc, ``-O2 -ffp-contract=off -fno-fast-math`` so that every
arithmetic operation is a single IEEE-rounded operation in source order.  This
serial build is the checker.  The same source is also built with ``-fopenmp``
into ``oracle/liboracle_omp.so``: its patch loops then run on several cores, with
every cell computed by the same operations, and it serves only to time the oracle
on all host cores beside the serial timing.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")


def _cmd(out, openmp):
    src = os.path.join(HERE, "oracle.c")
    return (["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
             "-Wall", "-Wextra", "-Wno-unused-parameter"] + (["-fopenmp"] if openmp else ["-Wno-unknown-pragmas"])
            + ["-o", out + ".tmp", src, "-lm"])


def build(verbose: bool = False) -> str:
    for out, omp in ((LIB, False), (LIB_OMP, True)):
        cmd = _cmd(out, omp)
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
