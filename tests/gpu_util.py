"""Helpers shared by the GPU tests: run the HIP library and the CPU oracle on
the same seeded inputs and compare per cell and variable."""
import math
import sys

import numpy as np


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def active_all(ps, U):
    """(nvar, cells) array of the active cells of every patch (patch order)."""
    return np.concatenate([ps.active(U, p).reshape(ps.nvar, -1) for p in range(ps.npatch)], axis=1)


def rel_err(got, ref):
    """Per-variable max |got - ref| / max |ref| (the relative-per-cell tolerance with the
    variable's own scale, so that near-zero momenta do not make it meaningless)."""
    out = []
    for k in range(len(ref)):
        scale = max(np.max(np.abs(ref[k])), 1e-300)
        out.append(float(np.max(np.abs(got[k] - ref[k])) / scale))
    return out


def l1_rel(got, ref, k=0):
    return float(np.sum(np.abs(got[k] - ref[k])) / np.sum(np.abs(ref[k])))


def totals(A):
    return [math.fsum(A[k]) for k in range(len(A))]
