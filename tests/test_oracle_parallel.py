"""The OpenMP build of the oracle (used only to time it on all host cores) computes
every cell with the serial build's operations: same bits on uneven patches, with
EXTERNAL siblings and on a two-level hierarchy's level steps."""
import numpy as np

from paper_0910_5547_amd import workloads as W


def _active(ps, U):
    return np.concatenate([ps.active(U, p).ravel() for p in range(ps.npatch)])


def test_openmp_build_gives_the_serial_bits(oracle_lib):
    O = oracle_lib
    ps, U = W.uneven_patches(npatch=48, seed=35)
    out = []
    for par in (False, True):
        o = O.Oracle(ps, parallel=par)
        V = U.copy()
        for _ in range(3):
            assert o.rk2_step(V, o.cfl_dt(V, 0.8)) == 0
        out.append(_active(ps, V))
    assert O.lib(True).or_threads() >= 1 and O.lib().or_threads() == 1
    assert np.array_equal(out[0], out[1])


def test_openmp_build_external_siblings(oracle_lib):
    O = oracle_lib
    ps, U = W.periodic_turbulent_box(N=32, seed=20, kmax=8.0, patch=8, ng=3)
    out = []
    for par in (False, True):
        o = O.Oracle(ps, periodic=7, domain=(32, 32, 32), parallel=par)
        V = U.copy()
        for _ in range(2):
            assert o.rk2_step(V, o.cfl_dt(V, 0.8)) == 0
        out.append(_active(ps, V))
    assert np.array_equal(out[0], out[1])
