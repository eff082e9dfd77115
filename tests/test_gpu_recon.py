"""GPU parity of the pressure reconstruction (AMR_RECON_P: p is reconstructed instead
of e) against the oracle with the same flag, for hydro, MHD and a hierarchy.

Bars as for the default reconstruction: FP64 bitwise (within 1e-12 per cell and
variable) against the oracle; mixed L1(rho) <= 1e-5 with totals conserved to 1e-12.
"""
import math

import numpy as np
import pytest

from paper_0910_5547_amd import workloads as W
from tests.gpu_util import active_all, l1_rel, log, rel_err, totals

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import oracle as O
    from paper_0910_5547_amd import amr as A
    A.lib()
    return torch, A, O


def run_pair(env, ps, U, steps, prec=0, periodic=0, domain=(0, 0, 0), shape=None, check_dt=True):
    torch, A, O = env
    T = A.Table(ps, precision=prec, periodic=periodic, domain=domain, recon=A.AMR_RECON_P)
    if shape is not None:
        A.amr_table_set_tiling(T.h, shape, 0)
    Ud = T.upload(U)
    o = O.Oracle(ps, periodic=periodic, domain=domain, recon=O.RECON_P)
    Uo = U.copy()
    for s in range(steps):
        dt = T.cfl_dt(Ud, 0.8)
        if check_dt:
            assert dt == o.cfl_dt(Uo, 0.8), s
        T.step(Ud)
        assert o.rk2_step(Uo, dt) == 0
    torch.cuda.synchronize()
    assert T.status() == A.AMR_OK
    Ug = Ud.cpu().numpy()
    T.close()
    return Ug, Uo


def _check(ps, Ug, Uo, what):
    g, r = active_all(ps, Ug), active_all(ps, Uo)
    e = rel_err(g, r)
    log(f"{what}: max rel err {max(e):.2e} bitwise={np.array_equal(g, r)}")
    assert np.array_equal(g, r) and max(e) <= 1e-12


def test_sod_fp64(env):
    log("case recon-p sod")
    ps, U = W.sod(400)
    Ug, Uo = run_pair(env, ps, U, 60)
    _check(ps, Ug, Uo, "recon-p sod")


@pytest.mark.parametrize("shape", [1, 4, 5])
def test_ragged_3d_fp64(env, shape):
    log(f"case recon-p ragged shape={shape}")
    bcs = [W.BC_REFLECT, W.BC_OUTFLOW, W.BC_PERIODIC, W.BC_PERIODIC, W.BC_OUTFLOW, W.BC_REFLECT]
    ps = W.make_patchset(3, [[37, 13, 11], [9, 26, 19]], 3, bcs, gamma=1.4, dx0=(0.03, 0.05, 0.04))
    U = W.random_state(ps, 14, shocks=1.0)
    Ug, Uo = run_pair(env, ps, U, 3, shape=shape)
    _check(ps, Ug, Uo, f"recon-p ragged shape={shape}")


def test_mhd_vortex_fp64_and_mixed(env):
    log("case recon-p mhd vortex")
    N = 48
    ps, U = W.mhd_vortex_box(N, patch=16, seed=50)
    Ug, Uo = run_pair(env, ps, U, 3, periodic=7, domain=(N, N, N))
    _check(ps, Ug, Uo, "recon-p mhd vortex48")
    A0 = active_all(ps, U)
    Ug, Uo = run_pair(env, ps, U, 6, prec=1, periodic=7, domain=(N, N, N), check_dt=False)
    g, r = active_all(ps, Ug), active_all(ps, Uo)
    assert l1_rel(g, r) <= 1e-5
    t0, t1 = totals(A0), totals(g)
    for k in range(8):
        scale = max(math.fsum(np.abs(A0[k])), math.fsum(np.abs(g[k])))
        assert abs(t1[k] - t0[k]) <= 1e-12 * scale, k


def test_mixed_box(env):
    log("case recon-p mixed box")
    ps, U = W.periodic_turbulent_box(N=32, seed=20, kmax=8.0)
    A0 = active_all(ps, U)
    Ug, Uo = run_pair(env, ps, U, 10, prec=1, check_dt=False)
    g, r = active_all(ps, Ug), active_all(ps, Uo)
    l1 = l1_rel(g, r)
    log(f"recon-p mixed box: L1(rho) {l1:.2e}")
    assert l1 <= 1e-5
    t0, t1 = totals(A0), totals(g)
    for k in range(5):
        assert abs(t1[k] - t0[k]) <= 1e-12 * math.fsum(np.abs(A0[k])), k


def test_hierarchy_fp64(env):
    """Two-level 3D box: refluxing recomputes the coarse fluxes with the same reconstruction."""
    torch, A, O = env
    log("case recon-p hierarchy")
    ps, U, per, dom = W.two_level_box(Nc=16, fine_lo=(4, 6, 4), fine_n=(8, 6, 8), coarse_split=2, seed=51)
    T = A.Table(ps, precision=0, exec_form=1, periodic=per, domain=dom, recon=A.AMR_RECON_P)
    Ud = T.upload(U)
    o = O.AmrOracle(ps, periodic=per, domain=dom, recon=O.RECON_P)
    Uo = U.copy()
    for s in range(3):
        dt = A.amr_cfl_dt(T.h, Ud, 0.8, -1, T.dt, host=True)
        assert dt == o.cfl_dt0(Uo, 0.8), s
        A.amr_hydro_advance(T.h, Ud, T.dt)
        o.advance(Uo, dt)
    assert T.status() == A.AMR_OK
    g, r = active_all(ps, Ud.cpu().numpy()), active_all(ps, Uo)
    T.close()
    e = rel_err(g, r)
    log(f"recon-p hierarchy: {max(e):.2e} bitwise={np.array_equal(g, r)}")
    assert max(e) <= 1e-12
