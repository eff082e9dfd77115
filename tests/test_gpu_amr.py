"""GPU parity of the hierarchy path (coarse/fine coupling): amr_hydro_advance and
amr_flux_correct against the oracle's subcycled two-/three-level step.

FP64: within 1e-12 of the oracle per cell and variable (the kernels repeat the
oracle's operations, so bitwise agreement is expected and reported); mixed:
relative L1 of density <= 1e-5 against the FP64 oracle.  Both conserve the
composite totals to round-off.
"""
import numpy as np
import pytest

from paper_0910_5547_amd import workloads as W
from tests.gpu_util import active_all, l1_rel, log, rel_err

pytestmark = pytest.mark.gpu

CASES = {
    "two_level_3d": lambda: W.two_level_box(Nc=16, fine_lo=(4, 6, 4), fine_n=(8, 6, 8), coarse_split=2, seed=51),
    "two_level_2d": lambda: W.two_level_box(Nc=32, fine_lo=(8, 6, 0), fine_n=(12, 10, 1), ndim=2, coarse_split=2,
                                            seed=52),
    "two_level_1d": lambda: W.two_level_box(Nc=64, fine_lo=(16, 0, 0), fine_n=(24, 1, 1), ndim=1, coarse_split=2,
                                            seed=53),
    "three_level_3d": lambda: W.nested_box(Nc=16, boxes=((4, 12), (10, 14)), seed=54),
}


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import oracle as O
    from paper_0910_5547_amd import amr as A
    A.lib()
    return torch, A, O


def run_pair(env, case, steps, prec=0, exe=1, shape=None):
    torch, A, O = env
    ps, U, per, dom = CASES[case]()
    T = A.Table(ps, precision=prec, exec_form=exe, periodic=per, domain=dom)
    if shape is not None:
        A.amr_table_set_tiling(T.h, shape, 0)
    Ud = T.upload(U)
    o = O.AmrOracle(ps, periodic=per, domain=dom)
    Uo = U.copy()
    for s in range(steps):
        dt = A.amr_cfl_dt(T.h, Ud, 0.8, -1, T.dt, host=True)
        if prec == 0:
            assert dt == o.cfl_dt0(Uo, 0.8), s
        A.amr_hydro_advance(T.h, Ud, T.dt)
        o.advance(Uo, dt)
    torch.cuda.synchronize()
    assert T.status() == A.AMR_OK
    Ug = Ud.cpu().numpy()
    T.close()
    return ps, U, Ug, Uo


@pytest.mark.parametrize("exe,shape", [(1, None), (0, None), (1, 1), (1, 4), (1, 5), (1, 6), (1, 7)])
@pytest.mark.parametrize("case", list(CASES))
def test_hierarchy_fp64_matches_oracle(env, case, exe, shape):
    """shape None: the library's default tiling; 1, 4, 5, 6, 7: 32x8 workgroup, 8x8 wavefront, 32x16 (512 threads),
    32x12 (384) and patch-fit tiles."""
    if shape is not None and case.endswith("1d"):
        pytest.skip("1D tables have the one 1D tiling")
    log(f"case amr {case} fp64 exec={exe} shape={shape}")
    ps, U0, Ug, Uo = run_pair(env, case, 3, prec=0, exe=exe, shape=shape)
    g, r = active_all(ps, Ug), active_all(ps, Uo)
    e = rel_err(g, r)
    log(f"{case} exec={exe} shape={shape}: rel err {['%.1e' % x for x in e]} bitwise={np.array_equal(g, r)}")
    assert max(e) <= 1e-12, e
    t0 = W.composite_totals(ps, U0)
    sc = W.composite_totals(ps, np.abs(U0))
    t1 = W.composite_totals(ps, Ug)
    assert np.all(np.abs(t1 - t0) <= 1e-12 * sc), (t1 - t0) / sc


@pytest.mark.parametrize("shape", [None, 1, 4, 5, 7])
@pytest.mark.parametrize("case", list(CASES))
def test_hierarchy_mixed(env, case, shape):
    if shape is not None and case.endswith("1d"):
        pytest.skip("1D tables have the one 1D tiling")
    log(f"case amr {case} mixed shape={shape}")
    ps, U0, Ug, Uo = run_pair(env, case, 3, prec=1, shape=shape)
    g, r = active_all(ps, Ug), active_all(ps, Uo)
    l1 = l1_rel(g, r)
    log(f"{case} mixed: L1(rho) {l1:.2e}")
    assert l1 <= 1e-5
    t0 = W.composite_totals(ps, U0)
    sc = W.composite_totals(ps, np.abs(U0))
    t1 = W.composite_totals(ps, Ug)
    assert np.all(np.abs(t1 - t0) <= 1e-12 * sc), (t1 - t0) / sc


def test_manual_level_steps_equal_advance(env):
    """Driving the recursion through amr_hydro_rk2_step (with the substep flag) and
    amr_flux_correct gives bitwise the result of amr_hydro_advance."""
    torch, A, O = env
    log("case amr manual drive")
    ps, U, per, dom = CASES["three_level_3d"]()
    T = A.Table(ps, precision=0, exec_form=1, periodic=per, domain=dom)
    Ua, Um = T.upload(U), T.upload(U)
    dt0 = A.amr_cfl_dt(T.h, Ua, 0.8, -1, T.dt, host=True)
    A.amr_hydro_advance(T.h, Ua, T.dt)
    dts = [torch.full((1,), dt0 / 2 ** l, dtype=torch.float64, device="cuda") for l in range(3)]

    def adv(l, sub):
        A.amr_hydro_rk2_step(T.h, Um, dts[l], l, A.AMR_STEP_SUBSTEP1 if sub else 0)
        if l < 2:
            adv(l + 1, 0)
            adv(l + 1, 1)
            A.amr_flux_correct(T.h, Um, l)

    adv(0, 0)
    torch.cuda.synchronize()
    assert np.array_equal(active_all(ps, Ua.cpu().numpy()), active_all(ps, Um.cpu().numpy()))
    T.close()


def _composite_mass_energy(ps, U):
    t = W.composite_totals(ps, U)
    return t[0], t[4]


def test_sedov_reduced_depth_matches_oracle(env):
    """Octant Sedov blast with the root and two refined levels: one subcycled root step
    on the GPU (FP64, batched) against the oracle."""
    torch, A, O = env
    log("case sedov 2 levels")
    ps, U, per, dom = W.sedov_hierarchy(levels=2)
    T = A.Table(ps, precision=0, exec_form=1, **W.SEDOV_FLOORS)
    Ud = T.upload(U)
    dt = A.amr_cfl_dt(T.h, Ud, 0.8, -1, T.dt, host=True)
    o = O.AmrOracle(ps, **W.SEDOV_FLOORS)
    Uo = U.copy()
    assert dt == o.cfl_dt0(Uo, 0.8)
    A.amr_hydro_advance(T.h, Ud, T.dt)
    o.advance(Uo, dt)
    assert T.status() == A.AMR_OK
    g, r = active_all(ps, Ud.cpu().numpy()), active_all(ps, Uo)
    e = rel_err(g, r)
    log(f"sedov 2 levels: {['%.1e' % x for x in e]} bitwise={np.array_equal(g, r)}")
    assert max(e) <= 1e-12
    T.close()


def test_sedov_full_hierarchy_conserves_and_mixed_tracks_fp64(env):
    """The full 7-level octant Sedov hierarchy (~6300 patches): two root steps in FP64 and
    mixed.  Reflecting walls and the outflow far faces (gas at rest) carry no mass or
    energy flux, so composite mass and energy are conserved to round-off; the mixed
    path's density stays within 1e-5 (relative L1) of the FP64 path's."""
    torch, A, O = env
    log("case sedov full")
    ps, U, per, dom = W.sedov_hierarchy()
    out = {}
    for prec in (0, 1):
        T = A.Table(ps, precision=prec, exec_form=1, **W.SEDOV_FLOORS)
        Ud = T.upload(U)
        for _ in range(2):
            A.amr_cfl_dt(T.h, Ud, 0.8, -1, T.dt)
            A.amr_hydro_advance(T.h, Ud, T.dt)
        torch.cuda.synchronize()
        assert T.status() == A.AMR_OK, prec
        out[prec] = Ud.cpu().numpy()
        T.close()
    m0, e0 = _composite_mass_energy(ps, U)
    sc = W.composite_totals(ps, np.abs(U))
    for prec in (0, 1):
        m, e = _composite_mass_energy(ps, out[prec])
        log(f"sedov prec={prec}: mass drift {(m - m0) / sc[0]:.2e}, energy drift {(e - e0) / sc[4]:.2e}")
        assert abs(m - m0) <= 1e-12 * sc[0] and abs(e - e0) <= 1e-12 * sc[4]
    l1 = l1_rel(active_all(ps, out[1]), active_all(ps, out[0]))
    log(f"sedov mixed vs fp64 L1(rho) = {l1:.2e}")
    assert l1 <= 1e-5


@pytest.mark.parametrize("exe,prec", [(1, 0), (0, 0), (1, 1)])
@pytest.mark.parametrize("ndim,nlev", [(1, 3), (3, 2), (3, 3)])
def test_subcycled_ramp_exact_on_gpu(env, ndim, nlev, exe, prec):
    """The advected linear ramp on a subcycled hierarchy (the oracle's time-schedule pin):
    the GPU's refined cells reproduce the exact solution, FP64 to 1e-13 and bitwise equal
    to the oracle, mixed to FP32 rounding (the face fluxes are FP32), with the ghosts of
    each stage taken at that stage's own fraction of the parent step."""
    from tests.test_oracle_amr_schedule import CASES as RC, ramp_errors, ramp_hierarchy
    torch, A, O = env
    log(f"case amr ramp ndim={ndim} levels={nlev} exec={exe} prec={prec}")
    Nc, boxes, grad, vel = RC[ndim]
    ps, U = ramp_hierarchy(ndim, Nc, boxes[:nlev - 1], grad, vel)
    T = A.Table(ps, precision=prec, exec_form=exe, recon=A.AMR_RECON_P)
    Ud = T.upload(U)
    o = O.AmrOracle(ps, recon=O.RECON_P)
    Uo = U.copy()
    t, steps = 0.0, 2
    for s in range(steps):
        dt = A.amr_cfl_dt(T.h, Ud, 0.8, -1, T.dt, host=True)
        dto = o.cfl_dt0(Uo, 0.8)
        if prec == 0:
            assert dt == dto, s
        T.dt.fill_(dto)  # both sides on the oracle's time step
        A.amr_hydro_advance(T.h, Ud, T.dt)
        o.advance(Uo, dto)
        t += dto
    torch.cuda.synchronize()
    assert T.status() == A.AMR_OK
    Ug = Ud.cpu().numpy()
    T.close()
    errs = ramp_errors(ps, Ug, t, steps)
    log(f"ramp ndim={ndim} levels={nlev} exec={exe} prec={prec}: max |U - exact| per level {errs}")
    tol = 1e-13 if prec == 0 else 1e-5
    assert max(errs.values()) <= tol, errs
    if prec == 0:
        assert np.array_equal(active_all(ps, Ug), active_all(ps, Uo))
