"""Acceptance runs against the oracle at the sizes the scope sets: the periodic box at 64^3
for 100 RK2 steps, 200 uneven patches for 10 steps, and one subcycled root step of the
octant Sedov hierarchy with four levels (root and three refined levels, about 1500
patches of 8^3-32^3 with 8^3 wavefront tiles on the deep levels).

Bars: FP64 within 1e-12 of the oracle per cell and variable (relative to the variable's
largest magnitude; bitwise agreement is expected and reported); mixed (FP32 reconstruction
and flux, FP64 accumulation) relative L1 of density within 1e-5 of the FP64 oracle, with
the totals conserved to 1e-12 where the boundaries conserve them (periodic box, periodic
patches; the Sedov octant's reflecting walls and quiescent outflow faces); on outflow patches
FP64 totals equal the oracle's to 1e-12.  The oracle is fed the GPU's time steps.
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


def _run(env, ps, U, steps, prec, kw=None, okw=None):
    torch, A, O = env
    T = A.Table(ps, precision=prec, exec_form=A.AMR_EXEC_BATCHED, **(kw or {}))
    Ud = T.upload(U)
    o = O.Oracle(ps, **(okw or {}))
    Uo = U.copy()
    for s in range(steps):
        dt = T.cfl_dt(Ud, 0.8)
        if prec == 0:
            assert dt == o.cfl_dt(Uo, 0.8), s
        T.step(Ud)
        assert o.rk2_step(Uo, dt) == 0, s
    torch.cuda.synchronize()
    assert T.status() == A.AMR_OK
    Ug = Ud.cpu().numpy()
    T.close()
    return active_all(ps, Ug), active_all(ps, Uo)


def _scale(A0):
    return [math.fsum(np.abs(A0[k])) for k in range(len(A0))]


@pytest.mark.parametrize("prec", [0, 1])
def test_periodic_box_64_for_100_steps(env, prec):
    log(f"case box64 x 100 prec={prec}")
    ps, U = W.periodic_turbulent_box(N=64, seed=20, kmax=16.0)
    A0 = active_all(ps, U)
    g, r = _run(env, ps, U, 100, prec)
    sc = _scale(A0)
    drift = [abs(a - b) / s for a, b, s in zip(totals(g), totals(A0), sc)]
    if prec == 0:
        e = rel_err(g, r)
        log(f"box64 fp64: max rel err {max(e):.1e}, bitwise={np.array_equal(g, r)}, drift {max(drift):.1e}")
        assert max(e) <= 1e-12
    else:
        l1 = l1_rel(g, r)
        log(f"box64 mixed: L1(rho) {l1:.2e}, L1 per var {['%.1e' % l1_rel(g, r, k) for k in range(5)]}, "
            f"drift {max(drift):.1e}")
        assert l1 <= 1e-5
    assert max(drift) <= 1e-12


@pytest.mark.parametrize("prec", [0, 1])
def test_uneven_patches_200_for_10_steps(env, prec):
    """The 4000-patch configuration's first 200 patches (outflow faces).  Their totals move
    by the boundary fluxes, which the mixed form evaluates in FP32: its totals follow the
    oracle's to FP32 rounding of those fluxes, and the same patches with periodic faces,
    whose totals the scheme conserves, check its conservation to 1e-12."""
    log(f"case uneven 200 x 10 prec={prec}")
    ps, U = W.uneven_patches(npatch=200, seed=30)
    g, r = _run(env, ps, U, 10, prec)
    sc = _scale(r)
    dtot = [abs(a - b) / s for a, b, s in zip(totals(g), totals(r), sc)]
    if prec == 0:
        e = rel_err(g, r)
        log(f"uneven200 fp64: max rel err {max(e):.1e}, bitwise={np.array_equal(g, r)}")
        assert max(e) <= 1e-12
        assert max(dtot) <= 1e-12
    else:
        l1 = l1_rel(g, r)
        log(f"uneven200 mixed: L1(rho) {l1:.2e}, totals vs oracle {max(dtot):.1e}")
        assert l1 <= 1e-5
        assert max(dtot) <= 1e-7
    psp = W.make_patchset(3, ps.n, ps.ng, [W.BC_PERIODIC] * 6, gamma=ps.gamma, dx0=ps.dx0)
    Up = W.new_arena(psp)
    for p in range(ps.npatch):
        psp.active(Up, p)[...] = ps.active(U, p)
    A0 = active_all(psp, Up)
    g, r = _run(env, psp, Up, 10, prec)
    drift = [abs(a - b) / s for a, b, s in zip(totals(g), totals(A0), _scale(A0))]
    log(f"uneven200 periodic faces prec={prec}: drift {max(drift):.1e}, L1(rho) {l1_rel(g, r):.2e}")
    assert max(drift) <= 1e-12
    assert l1_rel(g, r) <= (1e-12 if prec == 0 else 1e-5)


def test_sedov_four_levels_one_root_step(env):
    """One subcycled root step (levels 0-3, 15 level steps with refluxing and restriction)
    on the GPU in both precisions, against the oracle's hierarchy step with the same dt0."""
    torch, A, O = env
    log("case sedov levels 0-3")
    ps, U, _, _ = W.sedov_hierarchy(levels=3)
    o = O.AmrOracle(ps, **W.SEDOV_FLOORS)
    Uo = U.copy()
    dt0 = o.cfl_dt0(Uo, 0.8)
    o.advance(Uo, dt0)
    r = active_all(ps, Uo)
    m0 = W.composite_totals(ps, U)
    sc = W.composite_totals(ps, np.abs(U))
    mo = W.composite_totals(ps, Uo)
    assert abs(mo[0] - m0[0]) <= 1e-12 * sc[0] and abs(mo[4] - m0[4]) <= 1e-12 * sc[4]
    for prec in (0, 1):
        T = A.Table(ps, precision=prec, exec_form=A.AMR_EXEC_BATCHED, **W.SEDOV_FLOORS)
        Ud = T.upload(U)
        dt = A.amr_cfl_dt(T.h, Ud, 0.8, -1, T.dt, host=True)
        if prec == 0:
            assert dt == dt0
        T.dt.fill_(dt0)
        A.amr_hydro_advance(T.h, Ud, T.dt)
        torch.cuda.synchronize()
        assert T.status() == A.AMR_OK
        Ug = Ud.cpu().numpy()
        T.close()
        g = active_all(ps, Ug)
        mg = W.composite_totals(ps, Ug)
        drift = max(abs(mg[0] - m0[0]) / sc[0], abs(mg[4] - m0[4]) / sc[4])
        if prec == 0:
            e = rel_err(g, r)
            log(f"sedov 0-3 fp64: max rel err {max(e):.1e}, bitwise={np.array_equal(g, r)}, drift {drift:.1e}")
            assert max(e) <= 1e-12
        else:
            l1 = l1_rel(g, r)
            log(f"sedov 0-3 mixed: L1(rho) {l1:.2e}, drift {drift:.1e}")
            assert l1 <= 1e-5
        assert drift <= 1e-12
