"""Pins of the oracle's subcycled, refluxed hierarchy step for MHD (8 variables) and
GLM-MHD (9): the coarse/fine coupling of Sec. 3 (Berger-Colella) applied to the
paper's MHD system, every conserved variable alike.

* A uniform magnetised state stays uniform (prolongation and time interpolation of B
  and psi are exact on constants; the fine/coarse fluxes of a constant state agree).
* Composite totals of all nvar variables are conserved to round-off with refluxing,
  and drift far above round-off without it (the field's fluxes need the correction
  as much as the hydro ones).
* Covered coarse cells hold the mean of their children for every variable.
* A fine patch over the middle of a 1D MHD problem is closer to an all-fine run than
  an all-coarse run is.
"""
import numpy as np
import pytest

from paper_0910_5547_amd import workloads as W


def _run(oracle_lib, ps, U, per, dom, steps, correct=True, ch=0.0):
    a = oracle_lib.AmrOracle(ps, periodic=per, domain=dom, ch=ch)
    if not correct:
        a.correct = lambda U, l: None
    for _ in range(steps):
        a.advance(U, a.cfl_dt0(U, 0.8))
    return a


@pytest.mark.parametrize("nvar", [8, 9])
@pytest.mark.parametrize("ndim,split", [(3, 2), (2, 1), (1, 2)])
def test_uniform_magnetised_state_stays_uniform(oracle_lib, ndim, split, nvar):
    ps, U, per, dom = W.two_level_box(Nc=16, fine_lo=(4, 4, 4)[:ndim] + (0,) * (3 - ndim),
                                      fine_n=(8, 8, 8)[:ndim] + (1,) * (3 - ndim), uniform=True, ndim=ndim,
                                      coarse_split=split, nvar=nvar)
    U0 = U.copy()
    _run(oracle_lib, ps, U, per, dom, 3, ch=2.0)
    for p in range(ps.npatch):
        a, b = ps.active(U, p), ps.active(U0, p)
        assert np.max(np.abs(a - b) / np.maximum(np.abs(b), 1)) <= 1e-15


@pytest.mark.parametrize("nvar,ch", [(8, 0.0), (9, 2.5)])
@pytest.mark.parametrize("ndim", [3, 2, 1])
def test_composite_conservation_with_refluxing_mhd(oracle_lib, ndim, nvar, ch):
    lo = (4, 6, 4)[:ndim] + (0,) * (3 - ndim)
    n = (8, 6, 8)[:ndim] + (1,) * (3 - ndim)
    ps, U, per, dom = W.two_level_box(Nc=16, fine_lo=lo, fine_n=n, ndim=ndim, coarse_split=2, seed=71, nvar=nvar)
    t0 = W.composite_totals(ps, U)
    scale = W.composite_totals(ps, np.abs(U))
    _run(oracle_lib, ps, U, per, dom, 4, ch=ch)
    t1 = W.composite_totals(ps, U)
    scale = np.maximum(scale, W.composite_totals(ps, np.abs(U)))  # (rho v_y starts at 0 in 1D)
    assert np.all(np.abs(t1 - t0) <= 1e-13 * scale), (t1 - t0) / scale
    # negative control: without refluxing the totals drift, the field's included
    ps, U, per, dom = W.two_level_box(Nc=16, fine_lo=lo, fine_n=n, ndim=ndim, coarse_split=2, seed=71, nvar=nvar)
    _run(oracle_lib, ps, U, per, dom, 4, correct=False, ch=ch)
    t2 = W.composite_totals(ps, U)
    drift = np.abs(t2 - t0) / np.maximum(scale, 1e-300)
    assert drift[0] > 1e-8 and np.max(drift[5:8]) > 1e-8, drift


@pytest.mark.parametrize("nvar", [8, 9])
def test_restriction_is_the_mean_of_children_mhd(oracle_lib, nvar):
    ps, U, per, dom = W.two_level_box(Nc=16, coarse_split=1, seed=72, nvar=nvar)
    _run(oracle_lib, ps, U, per, dom, 2, ch=1.5)
    fine = [p for p in range(ps.npatch) if ps.level[p] == 1][0]
    f = ps.active(U, fine)
    mean = sum(f[:, dz::2, dy::2, dx::2] for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)) / 8
    lo, n = ps.lo[fine] // 2, ps.n[fine] // 2
    got = ps.active(U, 0)[:, lo[2]:lo[2] + n[2], lo[1]:lo[1] + n[1], lo[0]:lo[0] + n[0]]
    assert got.shape[0] == nvar
    assert np.allclose(got, mean, rtol=1e-15, atol=1e-15)


@pytest.mark.parametrize("nvar", [8, 9])
def test_three_levels_conserve_mhd(oracle_lib, nvar):
    ps, U, per, dom = W.nested_box(Nc=16, boxes=((4, 12), (10, 14)), seed=73, nvar=nvar)
    t0 = W.composite_totals(ps, U)
    scale = W.composite_totals(ps, np.abs(U))
    _run(oracle_lib, ps, U, per, dom, 3, ch=2.0)
    t1 = W.composite_totals(ps, U)
    scale = np.maximum(scale, W.composite_totals(ps, np.abs(U)))
    live = scale > 0
    assert np.all(np.abs(t1 - t0)[live] <= 1e-13 * scale[live])


def test_fine_patch_is_closer_to_fine_reference_mhd(oracle_lib):
    """1D MHD: a fine patch over the middle of the domain; after t = 0.05 its cells are closer
    to an all-fine run than the all-coarse run's cells are, in every variable that moves."""
    Nc = 64
    kw = dict(ndim=1, coarse_split=1, seed=74, amp=0.3, vamp=0.5, nvar=8)
    ps, U, per, dom = W.two_level_box(Nc=Nc, fine_lo=(16, 0, 0), fine_n=(32, 1, 1), **kw)
    fine = [p for p in range(ps.npatch) if ps.level[p] == 1][0]
    psf, Uf, _, _ = W.two_level_box(Nc=Nc, fine_lo=(0, 0, 0), fine_n=(Nc, 1, 1), **kw)
    full = [p for p in range(psf.npatch) if psf.level[p] == 1][0]
    ref_ps = W.make_patchset(1, [[2 * Nc, 1, 1]], 3, [W.BC_PERIODIC] * 6, gamma=ps.gamma, dx0=(0.5 / Nc, 1, 1),
                             nvar=8)
    ref = W.new_arena(ref_ps)
    ref_ps.active(ref, 0)[...] = psf.active(Uf, full)
    crs_ps = W.make_patchset(1, [[Nc, 1, 1]], 3, [W.BC_PERIODIC] * 6, gamma=ps.gamma, dx0=(1.0 / Nc, 1, 1), nvar=8)
    crs = W.new_arena(crs_ps)
    crs_ps.active(crs, 0)[...] = ps.active(U, 0)
    a = oracle_lib.AmrOracle(ps, periodic=per, domain=dom)
    oref, ocrs = oracle_lib.Oracle(ref_ps), oracle_lib.Oracle(crs_ps)
    t = 0.0
    while t < 0.05:
        dt0 = min(a.cfl_dt0(U, 0.4), ocrs.cfl_dt(crs, 0.4), 2 * oref.cfl_dt(ref, 0.4), 0.05 - t)
        a.advance(U, dt0)
        ocrs.rk2_step(crs, dt0)
        oref.rk2_step(ref, dt0 / 2)
        oref.rk2_step(ref, dt0 / 2)
        t += dt0
    for k in (0, 1, 4, 6, 7):  # rho, rho vx, energy, By, Bz (Bx is constant in 1D)
        r = ref_ps.active(ref, 0)[k, 0, 0, 32:96]
        comp = ps.active(U, fine)[k, 0, 0, :]
        coarse_on_fine = np.repeat(crs_ps.active(crs, 0)[k, 0, 0, 16:48], 2)
        assert np.abs(comp - r).sum() < 0.5 * np.abs(coarse_on_fine - r).sum(), k
