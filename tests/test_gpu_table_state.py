"""GPU tests of the table's state across calls: the autotuner leaves the caller's
U, the unphysical latch and the hierarchy's recursion state as they were, and the
maxima fused into a step's stage 2 are read once, so the recovery recipe of the
C ABI (clear the latch, restore U^n in place, rescan, retry) sees U^n's own dt.
"""
import numpy as np
import pytest

from paper_0910_5547_amd import workloads as W
from tests.gpu_util import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0910_5547_amd import amr as A
    A.lib()
    return torch, A


def _step_once(A, torch, ps, U, prec, tiling=None):
    T = A.Table(ps, precision=prec)
    if tiling is not None:
        A.amr_table_set_tiling(T.h, *tiling)
    Ud = T.upload(U)
    T.cfl_dt(Ud, 0.8)
    T.step(Ud)
    torch.cuda.synchronize()
    assert T.status() == A.AMR_OK
    out = Ud.cpu().numpy()
    T.close()
    return out


@pytest.mark.parametrize("prec", [0, 1])
def test_autotune_keeps_u_and_status_and_next_step_bits(env, prec):
    torch, A = env
    ps, U = W.uneven_patches(npatch=24, seed=31)
    log(f"case autotune uneven 24 prec={prec}")
    T = A.Table(ps, precision=prec)
    Ud = T.upload(U)
    T.cfl_dt(Ud, 0.8)
    before = Ud.clone()
    ms = A.amr_autotune(T.h, Ud, T.dt, -1, 2)
    torch.cuda.synchronize()
    assert ms > 0
    assert torch.equal(Ud.view(torch.int64), before.view(torch.int64)), "autotune modified U"  # ghosts hold NaN
    shape, zslab = A.amr_table_get_tiling(T.h)
    assert 1 <= shape < A.amr_table_num_tilings(T.h) and zslab >= 1
    assert T.status() == A.AMR_OK
    T.step(Ud)
    torch.cuda.synchronize()
    assert T.status() == A.AMR_OK
    tuned = Ud.cpu().numpy()
    T.close()
    untuned = _step_once(A, torch, ps, U, prec)
    assert np.array_equal(tuned, untuned, equal_nan=True)


def test_autotune_leaves_a_set_latch_set_and_a_clear_one_clear(env):
    torch, A = env
    ps, U = W.uneven_patches(npatch=8, seed=32)
    T = A.Table(ps, precision=0)
    # a state with negative density in one active cell of patch 0 latches the flag
    bad = U.copy()
    ps.active(bad, 0)[0, 1, 1, 1] = -1.0
    Ub = T.upload(bad)
    T.dt.fill_(1e-4)
    T.step(Ub)
    torch.cuda.synchronize()
    Ud = T.upload(U)
    A.amr_autotune(T.h, Ud, T.dt, -1, 1)
    assert T.status() == A.AMR_EUNPHYSICAL  # still the caller's latch
    assert T.status() == A.AMR_OK           # cleared by the status call
    # tuning on a bad copy of U does not latch the caller's table
    A.amr_autotune(T.h, Ub, T.dt, -1, 1)
    assert T.status() == A.AMR_OK
    T.close()


def test_autotune_refused_while_a_caller_recursion_is_open(env):
    torch, A = env
    ps, U, per, dom = W.two_level_box(Nc=16, fine_lo=(4, 4, 4), fine_n=(8, 8, 8), seed=41)
    T = A.Table(ps, precision=0, periodic=per, domain=dom)
    Ud = T.upload(U)
    T.cfl_dt(Ud, 0.8)
    dt0 = float(T.dt.item())
    # level 0 steps: its recursion is open until amr_flux_correct(0)
    A.amr_hydro_rk2_step(T.h, Ud, T.dt, 0, 0)
    with pytest.raises(A.AmrError) as ei:
        A.amr_autotune(T.h, Ud, T.dt, 1, 1)
    assert ei.value.status == A.AMR_ESTATE
    with pytest.raises(A.AmrError) as ei:
        A.amr_autotune(T.h, Ud, T.dt, -1, 1)  # a hierarchy needs one named level
    assert ei.value.status == A.AMR_EINVAL
    dt1 = torch.full((1,), dt0 / 2, dtype=torch.float64, device="cuda")
    A.amr_hydro_rk2_step(T.h, Ud, dt1, 1, 0)
    A.amr_hydro_rk2_step(T.h, Ud, dt1, 1, A.AMR_STEP_SUBSTEP1)
    A.amr_flux_correct(T.h, Ud, 0)
    # closed again: tuning is allowed, and the next root step is the untuned one's
    A.amr_autotune(T.h, Ud, dt1, 1, 1)
    T.dt.fill_(dt0)
    T.advance(Ud)
    torch.cuda.synchronize()
    assert T.status() == A.AMR_OK
    got = Ud.cpu().numpy()
    T.close()
    R = A.Table(ps, precision=0, periodic=per, domain=dom)
    Ur = R.upload(U)
    R.advance(Ur, dt0)
    R.advance(Ur, dt0)
    torch.cuda.synchronize()
    ref = Ur.cpu().numpy()
    R.close()
    for p in range(ps.npatch):
        assert np.array_equal(ps.active(got, p), ps.active(ref, p)), p


def test_second_substep_needs_the_first(env):
    """A level's second substep reuses the half-step ghosts its first substep prolonged: without
    that first substep since the parent's last step it is refused, and it is refused again once
    the parent has stepped anew; the refusal enqueues nothing."""
    torch, A = env
    ps, U, per, dom = W.two_level_box(Nc=16, fine_lo=(4, 4, 4), fine_n=(8, 8, 8), seed=42)
    T = A.Table(ps, precision=0, periodic=per, domain=dom)
    Ud = T.upload(U)
    T.cfl_dt(Ud, 0.8)
    dt1 = torch.full((1,), float(T.dt.item()) / 2, dtype=torch.float64, device="cuda")
    A.amr_hydro_rk2_step(T.h, Ud, T.dt, 0, 0)
    with pytest.raises(A.AmrError) as ei:
        A.amr_hydro_rk2_step(T.h, Ud, dt1, 1, A.AMR_STEP_SUBSTEP1)
    assert ei.value.status == A.AMR_ESTATE
    A.amr_hydro_rk2_step(T.h, Ud, dt1, 1, 0)
    A.amr_hydro_rk2_step(T.h, Ud, dt1, 1, A.AMR_STEP_SUBSTEP1)
    with pytest.raises(A.AmrError) as ei:  # used once per parent step
        A.amr_hydro_rk2_step(T.h, Ud, dt1, 1, A.AMR_STEP_SUBSTEP1)
    assert ei.value.status == A.AMR_ESTATE
    A.amr_flux_correct(T.h, Ud, 0)
    A.amr_hydro_rk2_step(T.h, Ud, T.dt, 0, 0)
    A.amr_hydro_rk2_step(T.h, Ud, dt1, 1, 0)
    A.amr_hydro_rk2_step(T.h, Ud, T.dt, 0, 0)  # the parent steps again: the half step is gone
    with pytest.raises(A.AmrError) as ei:
        A.amr_hydro_rk2_step(T.h, Ud, dt1, 1, A.AMR_STEP_SUBSTEP1)
    assert ei.value.status == A.AMR_ESTATE
    torch.cuda.synchronize()
    T.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_fused_maxima_are_read_once_recovery_recipe(env, prec):
    """The fused maxima are read by the first cfl_dt after the step only; after a fused step,
    status, then U^n restored into the same tensor, cfl_dt gives U^n's dt, not U^{n+1}'s."""
    torch, A = env
    ps, U = W.uneven_patches(npatch=16, seed=33)
    T = A.Table(ps, precision=prec)
    Ud = T.upload(U)
    dt_n = T.cfl_dt(Ud, 0.8)
    T.step(Ud, flags=A.AMR_STEP_FUSE_DT)
    dt_fused = T.cfl_dt(Ud, 0.8)           # reads the fused maxima of U^{n+1}
    dt_scan = T.cfl_dt(Ud, 0.8)            # a second call scans U^{n+1}
    assert dt_fused == dt_scan
    assert dt_fused != dt_n
    # the recipe after a rejected step: status (drops the fused maxima), restore U^n in
    # place, rescan, retry
    T.step(Ud, flags=A.AMR_STEP_FUSE_DT)
    assert T.status() == A.AMR_OK
    Ud.copy_(torch.from_numpy(U).to(Ud.device))
    dt_again = T.cfl_dt(Ud, 0.8)
    assert dt_again != dt_fused
    T2 = A.Table(ps, precision=prec)
    fresh = T2.cfl_dt(T2.upload(U), 0.8)
    T2.close()
    assert dt_again == fresh == dt_n
    T.close()


def test_latch_clears_fused_maxima_and_recipe_recovers(env):
    torch, A = env
    ps, U = W.uneven_patches(npatch=8, seed=34)
    T = A.Table(ps, precision=0)
    Ud = T.upload(U)
    dt_n = T.cfl_dt(Ud, 0.8)
    # far too large a dt drives the step unphysical
    T.dt.fill_(200 * dt_n)
    T.step(Ud, flags=A.AMR_STEP_FUSE_DT)
    with pytest.raises(A.AmrError) as ei:
        T.cfl_dt(Ud, 0.8)
    assert ei.value.status == A.AMR_EUNPHYSICAL
    with pytest.raises(A.AmrError):
        T.cfl_dt(Ud, 0.8)                  # the latch stays set until amr_table_status
    assert T.status() == A.AMR_EUNPHYSICAL
    Ud.copy_(torch.from_numpy(U).to(Ud.device))
    assert T.cfl_dt(Ud, 0.8) == dt_n
    T.step(Ud)
    torch.cuda.synchronize()
    assert T.status() == A.AMR_OK
    T.close()
