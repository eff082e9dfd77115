"""GPU parity of the GLM-MHD update (9 conserved variables: the ideal-MHD set and the
cleaning field psi, cleaning speed c_h) against the FP64 oracle with the same c_h.

Bars as for hydro and MHD: FP64 bitwise (within 1e-12 per cell and variable); mixed
L1(rho) <= 1e-5 with all nine totals conserved to 1e-12 on periodic domains.
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


def run_pair(env, ps, U, steps, ch, prec=0, exe=1, periodic=0, domain=(0, 0, 0), shape=None, check_dt=True, dt=None):
    torch, A, O = env
    T = A.Table(ps, precision=prec, exec_form=exe, periodic=periodic, domain=domain, ch=ch)
    if shape is not None:
        A.amr_table_set_tiling(T.h, shape, 0)
    Ud = T.upload(U)
    o = O.Oracle(ps, periodic=periodic, domain=domain, ch=ch)
    Uo = U.copy()
    for s in range(steps):
        if dt is None:
            d = T.cfl_dt(Ud, 0.8)
            if check_dt:
                assert d == o.cfl_dt(Uo, 0.8), s
            T.step(Ud)
        else:
            d = dt
            T.step(Ud, dt=d)
        assert o.rk2_step(Uo, d) == 0
    torch.cuda.synchronize()
    assert T.status() == A.AMR_OK
    Ug = Ud.cpu().numpy()
    T.close()
    return Ug, Uo


def _bitwise(ps, Ug, Uo, what):
    g, r = active_all(ps, Ug), active_all(ps, Uo)
    e = rel_err(g, r)
    log(f"{what}: max rel err {max(e):.2e} bitwise={np.array_equal(g, r)}")
    assert max(e) <= 1e-12
    assert np.array_equal(g, r)


def _glm_box(N, patch, seed=50):
    """The MHD vortex box with a psi field of the size of the divergence error a scheme makes."""
    ps8, U8 = W.mhd_vortex_box(N, patch=patch, seed=seed)
    ps = W.make_patchset(3, ps8.n, ps8.ng, ps8.bc, lo=ps8.lo, gamma=ps8.gamma, dx0=ps8.dx0, nvar=W.NVAR_GLM)
    U = W.new_arena(ps)
    rng = np.random.default_rng(seed)
    for p in range(ps.npatch):
        ps.active(U, p)[:8] = ps8.active(U8, p)
        ps.active(U, p)[8] = 0.01 * rng.standard_normal(ps.active(U, p)[8].shape)
    return ps, U


def test_cleaning_wave_fp64(env):
    log("case glm wave")
    ps, U = W.glm_wave(64, ch=2.0, eps=1e-3)
    Ug, Uo = run_pair(env, ps, U, 20, 2.0)
    _bitwise(ps, Ug, Uo, "glm wave")


@pytest.mark.parametrize("shape", [1, 4])
@pytest.mark.parametrize("bcs", [
    [W.BC_PERIODIC] * 6,
    [W.BC_REFLECT, W.BC_OUTFLOW, W.BC_PERIODIC, W.BC_PERIODIC, W.BC_OUTFLOW, W.BC_REFLECT],
])
def test_ragged_3d_fp64(env, bcs, shape):
    log(f"case glm ragged bcs={bcs} shape={shape}")
    ps = W.make_patchset(3, [[37, 13, 11], [9, 26, 19]], 2, bcs, gamma=5 / 3, dx0=(0.02, 0.05, 0.06), nvar=9)
    U = W.random_state(ps, 61, shocks=1.0)
    Ug, Uo = run_pair(env, ps, U, 3, 4.0, shape=shape)
    _bitwise(ps, Ug, Uo, f"glm ragged shape={shape}")


def test_two_dimensional_and_hll2_fp64(env):
    torch, A, O = env
    log("case glm 2d")
    ps = W.make_patchset(2, [[45, 29, 1]], 2, [W.BC_PERIODIC, W.BC_PERIODIC, W.BC_REFLECT, W.BC_OUTFLOW, 0, 0],
                         gamma=5 / 3, dx0=(0.02, 0.03, 1.0), nvar=9)
    U = W.random_state(ps, 62, shocks=1.0)
    Ug, Uo = run_pair(env, ps, U, 4, 3.0, shape=1)
    _bitwise(ps, Ug, Uo, "glm 2d")


@pytest.mark.parametrize("exe", [0, 1])
def test_vortex_box_external_patches_fp64(env, exe):
    log(f"case glm vortex48 exec={exe}")
    N = 48
    ps, U = _glm_box(N, 16)
    Ug, Uo = run_pair(env, ps, U, 3, 3.0, exe=exe, periodic=7, domain=(N, N, N))
    _bitwise(ps, Ug, Uo, f"glm vortex48 exec={exe}")


def test_zero_cleaning_speed_equals_mhd_library(env):
    """With c_h = 0 and psi = 0 the 9-variable kernels give the 8-variable kernels' bits."""
    torch, A, O = env
    log("case glm c_h=0")
    n = [[30, 17, 12]]
    ps8 = W.make_patchset(3, n, 2, [W.BC_PERIODIC] * 6, gamma=5 / 3, dx0=(0.03, 0.05, 0.07), nvar=8)
    U8 = W.random_state(ps8, 63, shocks=1.0)
    ps9 = W.make_patchset(3, n, 2, [W.BC_PERIODIC] * 6, gamma=5 / 3, dx0=(0.03, 0.05, 0.07), nvar=9)
    U9 = W.new_arena(ps9)
    ps9.active(U9, 0)[:8] = ps8.active(U8, 0)
    ps9.active(U9, 0)[8] = 0.0
    for prec in (0, 1):
        T8, T9 = A.Table(ps8, precision=prec), A.Table(ps9, precision=prec, ch=0.0)
        A.amr_table_set_tiling(T8.h, 1, 0)
        A.amr_table_set_tiling(T9.h, 1, 0)
        d8, d9 = T8.upload(U8), T9.upload(U9)
        for _ in range(3):
            dt = T8.cfl_dt(d8, 0.8)
            assert T9.cfl_dt(d9, 0.8) == dt
            T8.step(d8, dt=dt)
            T9.step(d9, dt=dt)
        g8, g9 = d8.cpu().numpy(), d9.cpu().numpy()
        T8.close()
        T9.close()
        assert np.array_equal(ps8.active(g8, 0), ps9.active(g9, 0)[:8]), prec
        assert not np.any(ps9.active(g9, 0)[8])


@pytest.mark.parametrize("shape", [1, 5])
def test_mixed_l1_and_conservation(env, shape):
    log(f"case glm mixed shape={shape}")
    N = 64
    ps, U = _glm_box(N, 32)
    A0 = active_all(ps, U)
    Ug, Uo = run_pair(env, ps, U, 10, 3.0, prec=1, shape=shape, periodic=7, domain=(N, N, N), check_dt=False)
    g, r = active_all(ps, Ug), active_all(ps, Uo)
    l1 = l1_rel(g, r)
    log(f"glm mixed shape={shape}: L1(rho) {l1:.2e}, L1(psi) {l1_rel(g, r, 8):.2e}")
    assert l1 <= 1e-5
    t0, t1 = totals(A0), totals(g)
    for k in range(9):
        scale = max(math.fsum(np.abs(A0[k])), math.fsum(np.abs(g[k])))
        assert abs(t1[k] - t0[k]) <= 1e-12 * scale, (k, t1[k] - t0[k])


def test_every_glm_tiling_gives_identical_bits(env):
    torch, A, O = env
    ps = W.make_patchset(3, [[40, 21, 18], [16, 16, 16]], 2, [W.BC_PERIODIC] * 6, gamma=5 / 3,
                         dx0=(0.02, 0.03, 0.025), nvar=9)
    U = W.random_state(ps, 64, shocks=1.0)
    for prec in (0, 1):
        ref = None
        T = A.Table(ps, precision=prec, exec_form=1, ch=3.0)
        for shape in range(1, A.amr_table_num_tilings(T.h)):
            if A.lib().amr_table_set_tiling(T.h, shape, 0) != A.AMR_OK:
                continue
            for z in (5, 64):
                log(f"case glm tiling prec={prec} shape={shape} zslab={z}")
                A.amr_table_set_tiling(T.h, shape, z)
                Ud = T.upload(U)
                for _ in range(2):
                    T.cfl_dt(Ud, 0.8)
                    T.step(Ud)
                out = active_all(ps, Ud.cpu().numpy())
                if ref is None:
                    ref = out
                else:
                    assert np.array_equal(out, ref), (prec, shape, z)
        T.close()
