"""GPU parity of the ideal-MHD update (8 conserved variables, the cleaning field at
zero): the HIP library through its C ABI against the FP64 CPU oracle on the same
seeded inputs.

Bars as for hydro: FP64 within 1e-12 of the oracle per cell and variable (the
FP64 kernels repeat the oracle's operations in its order, so cases are checked
bitwise where noted); mixed precision (FP32 reconstruction and flux): relative
L1 of density <= 1e-5 and totals of all eight variables conserved to 1e-12 on
periodic domains.
"""
import math

import numpy as np
import pytest

from paper_0910_5547_amd import workloads as W
from tests.gpu_util import active_all, l1_rel, log, rel_err, totals

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import oracle as O
    from paper_0910_5547_amd import amr as A
    A.lib()
    return torch, A, O


def run_pair(env, ps, U, steps, prec=0, exe=1, flux=0, cfl=0.8, periodic=0, domain=(0, 0, 0), shape=None,
             theta=None, check_dt=True):
    torch, A, O = env
    T = A.Table(ps, precision=prec, exec_form=exe, flux=flux, theta=theta, periodic=periodic, domain=domain)
    if shape is not None:
        A.amr_table_set_tiling(T.h, shape, 0)
    Ud = T.upload(U)
    o = O.Oracle(ps, flux=flux, theta=theta, periodic=periodic, domain=domain)
    Uo = U.copy()
    for s in range(steps):
        dt = T.cfl_dt(Ud, cfl)
        if check_dt:
            dto = o.cfl_dt(Uo, cfl)
            assert dt == dto, (s, dt, dto)
        T.step(Ud)
        assert o.rk2_step(Uo, dt) == 0
    torch.cuda.synchronize()
    assert T.status() == A.AMR_OK
    Ug = Ud.cpu().numpy()
    T.close()
    return Ug, Uo


def compare(ps, Ug, Uo, tol=TOL, bitwise=False, what=""):
    g, r = active_all(ps, Ug), active_all(ps, Uo)
    e = rel_err(g, r)
    log(f"{what}: max rel err per var {['%.2e' % x for x in e]}, bitwise={np.array_equal(g, r)}")
    assert max(e) <= tol, e
    if bitwise:
        assert np.array_equal(g, r)
    return e


def _random_mhd(n, bcs, seed, ndim=3, ng=2, gamma=5 / 3, shocks=1.0):
    dx0 = tuple(0.7 / n[0][d] if d < ndim else 1.0 for d in range(3))
    ps = W.make_patchset(ndim, n, ng, bcs, gamma=gamma, dx0=dx0, nvar=W.NVAR_MHD)
    return ps, W.random_state(ps, seed, shocks=shocks)


# ------------------------------------------------------------------ FP64
@pytest.mark.parametrize("exe", [0, 1])
def test_brio_wu_to_t01_fp64(env, exe):
    """Brio-Wu, N = 200, Gamma = 2, CFL 0.8, to t = 0.1: bitwise against the oracle."""
    torch, A, O = env
    log(f"case brio-wu exec={exe}")
    ps, U = W.brio_wu(200)
    T = A.Table(ps, precision=0, exec_form=exe)
    Ud = T.upload(U)
    o = O.Oracle(ps)
    Uo = U.copy()
    t, n = 0.0, 0
    while t < 0.1:
        dt = T.cfl_dt(Ud, 0.8)
        assert dt == o.cfl_dt(Uo, 0.8)
        if t + dt > 0.1:
            dt = 0.1 - t
        T.step(Ud, dt=dt)
        assert o.rk2_step(Uo, dt) == 0
        t += dt
        n += 1
    assert T.status() == A.AMR_OK
    Ug = Ud.cpu().numpy()
    T.close()
    assert n > 50
    compare(ps, Ug, Uo, bitwise=True, what=f"brio-wu exec={exe} steps={n}")


@pytest.mark.parametrize("shape", [1, 4, 7])
@pytest.mark.parametrize("bcs", [
    [W.BC_PERIODIC] * 6,
    [W.BC_REFLECT, W.BC_OUTFLOW, W.BC_PERIODIC, W.BC_PERIODIC, W.BC_OUTFLOW, W.BC_REFLECT],
    [W.BC_OUTFLOW, W.BC_REFLECT, W.BC_REFLECT, W.BC_OUTFLOW, W.BC_PERIODIC, W.BC_PERIODIC],
])
def test_ragged_3d_boundaries_fp64(env, bcs, shape):
    """Ragged sizes (not multiples of a tile), every on-the-fly boundary condition, planar shocks."""
    log(f"case mhd ragged bcs={bcs} shape={shape}")
    ps, U = _random_mhd([[37, 13, 11], [9, 26, 19]], bcs, seed=41)
    Ug, Uo = run_pair(env, ps, U, 3, shape=shape)
    compare(ps, Ug, Uo, bitwise=True, what=f"mhd ragged shape={shape}")


@pytest.mark.parametrize("shape", [1, 4, 7])
def test_two_dimensional_fp64(env, shape):
    log(f"case mhd 2d shape={shape}")
    ps, U = _random_mhd([[45, 29, 1]], [W.BC_PERIODIC, W.BC_PERIODIC, W.BC_REFLECT, W.BC_OUTFLOW, 0, 0],
                        seed=42, ndim=2)
    Ug, Uo = run_pair(env, ps, U, 4, shape=shape)
    compare(ps, Ug, Uo, bitwise=True, what=f"mhd 2d shape={shape}")


@pytest.mark.parametrize("exe", [0, 1])
def test_vortex_box_external_patches_fp64(env, exe):
    """The MHD vortex box (divergence-free random field) as 27 patches of 16^3 with EXTERNAL
    faces on a periodic root domain (sibling ghost copies of eight variables)."""
    log(f"case mhd vortex 48 exec={exe}")
    N = 48
    ps, U = W.mhd_vortex_box(N, patch=16, seed=50)
    Ug, Uo = run_pair(env, ps, U, 3, exe=exe, periodic=7, domain=(N, N, N))
    compare(ps, Ug, Uo, bitwise=True, what=f"mhd vortex48 exec={exe}")


def test_theta_and_hll2_fp64(env):
    log("case mhd theta 2 / hll2")
    ps, U = _random_mhd([[24, 20, 12]], [W.BC_PERIODIC] * 6, seed=43)
    Ug, Uo = run_pair(env, ps, U, 3, theta=2.0)
    compare(ps, Ug, Uo, bitwise=True, what="mhd theta=2")
    Ug, Uo = run_pair(env, ps, U, 3, flux=1)
    compare(ps, Ug, Uo, what="mhd hll2")


def test_zero_field_equals_hydro_library(env):
    """With B = 0 the MHD kernels give the hydro kernels' first five variables bit for bit."""
    torch, A, O = env
    log("case mhd zero field")
    n = [[30, 17, 12]]
    psh = W.make_patchset(3, n, 2, [W.BC_PERIODIC] * 6, gamma=5 / 3, dx0=(0.03, 0.05, 0.07))
    Uh = W.random_state(psh, 44, shocks=1.0)
    psm = W.make_patchset(3, n, 2, [W.BC_PERIODIC] * 6, gamma=5 / 3, dx0=(0.03, 0.05, 0.07), nvar=8)
    Um = W.new_arena(psm)
    psm.active(Um, 0)[:5] = psh.active(Uh, 0)
    psm.active(Um, 0)[5:] = 0.0
    for prec in (0, 1):
        Th, Tm = A.Table(psh, precision=prec), A.Table(psm, precision=prec)
        A.amr_table_set_tiling(Th.h, 1, 0)
        A.amr_table_set_tiling(Tm.h, 1, 0)
        dh, dm = Th.upload(Uh), Tm.upload(Um)
        for _ in range(3):
            dt = Th.cfl_dt(dh, 0.8)
            if prec == 0:
                assert Tm.cfl_dt(dm, 0.8) == dt
            Th.step(dh, dt=dt)
            Tm.step(dm, dt=dt)
        gh, gm = dh.cpu().numpy(), dm.cpu().numpy()
        Th.close()
        Tm.close()
        a, b = psh.active(gh, 0), psm.active(gm, 0)
        if prec == 0:
            assert np.array_equal(a, b[:5])
        else:
            assert l1_rel(a.reshape(5, -1), b[:5].reshape(5, -1)) <= 1e-6
        assert not np.any(b[5:])


# ------------------------------------------------------------------ mixed precision
@pytest.mark.parametrize("shape", [1, 4, 5, 6, 7])
def test_mixed_l1_and_conservation(env, shape):
    torch, A, O = env
    log(f"case mhd mixed shape={shape}")
    N = 64
    ps, U = W.mhd_vortex_box(N, patch=32, seed=50)
    A0 = active_all(ps, U)
    Ug, Uo = run_pair(env, ps, U, 10, prec=1, shape=shape, periodic=7, domain=(N, N, N), check_dt=False)
    g, r = active_all(ps, Ug), active_all(ps, Uo)
    l1 = l1_rel(g, r)
    log(f"mhd mixed shape={shape}: L1(rho) rel = {l1:.3e}, others {['%.1e' % l1_rel(g, r, k) for k in range(1, 8)]}")
    assert l1 <= 1e-5
    t0, t1 = totals(A0), totals(g)
    for k in range(8):
        # (rho v_z starts at exactly zero: its scale is the developed field's)
        scale = max(math.fsum(np.abs(A0[k])), math.fsum(np.abs(g[k])))
        assert abs(t1[k] - t0[k]) <= 1e-12 * scale, (k, t1[k] - t0[k])


def test_mixed_brio_wu(env):
    torch, A, O = env
    log("case mhd mixed brio-wu")
    ps, U = W.brio_wu(200)
    Ug, Uo = run_pair(env, ps, U, 60, prec=1, check_dt=False)
    l1 = l1_rel(active_all(ps, Ug), active_all(ps, Uo))
    log(f"mhd mixed brio-wu 60 steps: L1(rho) rel = {l1:.3e}")
    assert l1 <= 1e-5


@pytest.mark.parametrize("ndim", [3, 2])
def test_every_mhd_tiling_gives_identical_bits(env, ndim):
    """Face fluxes are computed once per face by the same code in every tile shape and z-slab
    (2D included: the single-barrier pass of the 32 x 16 tiles has its own 2D branch)."""
    torch, A, O = env
    if ndim == 3:
        ps, U = _random_mhd([[40, 21, 18], [16, 16, 16]], [W.BC_PERIODIC] * 6, seed=45)
    else:
        ps = W.make_patchset(2, [[45, 29, 1], [33, 17, 1]], 2, [W.BC_PERIODIC, W.BC_PERIODIC, W.BC_REFLECT,
                                                               W.BC_OUTFLOW, 0, 0], gamma=5 / 3,
                             dx0=(0.02, 0.03, 1.0), nvar=8)
        U = W.random_state(ps, 46, shocks=1.0)
    for prec in (0, 1):
        ref = None
        T = A.Table(ps, precision=prec, exec_form=1)
        for shape in range(1, A.amr_table_num_tilings(T.h)):
            if A.lib().amr_table_set_tiling(T.h, shape, 0) != A.AMR_OK:
                assert shape in ((2, 3, 5, 6) if prec == 0 else (2, 3))
                continue
            for z in (5, 64):
                log(f"case mhd tiling prec={prec} shape={shape} zslab={z}")
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


def test_fused_dt_equals_separate_reduction(env):
    torch, A, O = env
    log("case mhd fused dt")
    ps, U = _random_mhd([[32, 24, 16]], [W.BC_PERIODIC] * 6, seed=46)
    for prec in (0, 1):
        T = A.Table(ps, precision=prec)
        Ud = T.upload(U)
        T.cfl_dt(Ud, 0.8)
        for _ in range(3):
            A.amr_hydro_rk2_step(T.h, Ud, T.dt, -1, A.AMR_STEP_FUSE_DT)
            dt_f = A.amr_cfl_dt(T.h, Ud, 0.8, -1, T.dt, host=True)
            dt_s = A.amr_cfl_dt(T.h, Ud.clone(), 0.8, -1, T.dt, host=True)
            assert dt_f == dt_s
        T.close()


# ------------------------------------------------------------------ full size
def test_full_vortex_192_sampled_blocks(env):
    """The 192^3 MHD box as 216 patches of 32^3, one batched RK2 step in each precision;
    16^3 blocks (across patch boundaries and the periodic seam) are recomputed by the oracle
    on the block with a 4-cell halo (the step's domain of dependence)."""
    torch, A, O = env
    log("case mhd vortex192 sampled")
    N, P = 192, 32
    ps, U = W.mhd_vortex_box(N, patch=P, seed=50)
    full = np.empty((8, N, N, N))
    for p in range(ps.npatch):
        lo = ps.lo[p]
        full[:, lo[2]:lo[2] + P, lo[1]:lo[1] + P, lo[0]:lo[0] + P] = ps.active(U, p)
    for prec in (0, 1):
        T = A.Table(ps, precision=prec, exec_form=1, periodic=7, domain=(N, N, N))
        Ud = T.upload(U)
        dt = T.cfl_dt(Ud, 0.8)
        T.step(Ud)
        assert T.status() == A.AMR_OK
        Ug = Ud.cpu().numpy()
        T.close()
        rng = np.random.default_rng(3)
        corners = [(0, 0, 0), (24, 24, 24), (N - 8, N - 8, N - 8)] + [tuple(rng.integers(0, N, 3)) for _ in range(2)]
        for c in corners:
            B, H = 16, 4
            idx = [(np.arange(c[d] - H, c[d] + B + H) % N) for d in range(3)]
            blk = full[:, idx[2]][:, :, idx[1]][:, :, :, idx[0]]
            pb = W.make_patchset(3, [[B + 2 * H] * 3], 2, [W.BC_OUTFLOW] * 6, gamma=ps.gamma, dx0=ps.dx0, nvar=8)
            Ub = W.new_arena(pb)
            pb.active(Ub, 0)[...] = blk
            O.Oracle(pb).rk2_step(Ub, dt)
            ref = pb.active(Ub, 0)[:, H:H + B, H:H + B, H:H + B].reshape(8, -1)
            g = np.empty((8, B, B, B))
            for kz in range(B):
                for jy in range(B):
                    for ix in range(B):
                        x, y, z = idx[0][H + ix], idx[1][H + jy], idx[2][H + kz]
                        p = (z // P) * (N // P) ** 2 + (y // P) * (N // P) + x // P
                        g[:, kz, jy, ix] = ps.active(Ug, p)[:, z % P, y % P, x % P]
            g = g.reshape(8, -1)
            if prec == 0:
                e = rel_err(g, ref)
                log(f"vortex192 block {c}: {max(e):.2e}")
                assert max(e) <= TOL
            else:
                assert l1_rel(g, ref) <= 1e-5
