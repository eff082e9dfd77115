"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle
on the same seeded inputs.

Bars: plain and batched FP64 within 1e-12 of the oracle per cell and variable
(relative to the variable's largest magnitude); the FP64 kernels perform the
oracle's operations in the oracle's order, so most cases are expected to be
bitwise and are checked as such where noted.  Mixed precision (FP32
reconstruction and flux): relative L1 of density <= 1e-5 and totals conserved
to 1e-12.
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


def run_pair(env, ps, U, steps, prec=0, exe=1, flux=0, cfl=0.8, periodic=0, domain=(0, 0, 0), tiling=None,
             check_dt=True, theta=None):
    """Advance U on the GPU and with the oracle with identical dt (the GPU's); return both."""
    torch, A, O = env
    T = A.Table(ps, precision=prec, exec_form=exe, flux=flux, theta=theta, periodic=periodic, domain=domain)
    if tiling is not None:
        A.amr_table_set_tiling(T.h, *tiling)
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


# ------------------------------------------------------------------ configurations
@pytest.mark.parametrize("exe", [0, 1])
def test_sod_to_t02_fp64(env, exe):
    """Sod tube, 400 cells + 2 ghosts, CFL 0.8, outflow, to t = 0.2 (the 1D correctness config)."""
    torch, A, O = env
    log(f"case sod400 exec={exe}")
    ps, U = W.sod(400)
    T = A.Table(ps, precision=0, exec_form=exe)
    Ud = T.upload(U)
    o = O.Oracle(ps)
    Uo = U.copy()
    t, n = 0.0, 0
    while t < 0.2:
        dt = T.cfl_dt(Ud, 0.8)
        assert dt == o.cfl_dt(Uo, 0.8)
        if t + dt > 0.2:
            dt = 0.2 - t
        T.step(Ud, dt=dt)
        o.rk2_step(Uo, dt)
        t += dt
        n += 1
    assert T.status() == A.AMR_OK
    Ug = Ud.cpu().numpy()
    T.close()
    assert 150 <= n <= 250
    compare(ps, Ug, Uo, bitwise=True, what=f"sod400 exec={exe} steps={n}")


@pytest.mark.parametrize("N,steps", [(32, 20), (48, 5)])
def test_periodic_box_fp64(env, N, steps):
    log(f"case periodic box N={N}")
    ps, U = W.periodic_turbulent_box(N=N, seed=20, kmax=min(16.0, N / 4))
    Ug, Uo = run_pair(env, ps, U, steps)
    compare(ps, Ug, Uo, bitwise=True, what=f"box{N}")


@pytest.mark.parametrize("exe", [0, 1])
def test_uneven_patches_fp64(env, exe):
    log(f"case uneven patches exec={exe}")
    ps, U = W.uneven_patches(npatch=40, seed=31)
    Ug, Uo = run_pair(env, ps, U, 3, exe=exe)
    compare(ps, Ug, Uo, bitwise=True, what=f"uneven40 exec={exe}")


@pytest.mark.parametrize("bcs", [
    [W.BC_REFLECT, W.BC_OUTFLOW, W.BC_PERIODIC, W.BC_PERIODIC, W.BC_OUTFLOW, W.BC_REFLECT],
    [W.BC_OUTFLOW, W.BC_REFLECT, W.BC_REFLECT, W.BC_OUTFLOW, W.BC_PERIODIC, W.BC_PERIODIC],
])
def test_boundary_mix_ragged_3d(env, bcs):
    """Ragged sizes (not multiples of any tile) and every on-the-fly boundary condition."""
    log(f"case bc mix {bcs}")
    ps = W.make_patchset(3, [[37, 13, 11], [9, 26, 19]], 3, bcs, gamma=1.4, dx0=(0.03, 0.05, 0.04))
    U = W.random_state(ps, 7, shocks=1.0)
    Ug, Uo = run_pair(env, ps, U, 4)
    compare(ps, Ug, Uo, bitwise=True, what="bcmix")


@pytest.mark.parametrize("prec", [0, 1])
def test_patch_fit_tiles_on_ragged_widths(env, prec):
    """Patch-fit tiles (shape 7: width 8, 16 or 32 chosen per patch, height 256 / width) on
    widths below, at and between those sizes, with every on-the-fly boundary condition:
    FP64 bitwise against the oracle, mixed bitwise equal to the default tiling's."""
    torch, A, O = env
    bcs = [W.BC_REFLECT, W.BC_OUTFLOW, W.BC_PERIODIC, W.BC_PERIODIC, W.BC_OUTFLOW, W.BC_REFLECT]
    n = [[5, 40, 9], [8, 8, 8], [11, 33, 6], [16, 17, 12], [23, 9, 7], [32, 24, 10], [37, 70, 5]]
    ps = W.make_patchset(3, n, 3, bcs, gamma=5 / 3, dx0=(0.03, 0.05, 0.04))
    U = W.random_state(ps, 17, shocks=0.5)
    log(f"case patch-fit ragged prec={prec}")
    if prec == 0:
        Ug, Uo = run_pair(env, ps, U, 3, tiling=(7, 0))
        compare(ps, Ug, Uo, bitwise=True, what="patch-fit ragged")
    else:
        Ug, _ = run_pair(env, ps, U, 3, prec=1, tiling=(7, 0), check_dt=False)
        Ud, _ = run_pair(env, ps, U, 3, prec=1, check_dt=False)
        assert np.array_equal(active_all(ps, Ug), active_all(ps, Ud))


def test_two_dimensional(env):
    log("case 2d")
    ps = W.make_patchset(2, [[70, 45, 1]], 2, [W.BC_PERIODIC] * 2 + [W.BC_REFLECT] * 2 + [0, 0], gamma=5 / 3,
                         dx0=(1 / 70, 1 / 45, 1.0))
    U = W.random_state(ps, 8, shocks=1.0)
    Ug, Uo = run_pair(env, ps, U, 5)
    compare(ps, Ug, Uo, bitwise=True, what="2d")


@pytest.mark.parametrize("prec", [0, 1])
def test_two_dimensional_every_tiling(env, prec):
    """2D tables on every tile shape (the 32 x 16 tiles take the single-barrier face pass,
    whose 2D branch stages the plane ahead of its loop): FP64 bitwise against the oracle,
    mixed identical across shapes."""
    torch, A, O = env
    ps = W.make_patchset(2, [[70, 45, 1], [33, 17, 1]], 2, [W.BC_PERIODIC] * 2 + [W.BC_REFLECT] * 2 + [0, 0],
                         gamma=5 / 3, dx0=(1 / 70, 1 / 45, 1.0))
    U = W.random_state(ps, 9, shocks=1.0)
    T = A.Table(ps, precision=prec)
    shapes = [sh for sh in range(1, A.amr_table_num_tilings(T.h)) if A.lib().amr_table_set_tiling(T.h, sh, 0) == 0]
    T.close()
    assert 5 in shapes
    ref = None
    for sh in shapes:
        log(f"case 2d tiling prec={prec} shape={sh}")
        Ug, Uo = run_pair(env, ps, U, 3, prec=prec, tiling=(sh, 0), check_dt=prec == 0)
        if prec == 0:
            compare(ps, Ug, Uo, bitwise=True, what=f"2d shape {sh}")
        out = active_all(ps, Ug)
        if ref is None:
            ref = out
        else:
            assert np.array_equal(out, ref), sh


@pytest.mark.parametrize("shape", [None, 1, 4, 5, 7])
@pytest.mark.parametrize("bcs", [
    [W.BC_OUTFLOW] * 6,
    [W.BC_REFLECT, W.BC_OUTFLOW, W.BC_PERIODIC, W.BC_PERIODIC, W.BC_OUTFLOW, W.BC_REFLECT],
])
def test_smallest_patches(env, bcs, shape):
    """The smallest patches validation admits (n = ng = 2 in an active dimension) and near-minimal
    ragged ones, where almost every lane of a tile is idle: FP64 bitwise against the oracle in
    each tiling, the mixed path within 1e-5."""
    log(f"case smallest patches bcs={bcs} shape={shape}")
    ps = W.make_patchset(3, [[2, 2, 2], [2, 3, 4], [5, 2, 2], [3, 7, 2]], 2, bcs, gamma=5 / 3,
                         dx0=(0.05, 0.04, 0.06))
    U = W.random_state(ps, 12, shocks=1.0)
    tiling = None if shape is None else (shape, 0)
    Ug, Uo = run_pair(env, ps, U, 4, tiling=tiling)
    compare(ps, Ug, Uo, bitwise=True, what=f"smallest shape {shape}")
    Ug, Uo = run_pair(env, ps, U, 4, prec=1, tiling=tiling, check_dt=False)
    assert l1_rel(active_all(ps, Ug), active_all(ps, Uo)) <= 1e-5


@pytest.mark.parametrize("prec,shape", [(0, None), (0, 5), (1, 5)])
def test_patch_stored_beyond_2_31_elements(env, prec, shape):
    """A patch whose storage starts past element 2^31 of the arena (17 GB of FP64): every index
    of the stage, CFL and tile code is 64-bit.  FP64 bitwise against the oracle on a compact copy of
    the same patches; mixed within 1e-5."""
    import dataclasses
    torch, A, O = env
    ps = W.make_patchset(3, [[24, 20, 18], [20, 16, 12]], 2, [W.BC_PERIODIC] * 6, gamma=5 / 3,
                         dx0=(0.04, 0.05, 0.055))
    U = W.random_state(ps, 11, shocks=1.0)
    far = (2 ** 31 + 4096) // 64 * 64
    size1 = int(ps.arena - ps.offset[1])
    big = dataclasses.replace(ps, offset=np.array([0, far], np.int64), arena=far + size1)
    log(f"case far patch prec={prec} shape={shape} arena {big.arena}")
    T = A.Table(big, precision=prec)
    if shape is not None:
        assert A.lib().amr_table_set_tiling(T.h, shape, 0) == A.AMR_OK
    Ud = torch.empty(T.arena, dtype=torch.float64, device="cuda")
    Ud[:int(ps.offset[1])] = torch.from_numpy(U[:int(ps.offset[1])]).cuda()
    Ud[far:far + size1] = torch.from_numpy(U[int(ps.offset[1]):]).cuda()
    o = O.Oracle(ps)
    Uo = U.copy()
    for s in range(3):
        dt = T.cfl_dt(Ud, 0.8)
        if prec == 0:
            assert dt == o.cfl_dt(Uo, 0.8), s
        T.step(Ud)
        assert o.rk2_step(Uo, dt) == 0
    torch.cuda.synchronize()
    assert T.status() == A.AMR_OK
    Ug = np.concatenate([Ud[:int(ps.offset[1])].cpu().numpy(), Ud[far:far + size1].cpu().numpy()])
    T.close()
    del Ud
    torch.cuda.empty_cache()
    if prec == 0:
        compare(ps, Ug, Uo, bitwise=True, what=f"far patch shape {shape}")
    else:
        assert l1_rel(active_all(ps, Ug), active_all(ps, Uo)) <= 1e-5


@pytest.mark.parametrize("theta", [0.0, 0.5, 2.0])
def test_limiter_theta(env, theta):
    """theta != 1: the three-argument minmod path of the stage kernel (theta = 1 compiles to
    the two-argument form), bitwise against the oracle in FP64 and to 1e-5 in mixed."""
    log(f"case theta {theta}")
    ps, U = W.uneven_patches(npatch=8, seed=36)
    Ug, Uo = run_pair(env, ps, U, 3, theta=theta)
    compare(ps, Ug, Uo, bitwise=True, what=f"theta {theta}")
    Ug, Uo = run_pair(env, ps, U, 3, prec=1, theta=theta, check_dt=False)
    g, r = active_all(ps, Ug), active_all(ps, Uo)
    assert l1_rel(g, r) <= 1e-5


def test_hll2_flux(env):
    log("case hll2")
    ps, U = W.uneven_patches(npatch=8, seed=33)
    Ug, Uo = run_pair(env, ps, U, 2, flux=1)
    compare(ps, Ug, Uo, what="hll2")


def test_external_sibling_ghosts(env):
    """The periodic box cut into 8 patches with EXTERNAL faces equals the oracle's sibling fill."""
    log("case external siblings")
    N = 24
    ps, U = W.periodic_turbulent_box(N=N, seed=5, kmax=4.0, patch=12)
    Ug, Uo = run_pair(env, ps, U, 3, periodic=7, domain=(N, N, N))
    compare(ps, Ug, Uo, bitwise=True, what="external")


# ------------------------------------------------------------------ forms and tilings
def test_every_tiling_gives_identical_bits(env):
    """Each face flux is computed once per tile, by the same code: the result cannot depend
    on tile shape or z-slab length, in either precision."""
    torch, A, O = env
    ps = W.make_patchset(3, [[40, 21, 18], [16, 16, 16]], 2, [W.BC_PERIODIC] * 6, gamma=5 / 3,
                         dx0=(0.02, 0.03, 0.025))
    U = W.random_state(ps, 12, shocks=1.0)
    for prec in (0, 1):
        ref = None
        T = A.Table(ps, precision=prec, exec_form=1)
        for shape in range(1, A.amr_table_num_tilings(T.h)):
            for z in (4, 7, 64):
                log(f"case tiling prec={prec} shape={shape} zslab={z}")
                A.amr_table_set_tiling(T.h, shape, z)
                Ud = T.upload(U)
                for _ in range(2):
                    T.cfl_dt(Ud, 0.8)
                    T.step(Ud)
                out = Ud.cpu().numpy()
                if ref is None:
                    ref = out
                else:
                    assert np.array_equal(active_all(ps, out), active_all(ps, ref)), (prec, shape, z)
        T.close()


def test_batched_graph_replays_equal_plain(env):
    """Captured-graph replays with dt changing between steps equal the plain per-patch form bitwise."""
    torch, A, O = env
    log("case graph vs plain")
    ps, U = W.uneven_patches(npatch=30, seed=34)
    Tp = A.Table(ps, exec_form=0)
    Tb = A.Table(ps, exec_form=1)
    Up, Ub = Tp.upload(U), Tb.upload(U)
    for s in range(6):
        dt = Tp.cfl_dt(Up, 0.8)
        assert Tb.cfl_dt(Ub, 0.8) == dt
        Tp.step(Up)
        Tb.step(Ub)
        torch.cuda.synchronize()
        assert torch.equal(Up, Ub) or np.array_equal(active_all(ps, Up.cpu().numpy()),
                                                     active_all(ps, Ub.cpu().numpy())), s
    Tp.close()
    Tb.close()


def test_fused_dt_equals_separate_reduction(env):
    torch, A, O = env
    log("case fused dt")
    ps, U = W.periodic_turbulent_box(N=32, seed=21, kmax=8.0)
    T = A.Table(ps)
    Ud = T.upload(U)
    Uf = Ud.clone()
    T.cfl_dt(Ud, 0.8)
    for _ in range(3):
        A.amr_hydro_rk2_step(T.h, Uf, T.dt, -1, A.AMR_STEP_FUSE_DT)
        dt_f = A.amr_cfl_dt(T.h, Uf, 0.8, -1, T.dt, host=True)
        # the same state scanned separately (a different pointer, so no fused value)
        Uc = Uf.clone()
        dt_s = A.amr_cfl_dt(T.h, Uc, 0.8, -1, T.dt, host=True)
        assert dt_f == dt_s
    T.close()


# ------------------------------------------------------------------ mixed precision
@pytest.mark.parametrize("exe", [0, 1])
def test_mixed_precision_l1_and_conservation(env, exe):
    torch, A, O = env
    log(f"case mixed exec={exe}")
    ps, U = W.periodic_turbulent_box(N=32, seed=20, kmax=8.0)
    A0 = active_all(ps, U)
    Ug, Uo = run_pair(env, ps, U, 10, prec=1, exe=exe, check_dt=False)
    g, r = active_all(ps, Ug), active_all(ps, Uo)
    l1 = l1_rel(g, r)
    log(f"mixed exec={exe}: L1(rho) rel = {l1:.3e}, L1 others {[l1_rel(g, r, k) for k in (1, 2, 3, 4)]}")
    assert l1 <= 1e-5
    t0, t1 = totals(A0), totals(g)
    for k in range(5):
        scale = math.fsum(np.abs(A0[k]))
        assert abs(t1[k] - t0[k]) <= 1e-12 * scale, (k, t1[k] - t0[k])


def test_mixed_uneven_patches_with_shocks(env):
    log("case mixed uneven")
    ps, U = W.uneven_patches(npatch=40, seed=35)
    Ug, Uo = run_pair(env, ps, U, 3, prec=1, check_dt=False)
    g, r = active_all(ps, Ug), active_all(ps, Uo)
    l1 = l1_rel(g, r)
    log(f"mixed uneven: L1(rho) rel = {l1:.3e}")
    assert l1 <= 1e-5


# ------------------------------------------------------------------ failure reporting
def test_unphysical_state_is_reported(env):
    torch, A, O = env
    log("case unphysical")
    ps, U = W.uneven_patches(npatch=4, seed=36)
    T = A.Table(ps)
    Ud = T.upload(U)
    T.cfl_dt(Ud, 0.8)
    T.step(Ud)
    assert T.status() == A.AMR_OK
    U2 = U.copy()
    ps.active(U2, 2)[4, 1, 2, 3] = -5.0  # negative total energy in one cell
    Ud2 = T.upload(U2)
    with pytest.raises(A.AmrError) as ei:
        T.cfl_dt(Ud2, 0.8)
    assert ei.value.status == A.AMR_EUNPHYSICAL
    T.step(Ud2)
    assert T.status() == A.AMR_EUNPHYSICAL
    assert T.status() == A.AMR_OK  # latch cleared
    # patches that do not touch the bad cell are unaffected
    Ud3 = T.upload(U)
    T.step(Ud3)
    a2, a3 = Ud2.cpu().numpy(), Ud3.cpu().numpy()
    for p in (0, 1, 3):
        assert np.array_equal(ps.active(a2, p), ps.active(a3, p))
    T.close()


# ------------------------------------------------------------------ full-size checks
def test_full_box_256_sampled_blocks(env):
    """256^3 periodic box, one RK2 step in the benchmark's launch form (batched); sampled
    16^3 blocks (some across the periodic seam) are recomputed by the oracle on a block
    with a 4-cell halo (the step's domain of dependence) and must agree."""
    torch, A, O = env
    log("case box256 sampled")
    N = 256
    ps, U = W.periodic_turbulent_box(N=N, seed=20)
    for prec in (0, 1):
        T = A.Table(ps, precision=prec, exec_form=1)
        Ud = T.upload(U)
        dt = T.cfl_dt(Ud, 0.8)
        T.step(Ud)
        assert T.status() == A.AMR_OK
        Ug = Ud.cpu().numpy()
        T.close()
        full = ps.active(U, 0)
        got = ps.active(Ug, 0)
        rng = np.random.default_rng(1)
        corners = [(0, 0, 0), (N - 8, N - 8, N - 8)] + [tuple(rng.integers(0, N, 3)) for _ in range(2)]
        for c in corners:
            B, H = 16, 4
            idx = [(np.arange(c[d] - H, c[d] + B + H) % N) for d in range(3)]
            blk = full[:, idx[2]][:, :, idx[1]][:, :, :, idx[0]]
            pb = W.make_patchset(3, [[B + 2 * H] * 3], 2, [W.BC_OUTFLOW] * 6, gamma=ps.gamma, dx0=ps.dx0)
            Ub = W.new_arena(pb)
            pb.active(Ub, 0)[...] = blk
            o = O.Oracle(pb)
            o.rk2_step(Ub, dt)
            ref = pb.active(Ub, 0)[:, H:H + B, H:H + B, H:H + B]
            g = got[:, idx[2][H:H + B]][:, :, idx[1][H:H + B]][:, :, :, idx[0][H:H + B]]
            if prec == 0:
                e = rel_err(g.reshape(5, -1), ref.reshape(5, -1))
                log(f"box256 block {c}: {e}")
                assert max(e) <= TOL
            else:
                l1 = l1_rel(g.reshape(5, -1), ref.reshape(5, -1))
                assert l1 <= 1e-5, l1


def test_full_uneven_4000_sampled_patches(env):
    """4000 uneven patches (seed 30), one batched RK2 step; 25 patches recomputed by the oracle."""
    torch, A, O = env
    log("case uneven4000 sampled")
    ps, U = W.uneven_patches(npatch=4000, seed=30)
    rng = np.random.default_rng(2)
    pick = rng.choice(ps.npatch, 25, replace=False)
    for prec in (0, 1):
        T = A.Table(ps, precision=prec, exec_form=1)
        Ud = T.upload(U)
        dt = T.cfl_dt(Ud, 0.8)
        T.step(Ud)
        assert T.status() == A.AMR_OK
        Ug = Ud.cpu().numpy()
        T.close()
        for p in pick:
            pb = W.make_patchset(3, [ps.n[p]], int(ps.ng[p]), [W.BC_OUTFLOW] * 6, gamma=ps.gamma, dx0=ps.dx0)
            Ub = W.new_arena(pb)
            pb.active(Ub, 0)[...] = ps.active(U, p)
            O.Oracle(pb).rk2_step(Ub, dt)
            g, r = ps.active(Ug, p).reshape(5, -1), pb.active(Ub, 0).reshape(5, -1)
            if prec == 0:
                assert np.array_equal(g, r) or max(rel_err(g, r)) <= TOL, p
            else:
                assert l1_rel(g, r) <= 1e-5, p
