"""GPU parity of ghost-free storage (ng = 0: patches that store no ghost layers, their faces
applied by index maps or read directly from a same-shaped sibling): the same bits as the
oracle run on a copy of the state that stores three ghost layers (FP64), and as the library
on that copy (mixed), for uneven patches with every on-the-fly boundary condition, a
periodic box cut into patches with EXTERNAL faces, the MHD vortex box, the allocation-free
step and the refinement flags."""
import numpy as np
import pytest

from paper_0910_5547_amd import workloads as W
from tests.gpu_util import active_all, log, rel_err

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


def with_ghosts(ps, U, ng=3):
    """The same patches storing ng ghost layers per side, active cells copied."""
    q = W.make_patchset(ps.ndim, ps.n, ng, ps.bc, level=ps.level, lo=ps.lo, gamma=ps.gamma, theta=ps.theta,
                        dx0=ps.dx0, nvar=ps.nvar)
    V = W.new_arena(q)
    for p in range(ps.npatch):
        q.active(V, p)[...] = ps.active(U, p)
    return q, V


def gpu_steps(env, ps, U, steps, prec, kw=None, dts=None):
    torch, A, O = env
    T = A.Table(ps, precision=prec, **(kw or {}))
    Ud = T.upload(U)
    out = []
    for s in range(steps):
        if dts is None:
            out.append(T.cfl_dt(Ud, 0.8))
        else:
            T.dt.fill_(dts[s])
            out.append(dts[s])
        T.step(Ud)
    torch.cuda.synchronize()
    assert T.status() == A.AMR_OK
    Ug = Ud.cpu().numpy()
    T.close()
    return active_all(ps, Ug), out


def check(env, ps0, U0, steps, kw=None, okw=None):
    torch, A, O = env
    ps3, U3 = with_ghosts(ps0, U0)
    g, dts = gpu_steps(env, ps0, U0, steps, 0, kw)
    o = O.Oracle(ps3, **(okw or {}))
    Uo = U3.copy()
    for dt in dts:
        assert o.rk2_step(Uo, dt) == 0
    r = active_all(ps3, Uo)
    e = rel_err(g, r)
    log(f"ghost-free fp64: max rel err {max(e):.1e}, bitwise={np.array_equal(g, r)}")
    assert np.array_equal(g, r)
    gm, dtm = gpu_steps(env, ps0, U0, steps, 1, kw)
    rm, _ = gpu_steps(env, ps3, U3, steps, 1, kw, dts=dtm)
    assert np.array_equal(gm, rm)


def test_uneven_patches_without_ghost_storage(env):
    log("case ghost-free uneven")
    bcs = [W.BC_REFLECT, W.BC_OUTFLOW, W.BC_PERIODIC, W.BC_PERIODIC, W.BC_OUTFLOW, W.BC_REFLECT]
    ps, _ = W.uneven_patches(npatch=40, seed=36, with_state=False)
    ps0 = W.make_patchset(3, ps.n, 0, bcs, gamma=ps.gamma, dx0=ps.dx0)
    U0 = W.random_state(ps0, 37, amp=0.2, vamp=0.3, shocks=0.3)
    check(env, ps0, U0, 3)


def test_periodic_box_patches_read_siblings_directly(env):
    log("case ghost-free box patches")
    ps0, U0 = W.periodic_turbulent_box(N=48, seed=21, kmax=8.0, patch=16, ng=0)
    kw = dict(periodic=7, domain=(48, 48, 48))
    check(env, ps0, U0, 3, kw, kw)


def test_mhd_vortex_box_without_ghost_storage(env):
    log("case ghost-free mhd")
    ps0, U0 = W.mhd_vortex_box(N=64, patch=32, seed=50, ng=0)
    kw = dict(periodic=7, domain=(64, 64, 64))
    check(env, ps0, U0, 2, kw, kw)


def test_noalloc_step_on_ghost_free_patch(env):
    torch, A, O = env
    ps0 = W.make_patchset(3, [[24, 16, 40]], 0, [W.BC_PERIODIC] * 2 + [W.BC_REFLECT] * 2 + [W.BC_OUTFLOW] * 2,
                          gamma=5 / 3, dx0=(0.02,) * 3)
    U0 = W.random_state(ps0, 38, shocks=1.0)
    for prec in (0, 1):
        g, dts = gpu_steps(env, ps0, U0, 1, prec)
        Ud = torch.from_numpy(U0).cuda()
        flag = torch.zeros(1, dtype=torch.int32, device="cuda")
        dtd = torch.full((1,), dts[0], dtype=torch.float64, device="cuda")
        A.amr_patch_rk2_step_noalloc(A.descriptors(ps0)[0], A.physics(ps0, precision=prec), Ud, dtd, flag)
        torch.cuda.synchronize()
        assert int(flag.item()) == 0
        assert np.array_equal(active_all(ps0, Ud.cpu().numpy()), g)


def test_flags_on_ghost_free_siblings(env):
    torch, A, O = env
    ps0, U0 = W.periodic_turbulent_box(N=32, seed=22, kmax=8.0, patch=16, ng=0)
    kw = dict(periodic=7, domain=(32, 32, 32))
    ps3, U3 = with_ghosts(ps0, U0)
    T = A.Table(ps0, **kw)
    Ud = T.upload(U0)
    fl = torch.zeros(A.amr_table_cells(T.h, -1), dtype=torch.uint8, device="cuda")
    A.amr_flag_cells(T.h, Ud, -1, 0.05, fl)
    torch.cuda.synchronize()
    got = fl.cpu().numpy()
    T.close()
    ref = O.Oracle(ps3, **kw).flag_cells(U3.copy(), 0.05)
    assert got.sum() > 0 and np.array_equal(got, ref)
