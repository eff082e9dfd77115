"""GPU test of the allocation-free step (amr_patch_rk2_step_noalloc): its output
equals that of amr_hydro_rk2_step on a table of the same lone patch, bit for bit
(the same kernels), on two calls in a row, the second with a smaller patch, in
both precisions and for hydro and MHD; sizes beyond the scratch are refused."""
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


def _lone_patch(n, nvar, seed, bc):
    ps = W.make_patchset(3 if n[2] > 1 else (2 if n[1] > 1 else 1), [n], 3 if min(n[:2]) >= 3 else 2, bc,
                         gamma=5.0 / 3.0, dx0=(1.0 / 64,) * 3, nvar=nvar)
    ps.theta = 1.0
    U = W.random_state(ps, seed, amp=0.2, vamp=0.3, shocks=0.5)
    return ps, U


def _table_step(A, torch, ps, U, prec, dt):
    T = A.Table(ps, precision=prec)
    Ud = T.upload(U)
    T.step(Ud, dt=dt)
    torch.cuda.synchronize()
    assert T.status() == A.AMR_OK
    out = Ud.cpu().numpy()
    T.close()
    return out


CASES = [
    # (first patch, second smaller patch, nvar, bc)
    ((64, 48, 40), (24, 16, 8), 5, [W.BC_PERIODIC] * 6),
    ((96, 96, 64), (33, 17, 9), 5, [W.BC_OUTFLOW, W.BC_REFLECT, W.BC_PERIODIC, W.BC_PERIODIC, W.BC_REFLECT,
                                    W.BC_OUTFLOW]),
    ((40, 32, 24), (16, 8, 8), 8, [W.BC_PERIODIC] * 6),
    ((200, 1, 1), (37, 1, 1), 5, [W.BC_OUTFLOW] * 6),
    ((48, 40, 1), (12, 9, 1), 5, [W.BC_REFLECT] * 6),
]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_noalloc_step_equals_table_step_twice(env, prec, case):
    torch, A = env
    n1, n2, nvar, bc = CASES[case]
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    for n, seed in ((n1, 70 + case), (n2, 80 + case)):
        ps, U = _lone_patch(n, nvar, seed, bc)
        log(f"case noalloc n={n} nvar={nvar} prec={prec}")
        T = A.Table(ps, precision=prec)
        dt = T.cfl_dt(T.upload(U), 0.8)
        T.close()
        ref = _table_step(A, torch, ps, U, prec, dt)
        desc = A.descriptors(ps)[0]
        phys = A.physics(ps, precision=prec)
        Ud = torch.from_numpy(U).cuda()
        dtd = torch.full((1,), dt, dtype=torch.float64, device="cuda")
        A.amr_patch_rk2_step_noalloc(desc, phys, Ud, dtd, flag)
        torch.cuda.synchronize()
        got = Ud.cpu().numpy()
        assert int(flag.item()) == 0
        a, r = ps.active(got, 0), ps.active(ref, 0)
        assert np.array_equal(a, r), float(np.max(np.abs(a - r)))


def test_noalloc_refuses_oversize_and_external(env):
    torch, A = env
    ps, _ = W.uneven_patches(npatch=1, seed=30, with_state=False)
    phys = A.physics(ps)
    U = torch.zeros(8, dtype=torch.float64, device="cuda")
    dtd = torch.zeros(1, dtype=torch.float64, device="cuda")
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    big = A.descriptors(W.make_patchset(3, [(150, 150, 150)], 3, [W.BC_OUTFLOW] * 6))[0]
    with pytest.raises(A.AmrError) as ei:
        A.amr_patch_rk2_step_noalloc(big, phys, U, dtd, flag)
    assert ei.value.status == A.AMR_EINVAL
    ext = A.descriptors(W.make_patchset(3, [(16, 16, 16)], 3, [W.BC_EXTERNAL] * 6))[0]
    with pytest.raises(A.AmrError) as ei:
        A.amr_patch_rk2_step_noalloc(ext, phys, U, dtd, flag)
    assert ei.value.status == A.AMR_EINVAL


def test_noalloc_flags_an_unphysical_state(env):
    torch, A = env
    ps, U = _lone_patch((16, 16, 16), 5, 90, [W.BC_PERIODIC] * 6)
    ps.active(U, 0)[0, 3, 4, 5] = -1.0
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    Ud = torch.from_numpy(U).cuda()
    dtd = torch.full((1,), 1e-4, dtype=torch.float64, device="cuda")
    A.amr_patch_rk2_step_noalloc(A.descriptors(ps)[0], A.physics(ps), Ud, dtd, flag)
    torch.cuda.synchronize()
    assert int(flag.item()) != 0
