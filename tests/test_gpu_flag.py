"""GPU refinement flags (amr_flag_cells) against the oracle's: bit-exact, one byte per
active cell, on single-level tables (every boundary condition, direct sibling faces) and on
hierarchies (ghosts prolonged from the coarse level)."""
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
    from oracle import oracle as O
    from paper_0910_5547_amd import amr as A
    A.lib()
    return torch, A, O


def _gpu_flags(env, T, Ud, level, eps):
    torch, A, O = env
    n = A.amr_table_cells(T.h, level)
    f = torch.zeros(n, dtype=torch.uint8, device="cuda")
    A.amr_flag_cells(T.h, Ud, level, eps, f)
    torch.cuda.synchronize()
    return f.cpu().numpy()


@pytest.mark.parametrize("case", ["uneven", "ragged_bcs", "siblings"])
def test_single_level_flags_match_oracle(env, case):
    torch, A, O = env
    log(f"case flags {case}")
    kw = {}
    if case == "uneven":
        ps, U = W.uneven_patches(npatch=30, seed=37)
    elif case == "ragged_bcs":
        bcs = [W.BC_REFLECT, W.BC_OUTFLOW, W.BC_PERIODIC, W.BC_PERIODIC, W.BC_OUTFLOW, W.BC_REFLECT]
        ps = W.make_patchset(3, [[37, 13, 11], [9, 26, 19]], 3, bcs, gamma=1.4, dx0=(0.03, 0.05, 0.04))
        U = W.random_state(ps, 15, shocks=1.0)
    else:
        ps, U = W.periodic_turbulent_box(N=48, seed=5, kmax=8.0, patch=16)
        kw = dict(periodic=7, domain=(48, 48, 48))
    T = A.Table(ps, **kw)
    Ud = T.upload(U)
    o = O.Oracle(ps, **kw)
    for eps in (0.02, 0.1, 0.3):
        g = _gpu_flags(env, T, Ud, -1, eps)
        r = o.flag_cells(U.copy(), eps)
        log(f"{case} eps={eps}: {int(r.sum())} flagged of {r.size}")
        assert np.array_equal(g, r), (eps, int((g != r).sum()))
    T.close()


def test_hierarchy_flags_match_oracle(env):
    torch, A, O = env
    log("case flags hierarchy")
    ps, U, per, dom = W.two_level_box(Nc=16, fine_lo=(4, 6, 4), fine_n=(8, 6, 8), coarse_split=2, seed=51)
    T = A.Table(ps, periodic=per, domain=dom)
    Ud = T.upload(U)
    o = O.AmrOracle(ps, periodic=per, domain=dom)
    for level in (0, 1):
        g = _gpu_flags(env, T, Ud, level, 0.05)
        r = o.flag_cells(U.copy(), 0.05, level)
        assert g.size == r.size and np.array_equal(g, r), level
    T.close()
    ps, U, _, _ = W.sedov_hierarchy(levels=2)
    T = A.Table(ps, **W.SEDOV_FLOORS)
    Ud = T.upload(U)
    o = O.AmrOracle(ps, **W.SEDOV_FLOORS)
    for level in (0, 1, 2):
        g = _gpu_flags(env, T, Ud, level, 0.3)
        r = o.flag_cells(U.copy(), 0.3, level)
        log(f"sedov level {level}: {int(r.sum())} flagged of {r.size}")
        assert np.array_equal(g, r), level
    T.close()
