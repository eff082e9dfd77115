"""A dynamic hierarchy on the GPU: the uniform-grid blast (32^3 root) refined up to two
levels around its shock by the density-gradient flags, rebuilt every two root steps
(flags on the GPU, host clustering, regrid fill), advanced by subcycled root steps.

Checks: the finest level covers the shock sphere after the last rebuild, composite mass
and energy are conserved through steps and rebuilds (the blast does not reach the outflow
faces), and the shock radius on the root level follows the similarity law to within one
root cell."""
import math

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
    from paper_0910_5547_amd import dynamic as D
    A.lib()
    return torch, A, D


def test_blast_with_a_dynamic_hierarchy(env):
    torch, A, D = env
    N = 32
    ps, U, sol = W.sedov_uniform(N, t0=0.01)
    tot0 = W.composite_totals(ps, U)
    dh = D.DynamicHierarchy(ps, U, max_level=2, eps=0.3, every=2, t0=0.01, **W.SEDOV_FLOORS)
    dh.advance(0.014)
    ps2, U2 = dh.host_state()
    levels = np.bincount(ps2.level)
    log(f"steps {dh.steps}, rebuilds {dh.rebuilds}, patches per level {levels.tolist()}, t {dh.t:.5f}")
    assert dh.rebuilds >= 2 and len(levels) == 3 and levels[2] > 0
    tot = W.composite_totals(ps2, U2)
    scale = W.composite_totals(ps2, np.abs(U2))
    for k in (0, 4):
        assert abs(tot[k] - tot0[k]) <= 1e-12 * scale[k], (k, tot[k] - tot0[k])
    # the shock sphere lies on level 2 (level-2 index space: 4 N cells across the unit cube)
    rng = np.random.default_rng(0)
    R = sol.radius(1.0, dh.t)
    v = rng.standard_normal((200, 3))
    pts = 0.5 + R * v / np.linalg.norm(v, axis=1)[:, None]
    c = np.floor(pts * 4 * N).astype(int)
    fine = ps2.level == 2
    lo, hi = ps2.lo[fine], ps2.lo[fine] + ps2.n[fine]
    inside = [np.any(np.all((lo <= x) & (x < hi), axis=1)) for x in c]
    log(f"shock points on level 2: {np.mean(inside):.3f}")
    assert np.mean(inside) >= 0.99
    # the root level holds the restriction of the finer levels: its shock radius
    root = W.make_patchset(3, [[N] * 3], 2, [W.BC_OUTFLOW] * 6, dx0=ps.dx0)
    Ur = W.new_arena(root)
    Ur[...] = 0.0
    root.active(Ur, 0)[...] = ps2.active(U2, 0)
    Rm = W.shock_radius(root, Ur)
    log(f"root shock radius {Rm:.4f} exact {R:.4f}")
    assert abs(Rm - R) <= 1.0 / N
    dh.close()


@pytest.mark.parametrize("nvar,ch", [(8, 0.0), (9, 3.0)])
def test_magnetised_blast_with_a_dynamic_hierarchy(env, nvar, ch):
    """The MHD blast (weak uniform field, the paper's MHD Sedov set-up) on the same dynamic
    hierarchy: refined around the shock, every conserved total (B and psi included) kept
    through steps and rebuilds, the shock radius that of the hydro blast within a root cell."""
    torch, A, D = env
    N = 32
    ps, U, sol = W.sedov_uniform(N, t0=0.01, nvar=nvar, B0=0.01)
    tot0 = W.composite_totals(ps, U)
    dh = D.DynamicHierarchy(ps, U, max_level=2, eps=0.3, every=2, t0=0.01, ch=ch, **W.SEDOV_FLOORS)
    dh.advance(0.014)
    ps2, U2 = dh.host_state()
    levels = np.bincount(ps2.level)
    log(f"nvar {nvar}: steps {dh.steps}, rebuilds {dh.rebuilds}, patches per level {levels.tolist()}")
    assert dh.rebuilds >= 2 and len(levels) == 3 and levels[2] > 0
    tot = W.composite_totals(ps2, U2)
    scale = np.maximum(W.composite_totals(ps2, np.abs(U2)), W.composite_totals(ps, np.abs(U)))
    for k in range(nvar):
        assert abs(tot[k] - tot0[k]) <= 1e-12 * scale[k], (k, tot[k] - tot0[k])
    root = W.make_patchset(3, [[N] * 3], 2, [W.BC_OUTFLOW] * 6, dx0=ps.dx0, nvar=nvar)
    Ur = W.new_arena(root)
    Ur[...] = 0.0
    root.active(Ur, 0)[...] = ps2.active(U2, 0)
    R, Rm = sol.radius(1.0, dh.t), W.shock_radius(root, Ur)
    log(f"nvar {nvar}: root shock radius {Rm:.4f} exact (hydro) {R:.4f}")
    assert abs(Rm - R) <= 1.0 / N
    dh.close()
