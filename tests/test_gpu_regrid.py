"""GPU regridding (amr_regrid_fill): a new hierarchy's cells taken from the old hierarchy
where it holds them and prolonged from the new coarse level elsewhere.  Checked against what
the operation fixes: copied cells equal the old cells bit for bit, prolonged children
average to their coarse parent, a linear field is reproduced exactly, and the composite
totals are unchanged."""
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


def _fill(env, psA, UA, psB, kw=None):
    torch, A = env
    kw = kw or {}
    TA, TB = A.Table(psA, **kw), A.Table(psB, **kw)
    dA = TA.upload(UA)
    dB = TB.upload(W.new_arena(psB))
    A.amr_regrid_fill(TA.h, dA, TB.h, dB)
    torch.cuda.synchronize()
    out = dB.cpu().numpy()
    TA.close()
    TB.close()
    return out


def test_linear_field_is_prolonged_exactly(env):
    log("case regrid linear")
    Nc = 16
    psA = W.make_patchset(3, [[Nc] * 3], 2, [W.BC_OUTFLOW] * 6, dx0=(1 / Nc,) * 3)
    x = (np.arange(Nc) + 0.5) / Nc
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    UA = W.new_arena(psA)
    psA.active(UA, 0)[...] = W.conserved(1 + 0.2 * X + 0.1 * Y - 0.3 * Z, 0.1 * X, 0.0, -0.2 * Y, 1 + 0.1 * Z, 1.4)
    bc1 = [W.BC_EXTERNAL] * 6
    psB = W.make_patchset(3, [[Nc] * 3, [12, 8, 16]], 2, [[W.BC_OUTFLOW] * 6, bc1], level=[0, 1],
                          lo=[[0, 0, 0], [8, 10, 6]], dx0=(1 / Nc,) * 3)
    UB = _fill(env, psA, UA, psB)
    assert np.array_equal(psB.active(UB, 0), psA.active(UA, 0))
    f = psB.active(UB, 1)
    xf = [(np.arange(psB.n[1][d]) + psB.lo[1][d] + 0.5) / (2 * Nc) for d in range(3)]
    Zf, Yf, Xf = np.meshgrid(xf[2], xf[1], xf[0], indexing="ij")
    rho = 1 + 0.2 * Xf + 0.1 * Yf - 0.3 * Zf
    assert np.max(np.abs(f[0] - rho)) <= 1e-14
    # the momenta and energy are linear too (momentum rho v is quadratic: compare their parents)
    c = psA.active(UA, 0)
    for k in range(5):
        kids = f[k].reshape(8, 2, 4, 2, 6, 2).mean(axis=(1, 3, 5))
        par = c[k][3:11, 5:9, 4:10]
        assert np.max(np.abs(kids - par)) <= 1e-14 * max(1.0, np.abs(par).max()), k


@pytest.mark.parametrize("nvar", [5, 8, 9])
def test_regrid_copies_old_fine_cells_and_conserves(env, nvar):
    torch, A = env
    log(f"case regrid two-level nvar={nvar}")
    psA, UA, per, dom = W.two_level_box(Nc=16, fine_lo=(4, 6, 4), fine_n=(8, 6, 8), coarse_split=2, seed=51,
                                        nvar=nvar)
    # the same root patches with a larger fine patch that overlaps the old one
    root = [p for p in range(psA.npatch) if psA.level[p] == 0]
    fine_lo, fine_n = np.array([6, 8, 4]), np.array([12, 10, 12])
    n = [list(psA.n[p]) for p in root] + [list(fine_n)]
    lo = [list(psA.lo[p]) for p in root] + [list(fine_lo)]
    bc = [list(psA.bc[p]) for p in root] + [[W.BC_EXTERNAL] * 6]
    psB = W.make_patchset(3, n, int(psA.ng[0]), bc, level=[0] * len(root) + [1], lo=lo, gamma=psA.gamma,
                          dx0=psA.dx0, nvar=nvar)
    kw = dict(periodic=per, domain=dom, ch=1.0 if nvar == 9 else 0.0)
    UB = _fill(env, psA, UA, psB, kw)
    for i, p in enumerate(root):
        assert np.array_equal(psB.active(UB, i), psA.active(UA, p))
    fA = [p for p in range(psA.npatch) if psA.level[p] == 1][0]
    a, b = psA.active(UA, fA), psB.active(UB, len(root))
    loA, loB = psA.lo[fA], fine_lo
    ov_lo, ov_hi = np.maximum(loA, loB), np.minimum(loA + psA.n[fA], loB + fine_n)
    sa = tuple(slice(ov_lo[d] - loA[d], ov_hi[d] - loA[d]) for d in (2, 1, 0))
    sb = tuple(slice(ov_lo[d] - loB[d], ov_hi[d] - loB[d]) for d in (2, 1, 0))
    assert np.array_equal(b[(slice(None),) + sb], a[(slice(None),) + sa])
    tA, tB = W.composite_totals(psA, UA), W.composite_totals(psB, UB)
    scale = W.composite_totals(psA, np.abs(UA))
    assert np.all(np.abs(tB - tA) <= 1e-13 * scale), (tB - tA) / scale


@pytest.mark.parametrize("nvar", [5, 8, 9])
def test_regrid_matches_the_oracle_cell_by_cell(env, nvar):
    """A three-level hierarchy on a nonlinear periodic field rebuilt with moved level-1 and
    level-2 patches: every new active cell (copied where an old patch of its level holds
    it, else prolonged from the new level below, itself partly prolonged) equals the
    oracle's regrid of the same hierarchies."""
    from oracle import oracle as O
    from tests.gpu_util import active_all, rel_err
    torch, A = env
    log(f"case regrid vs oracle nvar={nvar}")
    psA, UA, per, dom = W.nested_box(Nc=16, boxes=((4, 12), (14, 20)), seed=55, nvar=nvar)
    # new level 1 over root cells [6, 14), new level 2 over its cells [15, 23): overlapping the
    # old patches of their levels and sticking out of them
    n = [list(psA.n[0]), [16, 16, 16], [16, 16, 16]]
    lo = [list(psA.lo[0]), [12, 12, 12], [30, 30, 30]]
    psB = W.make_patchset(3, n, int(psA.ng[0]), [W.BC_EXTERNAL] * 6, level=[0, 1, 2], lo=lo, gamma=psA.gamma,
                          dx0=psA.dx0, nvar=nvar)
    ch = 1.0 if nvar == 9 else 0.0
    UB = _fill(env, psA, UA, psB, dict(periodic=per, domain=dom, ch=ch))
    Uo = W.new_arena(psB)
    missing = O.AmrOracle(psB, periodic=per, domain=dom, ch=ch).regrid_fill(psA, UA, Uo)
    assert missing == 0
    g, r = active_all(psB, UB), active_all(psB, Uo)
    e = rel_err(g, r)
    log(f"regrid nvar={nvar}: max rel err {max(e):.1e}, bitwise={np.array_equal(g, r)}")
    assert max(e) <= 1e-14
