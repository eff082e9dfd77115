"""Pins of the oracle's regrid fill (a hierarchy rebuilt: every new cell copied from an old
patch of its level, else prolonged from the new level below), against what the rebuild rule
and the conservative prolongation fix: copied cells equal the old cells bit for bit, a linear
field is reproduced exactly on every new level (also through a level that was itself
prolonged), the 2^d children of a coarse cell average to it, and a new root that no old root
covers is reported."""
import numpy as np

from paper_0910_5547_amd import workloads as W

NC = 16


def _linear(ps, p, coef=(0.2, 0.1, -0.3), nvar=5):
    """Conserved state of a field linear in the position (density, velocity, pressure)."""
    lvl = int(ps.level[p])
    x = [(np.arange(int(ps.n[p, d])) + int(ps.lo[p, d]) + 0.5) / (NC << lvl) for d in range(3)]
    Z, Y, X = np.meshgrid(x[2], x[1], x[0], indexing="ij")
    rho = 1.0 + coef[0] * X + coef[1] * Y + coef[2] * Z
    return X, Y, Z, rho


def _root_only(nvar=5):
    ps = W.make_patchset(3, [[NC] * 3], 2, [W.BC_OUTFLOW] * 6, dx0=(1 / NC,) * 3, nvar=nvar)
    U = W.new_arena(ps)
    return ps, U


def _hier(boxes, nvar=5):
    """Root NC^3 plus patches (level, lo, n) with EXTERNAL faces."""
    n = [[NC] * 3] + [b[2] for b in boxes]
    lo = [[0, 0, 0]] + [b[1] for b in boxes]
    lv = [0] + [b[0] for b in boxes]
    bc = [[W.BC_OUTFLOW] * 6] + [[W.BC_EXTERNAL] * 6 for _ in boxes]
    return W.make_patchset(3, n, 2, bc, level=lv, lo=lo, dx0=(1 / NC,) * 3, nvar=nvar)


def _fill_linear_root(ps, U):
    X, Y, Z, rho = _linear(ps, 0)
    # density linear; velocity and pressure constant, so every conserved variable is linear
    ps.active(U, 0)[...] = W.conserved(rho, 0.3, -0.2, 0.1, 1.0 + 0 * X, 1.4)


def _regrid(oracle_lib, ps_old, U_old, ps_new):
    O = oracle_lib
    U_new = W.new_arena(ps_new)
    missing = O.AmrOracle(ps_new).regrid_fill(ps_old, U_old, U_new)
    return U_new, missing


def test_linear_field_prolonged_exactly_on_two_new_levels(oracle_lib):
    psA, UA = _root_only()
    _fill_linear_root(psA, UA)
    # the level-2 patch starts at the level-1 patch's low x edge: its prolongation stencils
    # read that patch's ghost layer, itself prolonged from the root
    psB = _hier([(1, [8, 6, 10], [12, 16, 8]), (2, [16, 16, 24], [8, 8, 8])])
    UB, missing = _regrid(oracle_lib, psA, UA, psB)
    assert missing == 0
    assert np.array_equal(psB.active(UB, 0), psA.active(UA, 0))
    for p in (1, 2):
        X, Y, Z, rho = _linear(psB, p)
        ref = W.conserved(rho, 0.3, -0.2, 0.1, 1.0 + 0 * X, 1.4)
        got = psB.active(UB, p)
        for k in range(5):
            assert np.max(np.abs(got[k] - ref[k])) <= 1e-14 * np.max(np.abs(ref[k])), (p, k)


def test_children_average_to_their_parent_on_a_nonlinear_field(oracle_lib):
    psA, UA = _root_only()
    W.random_state(psA, 5, U=UA, amp=0.3, vamp=0.4, shocks=1.0)
    psB = _hier([(1, [4, 8, 6], [16, 8, 12])])
    UB, missing = _regrid(oracle_lib, psA, UA, psB)
    assert missing == 0
    f = psB.active(UB, 1)
    c = psA.active(UA, 0)[:, 3:9, 4:8, 2:10]
    kids = f.reshape(5, 6, 2, 4, 2, 8, 2).mean(axis=(2, 4, 6))
    assert np.max(np.abs(kids - c) / np.abs(c).max(axis=(1, 2, 3), keepdims=True)) <= 1e-15
    # the limiter: no child leaves the range of its parent and the parent's face neighbours
    from oracle import oracle as O
    O.Oracle(psA).fill_ghosts(UA)
    v = psA.view(UA, 0)[0]
    nb = [v[2:-2, 2:-2, 2:-2], v[2:-2, 2:-2, 1:-3], v[2:-2, 2:-2, 3:-1], v[2:-2, 1:-3, 2:-2], v[2:-2, 3:-1, 2:-2],
          v[1:-3, 2:-2, 2:-2], v[3:-1, 2:-2, 2:-2]]
    lo = np.minimum.reduce(nb)[3:9, 4:8, 2:10]
    hi = np.maximum.reduce(nb)[3:9, 4:8, 2:10]
    rho = f[0].reshape(6, 2, 4, 2, 8, 2)
    for a in range(2):
        for b in range(2):
            for d in range(2):
                r = rho[:, a, :, b, :, d]
                assert np.all(r >= lo - 1e-13) and np.all(r <= hi + 1e-13)


def test_old_cells_are_copied_and_the_rest_prolonged(oracle_lib):
    # old hierarchy: root + a level-1 patch holding a state unrelated to the root's
    psA = _hier([(1, [8, 8, 8], [16, 16, 16])])
    UA = W.new_arena(psA)
    W.random_state(psA, 6, U=UA, amp=0.3, vamp=0.4, shocks=1.0)
    # new level-1 patch overlaps the old one in [12, 24) x [8, 20) x [10, 22) and sticks out
    psB = _hier([(1, [12, 4, 10], [16, 16, 16])])
    UB, missing = _regrid(oracle_lib, psA, UA, psB)
    assert missing == 0
    new, old = psB.active(UB, 1), psA.active(UA, 1)
    ov_new = new[:, 0:12, 4:16, 0:12]  # z 10..22, y 8..20, x 12..24 in level-1 space
    ov_old = old[:, 2:14, 0:12, 4:16]
    assert np.array_equal(ov_new, ov_old)
    # a cell outside the old patch is the prolongation of the root: children average to it
    out = new[:, :, 0:4, :]  # y 4..8: no old level-1 cell there
    par = psA.active(UA, 0)[:, 5:13, 2:4, 6:14]
    kids = out.reshape(5, 8, 2, 2, 2, 8, 2).mean(axis=(2, 4, 6))
    assert np.max(np.abs(kids - par) / np.abs(par).max(axis=(1, 2, 3), keepdims=True)) <= 1e-15


def test_a_new_root_without_an_old_source_is_reported(oracle_lib):
    psA = W.make_patchset(3, [[8, 16, 16]], 2, [W.BC_OUTFLOW] * 6, dx0=(1 / NC,) * 3)
    UA = W.new_arena(psA)
    W.random_state(psA, 7, U=UA)
    psB, _ = _root_only()
    _, missing = _regrid(oracle_lib, psA, UA, psB)
    assert missing == 8 * 16 * 16
