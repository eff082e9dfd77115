"""Host clustering (amr_cluster_flags; no device work): the flagged cells of one level become
the next level's boxes by the brick rule that places the deep-AMR configuration's levels.

Pinned against the configuration's own hierarchy: flags computed from the analytic blast
profile on each level's patches (the criterion and points the set-up uses) must give back
exactly the boxes of the next level; and on random flags the boxes must cover the children
of every flagged cell whose bricks nest, be disjoint, brick-aligned, at most a block wide,
and properly nested in the level below."""
import numpy as np
import pytest

from paper_0910_5547_amd import workloads as W


@pytest.fixture(scope="module")
def amr():
    from paper_0910_5547_amd import amr as A
    A.lib()
    return A


def _analytic_flags(ps, level, sol, E, t, eps, rho_floor, p1, root):
    dx = 1.0 / (root << level)
    out = []
    for p in range(ps.npatch):
        if ps.level[p] != level:
            continue
        lo, n = ps.lo[p], ps.n[p]
        ax = [(np.arange(-1, n[d] + 1) + lo[d] + 0.5) * dx for d in range(3)]
        Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
        rho = sol.state(np.sqrt(X * X + Y * Y + Z * Z), E, t, 1.0, p1, rho_floor)[0]
        c = rho[1:-1, 1:-1, 1:-1]
        jump = np.zeros_like(c)
        for sl in ((slice(2, None), slice(1, -1), slice(1, -1)), (slice(0, -2), slice(1, -1), slice(1, -1)),
                   (slice(1, -1), slice(2, None), slice(1, -1)), (slice(1, -1), slice(0, -2), slice(1, -1)),
                   (slice(1, -1), slice(1, -1), slice(2, None)), (slice(1, -1), slice(1, -1), slice(0, -2))):
            nb = rho[sl]
            jump = np.maximum(jump, np.abs(nb - c) / np.minimum(nb, c))
        out.append((jump > eps).astype(np.uint8).ravel())
    return np.concatenate(out)


def test_clustering_rebuilds_the_deep_amr_hierarchy(amr):
    root, t, eps, rho_floor, p1 = 64, 0.05, 0.3, 1e-2, 1e-5
    ps, _, _, dom = W.sedov_hierarchy(root=root, levels=6, with_state=False)
    sol = W.SedovSolution(5.0 / 3.0)
    descs = amr.descriptors(ps)
    nlev = int(ps.level.max()) + 1
    for l in range(nlev - 1):
        flags = _analytic_flags(ps, l, sol, 8.0, t, eps, rho_floor, p1, root)
        boxes = amr.amr_cluster_flags(descs, 3, dom, l, flags)
        want = sorted((tuple(int(x) for x in ps.lo[p]) + tuple(int(x) for x in ps.n[p]))
                      for p in range(ps.npatch) if ps.level[p] == l + 1)
        got = [tuple(int(x) for x in b) for b in boxes]
        assert got == want, (l, len(got), len(want))


def test_random_flags_give_nested_disjoint_covering_boxes(amr):
    rng = np.random.default_rng(4)
    N = 32
    ps = W.make_patchset(3, [[16, 16, 16]] * 8, 2, [W.BC_OUTFLOW] * 6,
                         lo=[[16 * i, 16 * j, 16 * k] for k in range(2) for j in range(2) for i in range(2)])
    descs = amr.descriptors(ps)
    flags = (rng.random(ps.active_cells()) < 0.01).astype(np.uint8)
    boxes = amr.amr_cluster_flags(descs, 3, (N, N, N), 0, flags, brick=8, block=32)
    assert len(boxes) > 0
    occ = np.zeros((2 * N,) * 3, np.int32)
    for b in boxes:
        lo, n = b[:3], b[3:]
        assert np.all(lo % 8 == 0) and np.all(n % 8 == 0) and np.all(n <= 32) and np.all(n >= 8)
        occ[lo[2]:lo[2] + n[2], lo[1]:lo[1] + n[1], lo[0]:lo[0] + n[0]] += 1
    assert occ.max() == 1  # disjoint
    # every flagged cell whose children's bricks nest inside the domain is covered
    w = 0
    for p in range(ps.npatch):
        lo, n = ps.lo[p], ps.n[p]
        for k in range(n[2]):
            for j in range(n[1]):
                for i in range(n[0]):
                    if flags[w]:
                        c = np.array([lo[0] + i, lo[1] + j, lo[2] + k])
                        # a brick with a footprint one coarse cell from the domain edge nests on
                        # this fully covered level, so every flagged cell is refined
                        assert occ[2 * c[2], 2 * c[1], 2 * c[0]] == 1, c
                    w += 1
    # a hole in the level below: bricks whose dilated footprint reaches it are dropped
    descs2 = amr.descriptors(W.make_patchset(3, [[16, 16, 16]] * 7, 2, [W.BC_OUTFLOW] * 6,
                                             lo=[[16 * i, 16 * j, 16 * k] for k in range(2) for j in range(2)
                                                 for i in range(2)][:7]))
    f2 = np.ones(7 * 16 ** 3, np.uint8)
    boxes2 = amr.amr_cluster_flags(descs2, 3, (N, N, N), 0, f2)
    for b in boxes2:
        lo, n = b[:3], b[3:]
        clo, chi = np.maximum(lo // 2 - 1, 0), np.minimum((lo + n + 1) // 2 + 1, N)
        assert not (np.all(chi > 16) and np.all(clo < 32) and np.all(chi > 16))  # misses the missing block


def test_bad_arguments(amr):
    ps = W.make_patchset(3, [[12, 16, 16]], 2, [W.BC_OUTFLOW] * 6)  # not brick-aligned
    import ctypes as C
    descs = amr.descriptors(ps)
    out = np.zeros(60, np.int32)
    n = C.c_int32(0)
    dom = (C.c_int32 * 3)(12, 16, 16)
    f = np.zeros(12 * 16 * 16, np.uint8)
    st = amr.lib().amr_cluster_flags(descs, 1, 3, dom, 0, f.ctypes.data_as(C.POINTER(C.c_uint8)), 8, 32,
                                     out.ctypes.data_as(C.POINTER(C.c_int32)), 10, C.byref(n))
    assert st == amr.AMR_EINVAL


def test_level_whose_extent_overflows_is_rejected(amr):
    """A level whose index extent (domain << level) exceeds an int32 is an invalid argument."""
    import ctypes as C
    ps = W.make_patchset(3, [[16, 16, 16]], 2, [W.BC_OUTFLOW] * 6)
    descs = amr.descriptors(ps)
    out = np.zeros(60, np.int32)
    n = C.c_int32(0)
    dom = (C.c_int32 * 3)(16, 16, 16)
    f = np.zeros(16 ** 3, np.uint8)
    for level in (28, 31):
        st = amr.lib().amr_cluster_flags(descs, 1, 3, dom, level, f.ctypes.data_as(C.POINTER(C.c_uint8)), 8, 32,
                                         out.ctypes.data_as(C.POINTER(C.c_int32)), 10, C.byref(n))
        assert st == amr.AMR_EINVAL, level


def test_short_flags_are_rejected_by_the_binding(amr):
    """The binding checks the host flags against the level's cell count before the library reads them."""
    ps = W.make_patchset(3, [[16, 16, 16]], 2, [W.BC_OUTFLOW] * 6)
    with pytest.raises(ValueError):
        amr.amr_cluster_flags(amr.descriptors(ps), 3, (16, 16, 16), 0, np.zeros(16 ** 3 - 1, np.uint8))
