"""Pins of the oracle's refinement flags (the density-gradient criterion the deep-AMR
set-up places its levels with): a cell is flagged where |rho_n - rho_c| / min(rho_n, rho_c)
exceeds eps for a face neighbour n."""
import numpy as np

from paper_0910_5547_amd import workloads as W


def _patch(n, bc, rho):
    ps = W.make_patchset(3, [n], 2, [bc] * 6, gamma=1.4, dx0=(0.1, 0.1, 0.1))
    U = W.new_arena(ps)
    ps.active(U, 0)[...] = W.conserved(rho, 0.0, 0.0, 0.0, 1.0, 1.4)
    return ps, U


def test_step_flags_exactly_the_two_layers_at_the_jump(oracle_lib):
    n = [12, 7, 5]
    rho = np.ones((5, 7, 12))
    rho[:, :, 6:] = 1.5  # jump of 50 % between x = 5 and x = 6
    for bc in (W.BC_OUTFLOW, W.BC_REFLECT):
        ps, U = _patch(n, bc, rho)
        o = oracle_lib.Oracle(ps)
        f = o.flag_cells(U, 0.3).reshape(5, 7, 12)
        expect = np.zeros((5, 7, 12), np.uint8)
        expect[:, :, 5:7] = 1
        assert np.array_equal(f, expect), bc
        assert not o.flag_cells(U, 0.5).any()  # the jump is exactly 0.5: not above it


def test_periodic_seam_and_linear_ramp(oracle_lib):
    n = [10, 4, 4]
    x = np.arange(10)
    rho = np.broadcast_to(1.0 + 0.1 * x, (4, 4, 10)).copy()  # ratio of neighbours (1+0.1(i+1))/(1+0.1 i)
    ps, U = _patch(n, W.BC_PERIODIC, rho)
    o = oracle_lib.Oracle(ps)
    f = o.flag_cells(U, 0.3).reshape(4, 4, 10)
    # inside the ramp every jump is 0.1/(1+0.1 i) <= 0.1; across the seam rho goes 1.9 -> 1.0 (0.9)
    expect = np.zeros((4, 4, 10), np.uint8)
    expect[:, :, 0] = expect[:, :, 9] = 1
    assert np.array_equal(f, expect)
    assert o.flag_cells(U, 0.05).reshape(4, 4, 10)[:, :, :6].all()  # 0.1/(1+0.1 i) > 0.05 for i < 10


def test_uniform_state_has_no_flags_and_counts_match(oracle_lib):
    ps, U = W.uneven_patches(npatch=5, seed=3)
    o = oracle_lib.Oracle(ps)
    f = o.flag_cells(U, 0.2)
    assert f.size == ps.active_cells()
    ps2, U2 = _patch([6, 6, 6], W.BC_PERIODIC, np.full((6, 6, 6), 2.0))
    assert not oracle_lib.Oracle(ps2).flag_cells(U2, 1e-12).any()
