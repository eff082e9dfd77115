"""Pins of the oracle's ideal-MHD path (8 variables, the cleaning field held at zero).

The MHD section of the paper gives the conserved variables and the three flux
vectors; the checks here come from outside the oracle's own formulas:

* with B = 0 the MHD update must reduce to the hydro update bit for bit;
* the fast magnetosonic speed has closed forms along and across the field;
* a circularly polarised Alfven wave is an exact nonlinear travelling solution
  of ideal MHD: the scheme must converge to it along x, y and z (the y and z
  runs exercise the y and z flux vectors, whose printed induction entries are
  permuted; a wrong entry makes the wave fall apart);
* exact symmetries (mirror x -> -x with v_x, B_x negated; x <-> y exchange),
  telescoping conservation, the constancy of the normal field in 1D and the
  exact integral balance of the Brio-Wu tube before its waves reach the ends.

Brio-Wu itself has no closed-form solution: beyond these invariants its
profile is parity unpinned.
"""
import math

import numpy as np
import pytest

from paper_0910_5547_amd import workloads as W


def _mhd_random(n, bc, seed, ndim=3, ng=2, gamma=5.0 / 3.0, theta=1.0, shocks=0.0, bamp=0.5):
    dx0 = tuple(1.0 / n[d] if d < ndim else 1.0 for d in range(3))
    ps = W.make_patchset(ndim, [n], ng, [bc] * 6, gamma=gamma, theta=theta, dx0=dx0, nvar=W.NVAR_MHD)
    U = W.random_state(ps, seed, shocks=shocks, bamp=bamp)
    return ps, U


def test_zero_field_reduces_to_hydro_bitwise(oracle_lib):
    n = [10, 8, 6]
    psh = W.make_patchset(3, [n], 2, [W.BC_OUTFLOW] * 6, gamma=5 / 3, dx0=(0.1, 0.125, 1 / 6))
    Uh = W.random_state(psh, 7, shocks=1.0)
    psm = W.make_patchset(3, [n], 2, [W.BC_OUTFLOW] * 6, gamma=5 / 3, dx0=(0.1, 0.125, 1 / 6), nvar=W.NVAR_MHD)
    Um = W.new_arena(psm)
    am = psm.active(Um, 0)
    am[:5] = psh.active(Uh, 0)
    am[5:] = 0.0
    oh, om = oracle_lib.Oracle(psh), oracle_lib.Oracle(psm)
    for _ in range(4):
        dt = oh.cfl_dt(Uh, 0.8)
        assert dt == om.cfl_dt(Um, 0.8)
        oh.rk2_step(Uh, dt)
        om.rk2_step(Um, dt)
    assert np.array_equal(psm.active(Um, 0)[:5], psh.active(Uh, 0))
    assert not np.any(psm.active(Um, 0)[5:])


def test_fast_speed_closed_forms(oracle_lib):
    rng = np.random.default_rng(4)
    ph = oracle_lib.phys(gamma=5 / 3, nvar=8)
    for _ in range(300):
        rho, e = rng.uniform(0.1, 3.0, 2)
        v = rng.uniform(-1, 1, 3)
        a2 = 5 / 3 * (2 / 3) * e  # gamma p / rho with p = (gamma - 1) rho e
        for d in range(3):
            B = np.zeros(3)
            B[d] = rng.uniform(-3, 3)  # field along d: c_f = max(a, |B_d| / sqrt(rho))
            q = np.r_[rho, e, v, B]
            cf = oracle_lib.signal_speed(ph, d, q)
            assert abs(cf - max(math.sqrt(a2), abs(B[d]) / math.sqrt(rho))) <= 4e-16 * cf
            B = rng.uniform(-3, 3, 3)
            B[d] = 0.0  # field across d: c_f^2 = a^2 + B^2 / rho
            q = np.r_[rho, e, v, B]
            cf = oracle_lib.signal_speed(ph, d, q)
            assert abs(cf - math.sqrt(a2 + B @ B / rho)) <= 4e-16 * cf
            B = rng.uniform(-3, 3, 3)  # general: c_f is the larger root of the fast/slow quartic
            q = np.r_[rho, e, v, B]
            cf = oracle_lib.signal_speed(ph, d, q)
            b2, bd2 = B @ B / rho, B[d] ** 2 / rho
            quartic = cf ** 4 - (a2 + b2) * cf ** 2 + a2 * bd2
            assert abs(quartic) <= 1e-13 * (a2 + b2) ** 2
            assert cf ** 2 >= 0.5 * (a2 + b2) * (1 - 1e-15)
    # no field: the sound speed
    assert oracle_lib.signal_speed(ph, 0, np.r_[2.0, 1.5, 0, 0, 0, 0, 0, 0]) == math.sqrt(5 / 3 * 2 / 3 * 1.5)


def test_flux_consistency_mhd(oracle_lib):
    """F(q, q) = F^d(U(q)) exactly for the printed flux, and F^d of B_d is zero."""
    rng = np.random.default_rng(5)
    ph = oracle_lib.phys(gamma=1.4, nvar=8)
    for _ in range(200):
        q = np.r_[rng.uniform(0.1, 3, 2), rng.uniform(-2, 2, 6)]
        for d in range(3):
            F = oracle_lib.phys_flux(ph, d, q)
            assert np.array_equal(oracle_lib.face_flux(ph, d, q, q), F)
            assert F[5 + d] == 0.0
            assert F[0] == q[0] * q[2 + d]


def _alfven_run(oracle_lib, N, ndim, axis, t, dt=None):
    """Run the wave to t (CFL 0.8 steps, or fixed steps dt); return the L1 error of the first
    transverse field component against its exact cell averages, and the variables along one
    line in wave-frame order (rho, v_par, v_t1, v_t2, energy, B_par, B_t1, B_t2)."""
    ps, U = W.alfven_wave(N, ndim=ndim, axis=axis)
    o = oracle_lib.Oracle(ps)
    if dt is None:
        o.run(U, t, cfl=0.8)
    else:
        for _ in range(int(round(t / dt))):
            o.rk2_step(U, dt)
    a = ps.active(U, 0)
    b1, b2 = (axis + 1) % 3, (axis + 2) % 3
    order = [0, 1 + axis, 1 + b1, 1 + b2, 4, 5 + axis, 5 + b1, 5 + b2]
    lines = np.stack([np.moveaxis(a[k], 2 - axis, -1).reshape(-1, N) for k in order])
    assert np.all(lines == lines[:, :1])  # every line across the wave is identical
    xl = np.arange(N) / N  # B_t1 = amp sin(2 pi (x - t)): exact cell averages over [x_l, x_l + 1/N]
    exact = 0.1 * (np.cos(2 * np.pi * (xl - t)) - np.cos(2 * np.pi * (xl + 1.0 / N - t))) * N / (2 * np.pi)
    return np.abs(lines[6, 0] - exact).sum() / N, lines[:, 0]


def test_alfven_wave_converges_along_x(oracle_lib):
    """One period (t = 1): L1 error of B_y against the exact cell averages, mean |B_y| = 0.064."""
    errs = [_alfven_run(oracle_lib, N, 1, 0, 1.0)[0] for N in (32, 64, 128, 256, 512)]
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert order[-1] >= 1.6 and np.all(order > 1.0), (errs, order)
    assert errs[-1] < 2e-4, errs


@pytest.mark.parametrize("ndim,axis", [(2, 1), (3, 2)])
def test_alfven_wave_along_y_and_z_matches_x(oracle_lib, ndim, axis):
    """The wave along y (z) uses only the y (z) flux vector.  With the same fixed steps it must
    reproduce the x run to round-off in every variable, so the y and z flux vectors are the x
    flux vector with permuted components.  The parallel velocity is zero in the exact solution
    and stays at truncation-error size."""
    N, dt, t = 32, 0.25 / 32, 0.25
    ex, lx = _alfven_run(oracle_lib, N, 1, 0, t, dt)
    ey, ly = _alfven_run(oracle_lib, N, ndim, axis, t, dt)
    assert ex < 5e-3
    assert np.max(np.abs(ly - lx)) <= 1e-13, np.max(np.abs(ly - lx), axis=1)
    assert np.max(np.abs(ly[1])) < 1e-3


def test_mirror_symmetry_bitwise_mhd(oracle_lib):
    """x -> 1 - x with v_x and B_x negated maps ideal-MHD solutions to solutions, exactly."""
    ps, U = _mhd_random([10, 7, 6], W.BC_OUTFLOW, seed=9, shocks=1.0)
    M = U.copy()
    a = ps.active(M, 0)
    a[...] = a[:, :, :, ::-1]
    a[1], a[5] = -a[1], -a[5]
    o = oracle_lib.Oracle(ps)
    for _ in range(5):
        dt = o.cfl_dt(U, 0.8)
        assert dt == o.cfl_dt(M, 0.8)
        o.rk2_step(U, dt)
        o.rk2_step(M, dt)
    b = ps.active(M, 0)[:, :, :, ::-1].copy()
    b[1], b[5] = -b[1], -b[5]
    assert np.array_equal(b, ps.active(U, 0))


def test_xy_exchange_bitwise_mhd(oracle_lib):
    """Exchanging x and y (data, velocity and field components, cell sizes) commutes with a step
    to the last bit: the x and y flux vectors are the same function of permuted arguments."""
    ps, U = _mhd_random([9, 7, 1], W.BC_PERIODIC, seed=11, ndim=2, shocks=1.0)
    n = ps.n[0]
    ps2 = W.make_patchset(2, [[n[1], n[0], 1]], 2, [W.BC_PERIODIC] * 6, gamma=ps.gamma,
                          dx0=(ps.dx0[1], ps.dx0[0], 1.0), nvar=8)
    U2 = W.new_arena(ps2)
    perm = [0, 2, 1, 3, 4, 6, 5, 7]
    ps2.active(U2, 0)[...] = np.swapaxes(ps.active(U, 0)[perm], 2, 3)
    o1, o2 = oracle_lib.Oracle(ps), oracle_lib.Oracle(ps2)
    dt = o1.cfl_dt(U, 0.8)
    assert abs(dt - o2.cfl_dt(U2, 0.8)) <= 1e-15 * dt
    for _ in range(2):
        o1.rk2_step(U, dt)
        o2.rk2_step(U2, dt)
    back = np.swapaxes(ps2.active(U2, 0), 2, 3)[perm]
    a = ps.active(U, 0)
    for k in range(8):
        assert np.max(np.abs(back[k] - a[k])) <= 1e-14 * np.abs(a[k]).max(), k


def test_cyclic_permutation_mhd(oracle_lib):
    """x -> y -> z -> x in 3D: the same solution up to the order of the directional sums."""
    ps, U = _mhd_random([8, 7, 6], W.BC_PERIODIC, seed=12, shocks=1.0)
    n = ps.n[0]
    ps2 = W.make_patchset(3, [[n[2], n[0], n[1]]], 2, [W.BC_PERIODIC] * 6, gamma=ps.gamma,
                          dx0=(ps.dx0[2], ps.dx0[0], ps.dx0[1]), nvar=8)
    U2 = W.new_arena(ps2)
    # new x = old z, new y = old x, new z = old y; arrays are (var, z, y, x)
    perm = [0, 3, 1, 2, 4, 7, 5, 6]
    ps2.active(U2, 0)[...] = np.transpose(ps.active(U, 0)[perm], (0, 2, 3, 1))
    o1, o2 = oracle_lib.Oracle(ps), oracle_lib.Oracle(ps2)
    dt = o1.cfl_dt(U, 0.8)
    o1.rk2_step(U, dt)
    o2.rk2_step(U2, dt)
    inv = [0, 2, 3, 1, 4, 6, 7, 5]
    back = np.transpose(ps2.active(U2, 0), (0, 3, 1, 2))[inv]
    a = ps.active(U, 0)
    for k in range(8):
        assert np.max(np.abs(back[k] - a[k])) <= 1e-13 * np.abs(a[k]).max(), k


def test_conservation_periodic_mhd(oracle_lib):
    ps, U = _mhd_random([12, 10, 8], W.BC_PERIODIC, seed=5, shocks=1.0)
    o = oracle_lib.Oracle(ps)
    A0 = ps.active(U, 0).reshape(8, -1).copy()
    for _ in range(20):
        o.rk2_step(U, o.cfl_dt(U, 0.8))
    A = ps.active(U, 0).reshape(8, -1)
    for k in range(8):
        scale = math.fsum(np.abs(A0[k]))
        assert abs(math.fsum(A[k]) - math.fsum(A0[k])) <= 1e-12 * scale, k
    assert not np.array_equal(A, A0)


def test_uniform_state_preserved_bitwise_mhd(oracle_lib):
    for bc, v in ((W.BC_PERIODIC, (0.3, -0.2, 0.1)), (W.BC_OUTFLOW, (0.3, -0.2, 0.1)), (W.BC_REFLECT, (0, 0, 0))):
        B = (0.7, -0.4, 0.9) if bc != W.BC_REFLECT else (0.0, 0.0, 0.0)
        ps = W.make_patchset(3, [[8, 6, 5]], 2, [bc] * 6, gamma=1.4, dx0=(0.1, 0.2, 0.3), nvar=8)
        U = W.new_arena(ps)
        ps.active(U, 0)[...] = W.conserved_mhd(np.full((5, 6, 8), 1.3), *v, 0.7, *B, 1.4)
        U0 = U.copy()
        o = oracle_lib.Oracle(ps)
        for _ in range(3):
            o.rk2_step(U, 0.01)
        assert np.array_equal(ps.active(U, 0), ps.active(U0, 0)), bc


def test_reflect_equals_mirrored_domain_mhd(oracle_lib):
    """A reflecting wall (normal v and B negated in the ghosts) equals the mirror-extended domain."""
    N = 48
    rng = np.random.default_rng(3)
    rho, p = 1 + 0.3 * rng.random(N), 1 + 0.3 * rng.random(N)
    u, w = 0.4 * (rng.random(N) - 0.5), 0.4 * (rng.random(N) - 0.5)
    bx, by, bz = (0.8 * (rng.random(N) - 0.5) for _ in range(3))
    z = np.zeros(N)
    ps1 = W.make_patchset(1, [[N, 1, 1]], 2, [W.BC_REFLECT, W.BC_OUTFLOW] + [0] * 4, dx0=(1.0 / N, 1, 1), nvar=8)
    U1 = W.new_arena(ps1)
    ps1.active(U1, 0)[...] = W.conserved_mhd(rho, u, w, z, p, bx, by, bz, 1.4).reshape(8, 1, 1, N)
    ps2 = W.make_patchset(1, [[2 * N, 1, 1]], 2, [W.BC_OUTFLOW] * 6, dx0=(1.0 / N, 1, 1), nvar=8)
    U2 = W.new_arena(ps2)
    r = lambda f, s=1.0: np.r_[s * f[::-1], f]  # noqa: E731
    full = W.conserved_mhd(r(rho), r(u, -1), r(w), r(z), r(p), r(bx, -1), r(by), r(bz), 1.4)
    ps2.active(U2, 0)[...] = full.reshape(8, 1, 1, 2 * N)
    o1, o2 = oracle_lib.Oracle(ps1), oracle_lib.Oracle(ps2)
    for _ in range(15):
        o1.rk2_step(U1, 0.2 / N)
        o2.rk2_step(U2, 0.2 / N)
    assert np.array_equal(ps1.active(U1, 0), ps2.active(U2, 0)[..., N:])


def test_external_sibling_ghosts_equal_single_patch_mhd(oracle_lib):
    N, P = 16, 8
    ps1, U1 = W.mhd_vortex_box(N, patch=None, seed=3)
    ps8, U8 = W.mhd_vortex_box(N, patch=P, seed=3)
    o1 = oracle_lib.Oracle(ps1)
    o8 = oracle_lib.Oracle(ps8, periodic=7, domain=(N, N, N))
    for _ in range(2):
        dt = o1.cfl_dt(U1, 0.8)
        assert dt == o8.cfl_dt(U8, 0.8)
        o1.rk2_step(U1, dt)
        o8.rk2_step(U8, dt)
    a = ps1.active(U1, 0)
    for p in range(ps8.npatch):
        lo = ps8.lo[p]
        assert np.array_equal(ps8.active(U8, p), a[:, lo[2]:lo[2] + P, lo[1]:lo[1] + P, lo[0]:lo[0] + P])


def test_brio_wu_invariants(oracle_lib):
    """Brio-Wu to t = 0.1 (N = 200): B_x stays 0.75 and v_z, B_z stay 0 exactly; the totals obey
    the exact integral balance of the end states (the waves have not reached the ends):
    d/dt sum(rho) = 0, d/dt sum(rho v_x) = Pi_L - Pi_R with Pi = p + B^2/2 - B_x^2,
    d/dt sum(rho v_y) = -B_x (B_y,R - B_y,L)... = -1.5, energy and B_y unchanged."""
    N, t = 200, 0.1
    ps, U = W.brio_wu(N)
    A0 = ps.active(U, 0)[:, 0, 0, :].copy()
    o = oracle_lib.Oracle(ps)
    steps = o.run(U, t, cfl=0.8)
    assert steps > 50
    A = ps.active(U, 0)[:, 0, 0, :]
    assert np.all(A[5] == 0.75) and not np.any(A[3]) and not np.any(A[7])
    dx = 1.0 / N
    tot = lambda k, X: math.fsum(X[k]) * dx  # noqa: E731
    PiL, PiR = 1.0 + 0.5 * (0.75 ** 2 + 1) - 0.75 ** 2, 0.1 + 0.5 * (0.75 ** 2 + 1) - 0.75 ** 2
    expect = {0: 0.0, 1: (PiL - PiR) * t, 2: (-0.75 - 0.75) * t, 4: 0.0, 6: 0.0}
    for k, d in expect.items():
        assert abs((tot(k, A) - tot(k, A0)) - d) <= 1e-13, (k, tot(k, A) - tot(k, A0), d)
    # the solution is bounded by the end states in density and is not the initial state
    assert A[0].min() > 0.1 and A[0].max() < 1.0 + 1e-12
    assert not np.array_equal(A, A0)
