"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

None of these tests re-types the oracle's formulas: they check it against an
exact Riemann solution, an exact advected solution, conservation, symmetry,
special cases that reduce to textbook limiters, and a hand-derived worked
example (tests/golden/).
"""
import json
import math
import os

import numpy as np
import pytest

from paper_0910_5547_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def pressure(U, gamma):
    return (gamma - 1.0) * (U[4] - 0.5 * (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / U[0])


# ------------------------------------------------------------------ exact Riemann
def test_exact_riemann_matches_published_sod_star():
    from oracle.exact import RiemannSolution
    g = json.load(open(os.path.join(GOLD, "sod_exact_star.json")))
    s = RiemannSolution(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, 1.4)
    tol = g["tolerance_abs"]
    assert abs(s.p - g["p_star"]) < tol
    assert abs(s.u - g["u_star"]) < tol
    assert abs(s.rhoL - g["rho_star_L"]) < tol
    assert abs(s.rhoR - g["rho_star_R"]) < tol
    assert abs(s.right_waves[0] - g["shock_speed"]) < tol


@pytest.mark.parametrize("flux", [0, 1])
def test_sod_converges_to_exact_solution(oracle_lib, flux):
    """Sec. 6.1 Sod tube at t = 0.2: L1(rho) falls with N at order in [0.6, 1.2];
    star plateaus match the exact values away from the waves."""
    from oracle.exact import RiemannSolution
    ex = RiemannSolution(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, 1.4)
    errs = []
    for N in (100, 200, 400, 800):
        ps, U = W.sod(N)
        o = oracle_lib.Oracle(ps, flux=flux)
        o.run(U, 0.2, cfl=0.8)
        Ua = ps.active(U, 0)[:, 0, 0, :]
        ref = ex.cell_averages(N, 0.2)
        errs.append(np.abs(Ua[0] - ref[0]).sum() / N)
        if N == 800:
            x = (np.arange(N) + 0.5) / N
            p = pressure(Ua, 1.4)
            u = Ua[1] / Ua[0]
            waves = [0.5 + s * 0.2 for s in ex.wave_speeds()]
            # plateaus 20 cells (2.5% of the tube) clear of every wave: the one-speed flux smears
            # the contact and the rarefaction tail over more than 10 cells at N = 800
            far = np.all(np.abs(x[:, None] - np.array(waves)[None, :]) > 20.0 / N, axis=1)
            star = far & (x > waves[1]) & (x < waves[-1])
            assert star.sum() > 20
            assert np.max(np.abs(p[star] - ex.p)) < 1e-3
            assert np.max(np.abs(u[star] - ex.u)) < 1e-3
            sl = star & (x < 0.5 + ex.u * 0.2)
            sr = star & (x > 0.5 + ex.u * 0.2)
            assert np.max(np.abs(Ua[0][sl] - ex.rhoL)) < 1e-3
            assert np.max(np.abs(Ua[0][sr] - ex.rhoR)) < 1e-3
    errs = np.array(errs)
    assert np.all(np.diff(errs) < 0), errs
    order = np.log2(errs[:-1] / errs[1:])
    assert np.all((order > 0.6) & (order < 1.2)), order


# ------------------------------------------------------------------ smooth convergence
@pytest.mark.parametrize("theta,min_order", [(2.0, 1.8), (1.0, 1.6)])
def test_second_order_on_advected_wave(oracle_lib, theta, min_order):
    """rho = 1 + 0.2 sin 2 pi x, v = 1, p = 1, periodic, t = 1: L1 against exact cell averages."""
    from oracle.exact import wave_cell_average
    errs = []
    Ns = (32, 64, 128, 256, 512)
    for N in Ns:
        ps, U = W.advected_wave(N, theta=theta)
        o = oracle_lib.Oracle(ps)
        o.run(U, 1.0, cfl=0.8)
        rho = ps.active(U, 0)[0, 0, 0, :]
        errs.append(np.abs(rho - wave_cell_average(N, 1.0)).sum() / N)
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert order[-1] >= min_order, (errs, order)
    assert np.all(order > 1.0), order


def test_second_order_along_y_and_z(oracle_lib):
    """The same wave advected along y (2D) and z (3D) converges at the same rate as along x."""
    from oracle.exact import wave_cell_average
    for ndim, axis in ((2, 1), (3, 2)):
        errs = []
        for N in (16, 32):
            ps, U = W.advected_wave(N, ndim=ndim, axis=axis, theta=2.0)
            o = oracle_lib.Oracle(ps)
            o.run(U, 0.25, cfl=0.8)
            rho = ps.active(U, 0)[0]
            line = np.moveaxis(rho, 2 - axis, -1).reshape(-1, N)
            # every line across the wave direction is identical
            assert np.all(line == line[0])
            errs.append(np.abs(line[0] - wave_cell_average(N, 0.25)).sum() / N)
        assert math.log2(errs[0] / errs[1]) > 1.5, errs


# ------------------------------------------------------------------ invariants
def _random_3d(n, bc, seed, ng=2, gamma=5.0 / 3.0, theta=1.0, shocks=0.0):
    ps = W.make_patchset(3, [n], ng, [bc] * 6, gamma=gamma, theta=theta, dx0=(1.0 / n[0], 1.0 / n[1], 1.0 / n[2]))
    U = W.random_state(ps, seed, shocks=shocks)
    return ps, U


def test_uniform_state_is_preserved_bitwise(oracle_lib):
    for bc, v in ((W.BC_PERIODIC, (0.3, -0.2, 0.1)), (W.BC_OUTFLOW, (0.3, -0.2, 0.1)), (W.BC_REFLECT, (0, 0, 0))):
        ps = W.make_patchset(3, [[8, 6, 5]], 2, [bc] * 6, gamma=1.4, dx0=(0.1, 0.2, 0.3))
        U = W.new_arena(ps)
        ps.active(U, 0)[...] = W.conserved(np.full((5, 6, 8), 1.3), v[0], v[1], v[2], 0.7, 1.4)
        U0 = U.copy()
        o = oracle_lib.Oracle(ps)
        for _ in range(3):
            o.rk2_step(U, 0.01)
        assert np.array_equal(ps.active(U, 0), ps.active(U0, 0)), bc


def test_conservation_with_periodic_boundaries(oracle_lib):
    """Telescoping of the MOL divergence: totals of rho, rho v, rho E constant to round-off."""
    ps, U = _random_3d([12, 10, 8], W.BC_PERIODIC, seed=5, shocks=1.0)
    o = oracle_lib.Oracle(ps)
    A0 = ps.active(U, 0).reshape(5, -1).copy()
    for _ in range(40):
        o.rk2_step(U, o.cfl_dt(U, 0.8))
    A = ps.active(U, 0).reshape(5, -1)
    for k in range(5):
        scale = math.fsum(np.abs(A0[k]))
        assert abs(math.fsum(A[k]) - math.fsum(A0[k])) <= 1e-12 * scale, k
    assert not np.array_equal(A, A0)


def test_mirror_symmetry_bitwise(oracle_lib):
    """x -> 1 - x with v_x -> -v_x maps solutions to solutions, exactly (Sec. 4 PLM and flux are odd)."""
    ps, U = _random_3d([10, 7, 6], W.BC_OUTFLOW, seed=9, shocks=1.0)
    M = U.copy()
    a = ps.active(M, 0)
    a[...] = a[:, :, :, ::-1]
    a[1] = -a[1]
    o = oracle_lib.Oracle(ps)
    for _ in range(5):
        dt = o.cfl_dt(U, 0.8)
        assert dt == o.cfl_dt(M, 0.8)
        o.rk2_step(U, dt)
        o.rk2_step(M, dt)
    b = ps.active(M, 0)[:, :, :, ::-1].copy()
    b[1] = -b[1]
    assert np.array_equal(b, ps.active(U, 0))


def test_sod_mirror_symmetry_bitwise(oracle_lib):
    ps, U = W.sod(200)
    M = U.copy()
    a = ps.active(M, 0)
    a[...] = a[..., ::-1]
    a[1] = -a[1]
    o = oracle_lib.Oracle(ps)
    for _ in range(50):
        dt = o.cfl_dt(U, 0.8)
        o.rk2_step(U, dt)
        o.rk2_step(M, dt)
    b = ps.active(M, 0)[..., ::-1].copy()
    b[1] = -b[1]
    assert np.array_equal(b, ps.active(U, 0))


def test_axis_permutation(oracle_lib):
    """Every dimension uses the same code: x<->y (data, velocities, dx) commutes with a step."""
    ps, U = _random_3d([9, 7, 6], W.BC_PERIODIC, seed=11, shocks=1.0)
    n = ps.n[0]
    ps2 = W.make_patchset(3, [[n[1], n[0], n[2]]], 2, [W.BC_PERIODIC] * 6, gamma=ps.gamma,
                          dx0=(ps.dx0[1], ps.dx0[0], ps.dx0[2]))
    U2 = W.new_arena(ps2)
    a = ps.active(U, 0)
    ps2.active(U2, 0)[...] = np.swapaxes(a[[0, 2, 1, 3, 4]], 2, 3)
    o1, o2 = oracle_lib.Oracle(ps), oracle_lib.Oracle(ps2)
    dt = o1.cfl_dt(U, 0.8)
    assert abs(dt - o2.cfl_dt(U2, 0.8)) <= 1e-15 * dt
    o1.rk2_step(U, dt)
    o2.rk2_step(U2, dt)
    back = np.swapaxes(ps2.active(U2, 0), 2, 3)[[0, 2, 1, 3, 4]]
    a = ps.active(U, 0)
    for k in range(5):
        scale = np.abs(a[k]).max()
        assert np.max(np.abs(back[k] - a[k])) <= 1e-14 * scale


def test_reflect_equals_mirrored_domain(oracle_lib):
    """A reflecting wall at x = 0 gives bitwise the same as the mirror-extended domain."""
    N = 64
    rng = np.random.default_rng(3)
    rho = 1 + 0.3 * rng.random(N)
    u = 0.4 * (rng.random(N) - 0.5)
    p = 1 + 0.3 * rng.random(N)
    z = np.zeros(N)
    ps1 = W.make_patchset(1, [[N, 1, 1]], 2, [W.BC_REFLECT, W.BC_OUTFLOW] + [0] * 4, dx0=(1.0 / N, 1, 1))
    U1 = W.new_arena(ps1)
    ps1.active(U1, 0)[...] = W.conserved(rho, u, z, z, p, 1.4).reshape(5, 1, 1, N)
    ps2 = W.make_patchset(1, [[2 * N, 1, 1]], 2, [W.BC_OUTFLOW] * 6, dx0=(1.0 / N, 1, 1))
    U2 = W.new_arena(ps2)
    full = W.conserved(np.r_[rho[::-1], rho], np.r_[-u[::-1], u], np.r_[z, z], np.r_[z, z], np.r_[p[::-1], p], 1.4)
    ps2.active(U2, 0)[...] = full.reshape(5, 1, 1, 2 * N)
    o1, o2 = oracle_lib.Oracle(ps1), oracle_lib.Oracle(ps2)
    for _ in range(20):
        o1.rk2_step(U1, 0.2 / N)
        o2.rk2_step(U2, 0.2 / N)
    assert np.array_equal(ps1.active(U1, 0), ps2.active(U2, 0)[..., N:])


def test_periodic_equals_replicated_domain(oracle_lib):
    """Periodic wrap: one period advanced equals the middle of three periods (outflow far away)."""
    N = 32
    ps1, U1 = W.advected_wave(N)
    o1 = oracle_lib.Oracle(ps1)
    ps3 = W.make_patchset(1, [[3 * N, 1, 1]], 2, [W.BC_OUTFLOW] * 6, dx0=(1.0 / N, 1, 1))
    U3 = W.new_arena(ps3)
    a = ps1.active(U1, 0)
    ps3.active(U3, 0)[...] = np.concatenate([a, a, a], axis=-1)
    o3 = oracle_lib.Oracle(ps3)
    for _ in range(4):
        o1.rk2_step(U1, 0.1 / N)
        o3.rk2_step(U3, 0.1 / N)
    assert np.array_equal(ps1.active(U1, 0), ps3.active(U3, 0)[..., N:2 * N])


# ------------------------------------------------------------------ pieces
def test_minmod_special_cases(oracle_lib):
    """theta = 1: classic minmod; theta = 2: the MC limiter; theta = 0: zero slope."""
    rng = np.random.default_rng(0)
    for _ in range(2000):
        a, b = rng.standard_normal(2) * 10.0 ** rng.integers(-3, 3, 2)
        if rng.random() < 0.1:
            b = a
        if rng.random() < 0.05:
            a = 0.0
        classic = 0.0 if a * b <= 0 else math.copysign(min(abs(a), abs(b)), a)
        assert oracle_lib.minmod3(a, b, (a + b) / 2) == classic
        mc = 0.0 if a * b <= 0 else math.copysign(min(2 * abs(a), 2 * abs(b), abs(a + b) / 2), a)
        assert oracle_lib.minmod3(2 * a, 2 * b, (a + b) / 2) == mc
        assert oracle_lib.minmod3(0 * a, 0 * b, (a + b) / 2) == 0.0
    # linear data: every theta >= 1 returns the difference itself
    for th in (1.0, 1.5, 2.0):
        assert oracle_lib.minmod3(th * 0.25, th * 0.25, 0.25) == 0.25


def test_flux_consistency(oracle_lib):
    """F(q, q) = F^d(U(q)): exactly for the printed one-speed flux (0.5 (F + F) - lambda0 * 0 = F);
    to round-off for the two-speed HLL, whose (a+ F + a- F)/(a+ + a-) is not exact in IEEE arithmetic."""
    rng = np.random.default_rng(1)
    for flux in (0, 1):
        ph = oracle_lib.phys(gamma=1.4, flux=flux)
        for _ in range(200):
            q = np.array([rng.uniform(0.1, 3), rng.uniform(0.1, 3), *rng.uniform(-2, 2, 3)])
            for d in range(3):
                a, b = oracle_lib.face_flux(ph, d, q, q), oracle_lib.phys_flux(ph, d, q)
                if flux == 0:
                    assert np.array_equal(a, b)
                else:
                    assert np.max(np.abs(a - b)) <= 4e-16 * np.max(np.abs(b))


def test_hll2_equals_printed_flux_when_speeds_are_symmetric(oracle_lib):
    """With a+ = a- the two-speed HLL flux reduces to the paper's printed formula."""
    rng = np.random.default_rng(2)
    p0, p1 = oracle_lib.phys(gamma=1.4, flux=0), oracle_lib.phys(gamma=1.4, flux=1)
    for _ in range(100):
        rho = rng.uniform(0.2, 2, 2)
        e = np.array([1.7, 1.7])  # equal e -> equal p/rho -> equal c; v_x = 0 -> a+ = a- = c
        qL = np.array([rho[0], e[0], 0, rng.uniform(-1, 1), rng.uniform(-1, 1)])
        qR = np.array([rho[1], e[1], 0, rng.uniform(-1, 1), rng.uniform(-1, 1)])
        a = oracle_lib.face_flux(p0, 0, qL, qR)
        b = oracle_lib.face_flux(p1, 0, qL, qR)
        assert np.allclose(a, b, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("theta", [0.0, 1.0, 2.0])
def test_worked_example_stage1(oracle_lib, theta):
    g = json.load(open(os.path.join(GOLD, "worked_stage1_1d.json")))
    s = g["setup"]
    N = s["n"]
    ps = W.make_patchset(1, [[N, 1, 1]], s["ng"], [W.BC_OUTFLOW] * 6, gamma=s["gamma"], theta=theta,
                         dx0=(s["dx"], 1, 1))
    U = W.new_arena(ps)
    c = np.array(s["cells_rho_v_p"])
    z = np.zeros(N)
    ps.active(U, 0)[...] = W.conserved(c[:, 0], c[:, 1], z, z, c[:, 2], s["gamma"]).reshape(5, 1, 1, N)
    o = oracle_lib.Oracle(ps)
    o.fill_ghosts(U)
    out = U.copy()
    o.stage(U, None, out, s["dt"], 1)
    got = ps.active(out, 0)[:, 0, 0, :].T
    assert np.max(np.abs(got - np.array(g["expected_U1"]))) <= g["tolerance_abs"]


def test_cfl_closed_form_on_uniform_state(oracle_lib):
    ps = W.make_patchset(3, [[6, 5, 4]], 2, [W.BC_PERIODIC] * 6, gamma=5 / 3, dx0=(0.1, 0.05, 0.2))
    U = W.new_arena(ps)
    v = (0.3, -0.7, 0.2)
    ps.active(U, 0)[...] = W.conserved(np.full((4, 5, 6), 2.0), *v, 3.0, 5 / 3)
    o = oracle_lib.Oracle(ps)
    c = math.sqrt(5 / 3 * 3.0 / 2.0)
    expect = 0.8 / ((abs(v[0]) + c) / 0.1 + (abs(v[1]) + c) / 0.05 + (abs(v[2]) + c) / 0.2)
    assert abs(o.cfl_dt(U, 0.8) - expect) <= 2e-16 * expect


def test_unphysical_state_is_flagged(oracle_lib):
    ps = W.make_patchset(1, [[8, 1, 1]], 2, [W.BC_OUTFLOW] * 6, dx0=(0.125, 1, 1))
    U = W.new_arena(ps)
    z = np.zeros(8)
    ps.active(U, 0)[...] = W.conserved(np.ones(8), z, z, z, np.ones(8), 1.4).reshape(5, 1, 1, 8)
    o = oracle_lib.Oracle(ps)
    assert o.rk2_step(U.copy(), 0.01) == 0
    ps.active(U, 0)[4, 0, 0, 3] = -1.0
    assert o.rk2_step(U, 0.01) == 1


def test_external_sibling_ghosts_equal_single_patch(oracle_lib):
    """A periodic box cut into 8 patches with EXTERNAL faces (sibling ghosts, periodic
    wrap of the root domain) evolves bitwise like the same box as one periodic patch."""
    N, P = 16, 8
    ps1, U1 = W.periodic_turbulent_box(N=N, seed=3, kmax=4.0)
    ps8, U8 = W.periodic_turbulent_box(N=N, seed=3, kmax=4.0, patch=P)
    o1 = oracle_lib.Oracle(ps1)
    o8 = oracle_lib.Oracle(ps8, periodic=7, domain=(N, N, N))
    for _ in range(3):
        dt = o1.cfl_dt(U1, 0.8)
        assert dt == o8.cfl_dt(U8, 0.8)
        o1.rk2_step(U1, dt)
        o8.rk2_step(U8, dt)
    a = ps1.active(U1, 0)
    for p in range(ps8.npatch):
        lo = ps8.lo[p]
        assert np.array_equal(ps8.active(U8, p), a[:, lo[2]:lo[2] + P, lo[1]:lo[1] + P, lo[0]:lo[0] + P])
