"""Pin of the subcycled step's time schedule (temporal refinement, Sec. 3; RK2
equation, Sec. 4).

A linear density ramp carried by a uniform velocity at uniform pressure,
rho = rho0 + g . (x - v t), is an exact solution of the Euler equations, and every
operator of the subcycled scheme reproduces it exactly (up to rounding) when the
reconstructed set is (rho, p, v) with theta = 1:

* PLM: the limited slope of linear data is the data's own slope, so both face
  states equal the face-centre value and the Riemann flux is the physical flux of
  that state (U_R - U_L = 0);
* the flux divergence of a linear field is constant, so L(U) is the same at both
  RK stages and RK2 integrates it exactly;
* the minmod-linear coarse -> fine prolongation is exact for linear data, and so
  is linear interpolation in time between a coarse level's old and new states,
  provided each stage takes the coarse state at the stage input's own time:
  fraction s/2 of the parent step for stage 1 of substep s, (s + 1)/2 for stage 2;
* refluxing corrects by zero (coarse and fine face fluxes agree) and restriction
  (the mean of the children) is exact for linear data.

Any other choice of those fractions (the same fraction for both stages, no time
interpolation, the two fractions exchanged) offsets the prolonged ghosts by about
g . v dt_c / 2 and the fine cells next to them by far more than round-off.  Root
faces are outflow (a ramp is not periodic); their zero-gradient ghosts perturb
only cells within 2 cells per stage of the domain faces, so the check covers every
refined cell and the root cells outside that band.
"""
import numpy as np
import pytest

from paper_0910_5547_amd import workloads as W

GAMMA = 1.4
P0 = 1.0
RHO0 = 1.0


def ramp_state(X, grad, vel, t):
    """Conserved state of the advected ramp at cell centres X (list of arrays)."""
    rho = RHO0 + sum(g * (x - v * t) for g, x, v in zip(grad, X, vel))
    v3 = list(vel) + [0.0] * (3 - len(vel))
    return W.conserved(rho, v3[0], v3[1], v3[2], P0, GAMMA)


def ramp_hierarchy(ndim, Nc, boxes, grad, vel, ng=3):
    """Root of Nc^ndim cells (outflow faces) and a chain of nested patches, boxes[i] =
    (lo, hi) in level-i cells in every dimension; the ramp at t = 0 everywhere."""
    los, ns, levels, bcs = [[0, 0, 0]], [[Nc if d < ndim else 1 for d in range(3)]], [0], [[W.BC_OUTFLOW] * 6]
    for i, (lo, hi) in enumerate(boxes):
        los.append([2 * lo if d < ndim else 0 for d in range(3)])
        ns.append([2 * (hi - lo) if d < ndim else 1 for d in range(3)])
        levels.append(i + 1)
        bcs.append([W.BC_EXTERNAL] * 6)
    dx0 = tuple(1.0 / Nc if d < ndim else 1.0 for d in range(3))
    ps = W.make_patchset(ndim, ns, ng, bcs, level=levels, lo=los, gamma=GAMMA, theta=1.0, dx0=dx0)
    U = W.new_arena(ps)
    for p in range(ps.npatch):
        ps.active(U, p)[...] = ramp_state(cell_centres(ps, p), grad, vel, 0.0)
    return ps, U


def cell_centres(ps, p):
    """Cell-centre coordinates (x, y, z)[:ndim] of patch p's active cells, (nz, ny, nx) arrays."""
    lvl = int(ps.level[p])
    axes = []
    for d in range(3):
        n = int(ps.n[p, d])
        h = ps.dx0[d] / 2 ** lvl
        axes.append((int(ps.lo[p, d]) + np.arange(n) + 0.5) * h)
    Z, Y, X = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return [X, Y, Z][:ps.ndim]


CASES = {
    # ndim: (root cells, nested boxes, density gradient, velocity)
    1: (64, [(24, 40), (56, 72)], (0.5,), (1.0,)),
    3: (32, [(12, 20), (28, 36)], (0.3, -0.2, 0.1), (1.0, 0.5, -0.25)),
}


def run_ramp(oracle_lib, ndim, nlev, steps=2):
    Nc, boxes, grad, vel = CASES[ndim]
    ps, U = ramp_hierarchy(ndim, Nc, boxes[:nlev - 1], grad, vel)
    a = oracle_lib.AmrOracle(ps, recon=oracle_lib.RECON_P)
    t = 0.0
    for _ in range(steps):
        dt0 = a.cfl_dt0(U, 0.8)
        a.advance(U, dt0)
        t += dt0
    return ps, U, t, steps


def ramp_errors(ps, U, t, steps):
    """Max |U - exact| over every refined cell and over the root cells at least
    4 root cells per root step from every domain face; per level."""
    ndim = ps.ndim
    Nc = int(ps.n[0, 0])
    band = 4 * steps
    errs = {}
    for p in range(ps.npatch):
        grad, vel = CASES[ndim][2], CASES[ndim][3]
        exact = ramp_state(cell_centres(ps, p), grad, vel, t)
        got = ps.active(U, p)
        diff = np.abs(got - exact)
        if ps.level[p] == 0:
            sl = tuple(slice(band, Nc - band) if d < ndim else slice(None) for d in (2, 1, 0))
            diff = diff[(slice(None),) + sl]
        lv = int(ps.level[p])
        errs[lv] = max(errs.get(lv, 0.0), float(diff.max()))
    return errs


@pytest.mark.parametrize("ndim,nlev", [(1, 2), (1, 3), (3, 2), (3, 3)])
def test_subcycled_ramp_is_exact(oracle_lib, ndim, nlev):
    ps, U, t, steps = run_ramp(oracle_lib, ndim, nlev)
    errs = ramp_errors(ps, U, t, steps)
    assert set(errs) == set(range(nlev))
    for lv, e in errs.items():
        assert e <= 1e-13, (lv, errs)


def test_outflow_band_is_where_the_ramp_is_not_exact(oracle_lib):
    """Negative control of the check's region: the root cells next to the outflow faces
    do depart from the ramp (the zero-gradient ghosts are not its extension), so the
    exactness above is a property of the refined region, not of the comparison."""
    ps, U, t, steps = run_ramp(oracle_lib, 1, 2)
    exact = ramp_state(cell_centres(ps, 0), CASES[1][2], CASES[1][3], t)
    edge = np.abs(ps.active(U, 0) - exact)[0, 0, 0, :2]
    assert edge.max() > 1e-4
