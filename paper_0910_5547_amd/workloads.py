"""Seeded synthetic inputs for the per-patch hydro update (shared by both sides).

This module holds the problem set-ups only: patch geometry (the descriptor
table in a neutral numpy form) and initial conserved states built from
primitive fields.  It contains none of the update's arithmetic (no
reconstruction, flux, divergence or time stepping) and imports neither the GPU
library nor the oracle; both sides marshal a :class:`PatchSet` into their own
formats.

Set-ups (the paper's workloads are analytic problems fully specified in its
text; no dataset is involved):

* :func:`sod` - the 1D shock tube of Sec. 6.1 (Sod 1978), at any N.
* :func:`grf` / :func:`periodic_turbulent_box` - a 3D periodic box with a
  Gaussian random density field and Mach 0.5 random velocities, the synthetic
  stand-in for the paper's uniform-grid 3D runs of Sec. 6.2.
* :func:`uneven_patches` - thousands of independent patches of uneven sizes
  8..32 per dimension with smooth states and random planar shocks, the
  synthetic stand-in for the many grids of an AMR hierarchy (Sec. 3, Sec. 6.3).
* :func:`advected_wave` - a smooth density wave advected at v = 1 (exact
  solution known), for convergence tests.
* :func:`brio_wu` - the 1D MHD shock tube of the paper's MHD section
  (Brio & Wu 1988), Gamma = 2, N = 200.
* :func:`alfven_wave` - a circularly polarised Alfven wave, an exact nonlinear
  travelling solution of ideal MHD, for convergence tests of the MHD fluxes.
* :func:`mhd_vortex_box` - a 3D periodic MHD box (Orszag-Tang-like vortex
  velocity, divergence-free random field B = curl A), split into patches with
  EXTERNAL faces: the synthetic stand-in for the paper's 3D MHD runs.

Initial states are set from (rho, v, p) with the ideal-gas relation of Sec. 4,
rho E = p/(gamma-1) + rho |v|^2 / 2 - the definition of the conserved energy,
needed identically by both sides to build the same input.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BC_OUTFLOW, BC_PERIODIC, BC_REFLECT, BC_EXTERNAL = 0, 1, 2, 3
NVAR = 5       # hydro: (rho, rho v, rho E)
NVAR_MHD = 8   # ideal MHD: (rho, rho v, rho E + B^2/2, B), the divergence-cleaning field held at 0
NVAR_GLM = 9   # GLM-MHD: (rho, rho v, rho E + B^2/2, B, psi)


@dataclasses.dataclass
class PatchSet:
    """A table of patches in a single FP64 arena (SoA per patch).

    Patch p stores ``s = n + 2 g`` cells per dimension (``g = ng`` in the first
    ``ndim`` dimensions, 0 elsewhere); variable k of patch p starts at element
    ``offset[p] + k * prod(s)``; x is the fastest index.
    """

    ndim: int
    level: np.ndarray   # (np,) int32
    lo: np.ndarray      # (np,3) int32, lower active index in level space
    n: np.ndarray       # (np,3) int32, active cells (1 in absent dims)
    ng: np.ndarray      # (np,) int32
    bc: np.ndarray      # (np,6) int32, faces -x,+x,-y,+y,-z,+z
    offset: np.ndarray  # (np,) int64
    arena: int          # total elements of one arena copy
    gamma: float = 1.4
    theta: float = 1.0
    dx0: tuple = (1.0, 1.0, 1.0)
    nvar: int = NVAR

    @property
    def npatch(self) -> int:
        return int(self.n.shape[0])

    def stored_shape(self, p: int):
        g = [int(self.ng[p]) if d < self.ndim else 0 for d in range(3)]
        return tuple(int(self.n[p, d]) + 2 * g[d] for d in range(3)), g

    def active_cells(self, level: int = -1) -> int:
        sel = np.ones(self.npatch, bool) if level < 0 else (self.level == level)
        return int(np.prod(self.n[sel].astype(np.int64), axis=1).sum())

    def meta(self) -> np.ndarray:
        """(np, 16) int32 rows: level, lo[3], n[3], ng, bc[6], 0, 0."""
        m = np.zeros((self.npatch, 16), np.int32)
        m[:, 0] = self.level
        m[:, 1:4] = self.lo
        m[:, 4:7] = self.n
        m[:, 7] = self.ng
        m[:, 8:14] = self.bc
        return m

    def view(self, U: np.ndarray, p: int) -> np.ndarray:
        """(nvar, sz, sy, sx) view of patch p (storage incl. ghosts) in arena U."""
        s, _ = self.stored_shape(p)
        S = s[0] * s[1] * s[2]
        o = int(self.offset[p])
        return U[o:o + self.nvar * S].reshape(self.nvar, s[2], s[1], s[0])

    def active(self, U: np.ndarray, p: int) -> np.ndarray:
        """(nvar, nz, ny, nx) view of the active cells of patch p."""
        v = self.view(U, p)
        _, g = self.stored_shape(p)
        n = self.n[p]
        return v[:, g[2]:g[2] + n[2], g[1]:g[1] + n[1], g[0]:g[0] + n[0]]


def make_patchset(ndim, n, ng, bc, level=None, lo=None, gamma=1.4, theta=1.0, dx0=(1.0, 1.0, 1.0),
                  align=64, nvar=NVAR) -> PatchSet:
    """Lay out patches back to back in one arena, each start aligned to ``align`` elements."""
    n = np.asarray(n, np.int32).reshape(-1, 3)
    npch = n.shape[0]
    ng = np.broadcast_to(np.asarray(ng, np.int32), (npch,)).copy()
    bc = np.broadcast_to(np.asarray(bc, np.int32), (npch, 6)).copy()
    level = np.zeros(npch, np.int32) if level is None else np.asarray(level, np.int32)
    lo = np.zeros((npch, 3), np.int32) if lo is None else np.asarray(lo, np.int32).reshape(-1, 3)
    off = np.zeros(npch, np.int64)
    cur = 0
    for p in range(npch):
        s = [int(n[p, d]) + (2 * int(ng[p]) if d < ndim else 0) for d in range(3)]
        cur = (cur + align - 1) // align * align
        off[p] = cur
        cur += nvar * s[0] * s[1] * s[2]
    return PatchSet(ndim, level, lo, n, ng, bc, off, cur, float(gamma), float(theta),
                    tuple(float(x) for x in dx0), int(nvar))


def conserved(rho, vx, vy, vz, p, gamma):
    """Conserved (rho, rho v, rho E) from primitives (Sec. 4 ideal gas)."""
    rho = np.asarray(rho, np.float64)
    E = p / (gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy + vz * vz)
    return np.stack(np.broadcast_arrays(rho, rho * vx, rho * vy, rho * vz, E))


def conserved_mhd(rho, vx, vy, vz, p, Bx, By, Bz, gamma):
    """Conserved ideal-MHD variables (rho, rho v, rho E + B^2/2, B) from primitives; the energy
    variable is the definition p/(gamma-1) + rho |v|^2/2 + |B|^2/2 of the paper's MHD section."""
    rho = np.asarray(rho, np.float64)
    E = p / (gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy + vz * vz) + 0.5 * (Bx * Bx + By * By + Bz * Bz)
    return np.stack(np.broadcast_arrays(rho, rho * vx, rho * vy, rho * vz, E, Bx, By, Bz)).astype(np.float64)


def conserved_glm(rho, vx, vy, vz, p, Bx, By, Bz, psi, gamma):
    """GLM-MHD conserved variables: the ideal-MHD set followed by the cleaning field psi."""
    U8 = conserved_mhd(rho, vx, vy, vz, p, Bx, By, Bz, gamma)
    return np.concatenate([U8, np.broadcast_to(np.asarray(psi, np.float64), U8.shape[1:])[None]])


def new_arena(ps: PatchSet, fill=np.nan) -> np.ndarray:
    """An arena whose ghost cells hold ``fill`` (NaN: any read of an unfilled ghost shows)."""
    return np.full(ps.arena, fill, np.float64)


# ---------------------------------------------------------------- 1D set-ups
def sod(N=400, ng=2, gamma=1.4, theta=1.0, x0=0.5):
    """Sod shock tube (Sec. 6.1): rho,p = 1,1 | 0.125,0.1, v = 0, on [0,1] with outflow ends.

    With N even the interface x0 = 0.5 lies on a cell face, so no cell is mixed.
    """
    ps = make_patchset(1, [[N, 1, 1]], ng, [BC_OUTFLOW] * 6, gamma=gamma, theta=theta,
                       dx0=(1.0 / N, 1.0, 1.0))
    x = (np.arange(N) + 0.5) / N
    left = x < x0
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    z = np.zeros(N)
    U = new_arena(ps)
    ps.active(U, 0)[...] = conserved(rho, z, z, z, p, gamma).reshape(5, 1, 1, N)
    return ps, U


def advected_wave(N, ng=2, gamma=1.4, theta=1.0, amp=0.2, ndim=1, axis=0):
    """rho = 1 + amp sin(2 pi x_axis), v_axis = 1, p = 1, periodic unit box (N^ndim)."""
    n = [N if d < ndim else 1 for d in range(3)]
    dx0 = tuple(1.0 / N if d < ndim else 1.0 for d in range(3))
    ps = make_patchset(ndim, [n], ng, [BC_PERIODIC] * 6, gamma=gamma, theta=theta, dx0=dx0)
    xc = (np.arange(N) + 0.5) / N
    shape = (n[2], n[1], n[0])
    coord = [xc.reshape((1, 1, N)), xc.reshape((1, N, 1)) if ndim > 1 else 0, xc.reshape((N, 1, 1)) if ndim > 2 else 0]
    rho = np.broadcast_to(1.0 + amp * np.sin(2 * np.pi * coord[axis]), shape)
    v = [np.zeros(shape) for _ in range(3)]
    v[axis] = np.ones(shape)
    U = new_arena(ps)
    ps.active(U, 0)[...] = conserved(rho, v[0], v[1], v[2], np.ones(shape), gamma)
    return ps, U


# ---------------------------------------------------------------- MHD set-ups
def brio_wu(N=200, ng=2, gamma=2.0, theta=1.0, x0=0.5):
    """Brio-Wu MHD shock tube on [0,1], outflow ends, Gamma = 2 (the paper's MHD section).

    Left: rho = 1, p = 1, v = 0, B = (0.75, 1, 0).  Right: rho = 0.125, p = 0.1, v = 0,
    B = (0.75, -1, 0) (the paper's right-state subscripts are misprinted as left ones).
    """
    ps = make_patchset(1, [[N, 1, 1]], ng, [BC_OUTFLOW] * 6, gamma=gamma, theta=theta,
                       dx0=(1.0 / N, 1.0, 1.0), nvar=NVAR_MHD)
    x = (np.arange(N) + 0.5) / N
    left = x < x0
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    By = np.where(left, 1.0, -1.0)
    z = np.zeros(N)
    U = new_arena(ps)
    ps.active(U, 0)[...] = conserved_mhd(rho, z, z, z, p, 0.75 + z, By, z, gamma).reshape(NVAR_MHD, 1, 1, N)
    return ps, U


def alfven_wave(N, ng=2, gamma=5.0 / 3.0, theta=1.0, amp=0.1, p=0.1, ndim=1, axis=0):
    """Circularly polarised Alfven wave travelling along ``axis`` of the periodic unit box.

    rho = 1, v_par = 0, B_par = 1 (Alfven speed 1), B_perp = amp (sin phi, cos phi),
    v_perp = -B_perp, phi = 2 pi x_axis.  |B_perp| is constant, so the total pressure
    is uniform and the profile translates at speed 1 without change of shape.
    """
    n = [N if d < ndim else 1 for d in range(3)]
    dx0 = tuple(1.0 / N if d < ndim else 1.0 for d in range(3))
    ps = make_patchset(ndim, [n], ng, [BC_PERIODIC] * 6, gamma=gamma, theta=theta, dx0=dx0, nvar=NVAR_MHD)
    shape = (n[2], n[1], n[0])
    xc = (np.arange(N) + 0.5) / N
    sh = [1, 1, 1]
    sh[2 - axis] = N
    phi = np.broadcast_to(2 * np.pi * xc.reshape(sh), shape)
    b1, b2 = (axis + 1) % 3, (axis + 2) % 3
    B = [np.zeros(shape) for _ in range(3)]
    v = [np.zeros(shape) for _ in range(3)]
    B[axis] = np.ones(shape)
    B[b1], B[b2] = amp * np.sin(phi), amp * np.cos(phi)
    v[b1], v[b2] = -B[b1], -B[b2]
    U = new_arena(ps)
    ps.active(U, 0)[...] = conserved_mhd(np.ones(shape), v[0], v[1], v[2], p, B[0], B[1], B[2], gamma)
    return ps, U


def glm_wave(N, ch=2.0, eps=1e-4, ng=2, gamma=5.0 / 3.0, theta=1.0, ndim=1, axis=0):
    """GLM cleaning wave on the periodic unit box: rho = 1, p = 1, v = 0, the field along ``axis``
    B_a = eps sin(2 pi x_a), psi = 0, no other field.  To first order in eps the pair (B_a, psi)
    obeys the wave equation with speed ch: B_a = eps sin(2 pi x) cos(2 pi ch t),
    psi = -ch eps cos(2 pi x) sin(2 pi ch t) (a standing wave)."""
    n = [N if d < ndim else 1 for d in range(3)]
    dx0 = tuple(1.0 / N if d < ndim else 1.0 for d in range(3))
    ps = make_patchset(ndim, [n], ng, [BC_PERIODIC] * 6, gamma=gamma, theta=theta, dx0=dx0, nvar=NVAR_GLM)
    shape = (n[2], n[1], n[0])
    xc = (np.arange(N) + 0.5) / N
    sh = [1, 1, 1]
    sh[2 - axis] = N
    B = [np.zeros(shape) for _ in range(3)]
    B[axis] = np.broadcast_to(eps * np.sin(2 * np.pi * xc.reshape(sh)), shape)
    U = new_arena(ps)
    ps.active(U, 0)[...] = conserved_glm(np.ones(shape), 0.0, 0.0, 0.0, 1.0, B[0], B[1], B[2], 0.0, gamma)
    return ps, U


def curl_spectral(A):
    """B = curl A of a periodic vector field A[3] (arrays indexed z, y, x) on the unit box,
    differentiated in Fourier space: the result is divergence-free to round-off in the same
    spectral sense."""
    shape = A[0].shape
    ks = [2 * np.pi * np.fft.fftfreq(s, 1.0 / s) for s in shape]   # z, y, x
    KZ, KY, KX = np.meshgrid(ks[0], ks[1], ks[2], indexing="ij")
    Ax, Ay, Az = (np.fft.fftn(a) for a in A)
    Bx = 1j * (KY * Az - KZ * Ay)
    By = 1j * (KZ * Ax - KX * Az)
    Bz = 1j * (KX * Ay - KY * Ax)
    return [np.real(np.fft.ifftn(b)) for b in (Bx, By, Bz)]


def mhd_vortex_box(N=192, patch=32, seed=50, gamma=5.0 / 3.0, theta=1.0, beta=1.7, ng=3):
    """3D periodic MHD box of N^3 cells on the unit cube, as (N/patch)^3 patches with EXTERNAL faces.

    rho = 25/(36 pi), p = 5/(12 pi) (sound speed 1 at gamma 5/3), v = (-sin 2 pi y, sin 2 pi x, 0);
    B = curl A with A_i = grf(seed + i, 1 <= |k| <= 4, k^-2), scaled so that the mean plasma beta
    2 p / <|B|^2> equals ``beta``.  Run it with the root domain periodic in all three dimensions
    (domain N^3) so EXTERNAL ghosts wrap.  ``patch=None`` gives one periodic N^3 patch.
    """
    shape = (N, N, N)
    x = (np.arange(N) + 0.5) / N
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    rho0, p0 = 25.0 / (36.0 * np.pi), 5.0 / (12.0 * np.pi)
    vx, vy = -np.sin(2 * np.pi * Y), np.sin(2 * np.pi * X)
    del Z, Y, X
    A = [grf(shape, seed + i, 1.0, 4.0, 2.0) for i in range(3)]
    B = curl_spectral(A)
    del A
    scale = math.sqrt(2.0 * p0 / beta / float(np.mean(B[0] ** 2 + B[1] ** 2 + B[2] ** 2)))
    B = [scale * b for b in B]
    Uf = conserved_mhd(rho0, vx, vy, 0.0, p0, B[0], B[1], B[2], gamma)
    del B, vx, vy
    if patch is None:
        ps = make_patchset(3, [[N, N, N]], ng, [BC_PERIODIC] * 6, gamma=gamma, theta=theta,
                           dx0=(1.0 / N,) * 3, nvar=NVAR_MHD)
        U = new_arena(ps)
        ps.active(U, 0)[...] = Uf
        return ps, U
    m = N // patch
    assert m * patch == N
    los = np.array([[i * patch, j * patch, k * patch] for k in range(m) for j in range(m) for i in range(m)],
                   np.int32)
    ps = make_patchset(3, [[patch] * 3] * len(los), ng, [BC_EXTERNAL] * 6, lo=los, gamma=gamma, theta=theta,
                       dx0=(1.0 / N,) * 3, nvar=NVAR_MHD)
    U = new_arena(ps)
    for p, lo in enumerate(los):
        ps.active(U, p)[...] = Uf[:, lo[2]:lo[2] + patch, lo[1]:lo[1] + patch, lo[0]:lo[0] + patch]
    return ps, U


# ---------------------------------------------------------------- random fields
def grf(shape, seed, kmin=1.0, kmax=16.0, alpha=2.0):
    """Gaussian random field on a periodic grid of ``shape`` (z, y, x).

    White N(0,1) noise (PCG64 ``default_rng(seed)``) -> rFFT -> multiply by
    |k|^(-alpha/2) for kmin <= |k| <= kmax (integer wave-vector components,
    Euclidean norm) and 0 elsewhere -> inverse FFT -> zero mean, unit rms.
    Per-mode power is therefore proportional to |k|^-alpha.
    """
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(shape)
    f = np.fft.rfftn(w)
    ks = [np.fft.fftfreq(s, 1.0 / s) for s in shape[:-1]] + [np.fft.rfftfreq(shape[-1], 1.0 / shape[-1])]
    kk = np.zeros(f.shape)
    for ax, k in enumerate(ks):
        sh = [1] * len(shape)
        sh[ax] = -1
        kk = kk + k.reshape(sh) ** 2
    kmag = np.sqrt(kk)
    band = (kmag >= kmin) & (kmag <= kmax)
    filt = np.zeros_like(kmag)
    filt[band] = kmag[band] ** (-alpha / 2.0)
    g = np.fft.irfftn(f * filt, s=shape, axes=tuple(range(len(shape))))
    g -= g.mean()
    g /= np.sqrt(np.mean(g * g))
    return g


def periodic_turbulent_box(N=256, seed=20, gamma=5.0 / 3.0, theta=1.0, mach=0.5, ng=2, kmax=16.0,
                           patch=None):
    """3D periodic unit box, rho = 1 + 0.1 g, v_d = A g_d (rms |v| = mach * c_s0), p = 1.

    g, g_x, g_y, g_z are :func:`grf` fields with seeds seed..seed+3 in 1 <= |k| <= kmax.
    ``patch=None`` gives one N^3 patch with periodic faces; ``patch=P`` splits the
    box into (N/P)^3 patches of P^3 whose faces are EXTERNAL (sibling ghosts).
    """
    shape = (N, N, N)
    rho = 1.0 + 0.1 * grf(shape, seed, 1.0, kmax)
    cs0 = math.sqrt(gamma * 1.0 / 1.0)
    A = mach * cs0 / math.sqrt(3.0)
    vx, vy, vz = (A * grf(shape, seed + 1 + i, 1.0, kmax) for i in range(3))
    U5 = conserved(rho, vx, vy, vz, np.ones(shape), gamma)
    if patch is None:
        ps = make_patchset(3, [[N, N, N]], ng, [BC_PERIODIC] * 6, gamma=gamma, theta=theta,
                           dx0=(1.0 / N,) * 3)
        U = new_arena(ps)
        ps.active(U, 0)[...] = U5
        return ps, U
    m = N // patch
    assert m * patch == N
    los = np.array([[i * patch, j * patch, k * patch] for k in range(m) for j in range(m) for i in range(m)],
                   np.int32)
    ps = make_patchset(3, [[patch] * 3] * len(los), ng, [BC_EXTERNAL] * 6, lo=los, gamma=gamma, theta=theta,
                       dx0=(1.0 / N,) * 3)
    U = new_arena(ps)
    for p, lo in enumerate(los):
        ps.active(U, p)[...] = U5[:, lo[2]:lo[2] + patch, lo[1]:lo[1] + patch, lo[0]:lo[0] + patch]
    return ps, U


def random_state(ps: PatchSet, seed, U=None, amp=0.3, vamp=0.5, shocks=0.0, bamp=0.5):
    """Smooth random state on every patch of ``ps`` (see :func:`uneven_patches`).

    For an MHD patch set each field component is ``bamp`` S (drawn after the hydro fields, so
    the hydro fields match those of a hydro set with the same seed).  This B is not
    divergence-free; it exercises every term of the MHD flux."""
    rng = np.random.default_rng(seed)
    g = ps.gamma
    U = new_arena(ps) if U is None else U
    for p in range(ps.npatch):
        n = ps.n[p]
        xi = [(np.arange(int(n[d])) + 0.5) / int(n[d]) for d in range(3)]
        Z, Y, X = np.meshgrid(xi[2], xi[1], xi[0], indexing="ij")
        pos = np.stack([X, Y, Z])

        def S():
            tot = np.zeros(X.shape)
            for _ in range(3):
                while True:
                    k = rng.integers(-2, 3, size=3)
                    k[ps.ndim:] = 0
                    if 0 < (k * k).sum() <= 4:
                        break
                ph = rng.uniform(0, 2 * np.pi)
                tot += np.sin(2 * np.pi * np.tensordot(k, pos, axes=1) + ph)
            return tot / 3.0

        rho = 1.0 + amp * S()
        vel = [vamp * S() if d < ps.ndim else np.zeros(X.shape) for d in range(3)]
        pr = 1.0 + amp * S()
        if shocks > 0 and rng.uniform() < shocks:
            nv = rng.standard_normal(3)
            nv[ps.ndim:] = 0
            nv /= np.linalg.norm(nv)
            x0 = rng.uniform(0.25, 0.75, size=3)
            down = np.tensordot(nv, pos - x0.reshape(3, 1, 1, 1), axes=1) < 0
            # Rankine-Hugoniot jump of pressure ratio 10 into the local pre-shock state
            p2 = 10.0 * pr
            ratio = ((g + 1) * 10.0 + (g - 1)) / ((g - 1) * 10.0 + (g + 1))
            A = 2.0 / ((g + 1) * rho)
            B = (g - 1) * pr / (g + 1)
            du = (p2 - pr) * np.sqrt(A / (p2 + B))
            for d in range(3):
                vel[d] = np.where(down, vel[d] + du * nv[d], vel[d])
            rho = np.where(down, rho * ratio, rho)
            pr = np.where(down, p2, pr)
        if ps.nvar == NVAR_MHD:
            B = [bamp * S() for _ in range(3)]
            ps.active(U, p)[...] = conserved_mhd(rho, vel[0], vel[1], vel[2], pr, B[0], B[1], B[2], g)
        elif ps.nvar == NVAR_GLM:
            B = [bamp * S() for _ in range(3)]
            ps.active(U, p)[...] = conserved_glm(rho, vel[0], vel[1], vel[2], pr, B[0], B[1], B[2], bamp * S(), g)
        else:
            ps.active(U, p)[...] = conserved(rho, vel[0], vel[1], vel[2], pr, g)
    return U


def uneven_patches(npatch=4000, seed=30, sizes=(8, 16, 24, 32), ng=3, gamma=5.0 / 3.0, theta=1.0,
                   dx=1.0 / 64, shock_frac=0.2, with_state=True):
    """Independent patches with each n_d drawn uniformly from ``sizes`` (seeded).

    Outflow on every face.  State per patch in local coordinates xi in [0,1]^3:
    rho = 1 + 0.2 S, v_d = 0.3 S, p = 1 + 0.2 S, each S the mean of 3 sinusoids
    with random integer wave vectors (|k| <= 2) and phases; a Bernoulli(shock_frac)
    subset gets a planar shock of pressure ratio 10 (normal uniform on the sphere,
    through a uniform point of the central half of the patch).
    """
    rng = np.random.default_rng(seed)
    n = rng.choice(np.asarray(sizes, np.int32), size=(npatch, 3))
    ps = make_patchset(3, n, ng, [BC_OUTFLOW] * 6, gamma=gamma, theta=theta, dx0=(dx, dx, dx))
    if not with_state:
        return ps, None
    U = random_state(ps, seed + 1, amp=0.2, vamp=0.3, shocks=shock_frac)
    return ps, U


def _with_fields(rho, vel, pr, gamma, nvar, field, bamp, uniform):
    """Conserved state of the smooth set-ups: hydro (nvar 5), or with a magnetic field
    B = B0 + bamp * field() per component, B0 = (0.6, -0.4, 0.3) (nvar 8), and a cleaning
    field psi = 0.1 * field() (nvar 9).  The draws follow the hydro ones, so the hydro
    state of a seed is the same for every nvar; a uniform set-up has B = B0, psi = 0."""
    if nvar == NVAR:
        return conserved(rho, vel[0], vel[1], vel[2], pr, gamma)
    B0 = (0.6, -0.4, 0.3)
    if uniform:
        B = [np.full(rho.shape, b) for b in B0]
        psi = np.zeros(rho.shape)
    else:
        B = [b + bamp * field() for b in B0]
        psi = 0.1 * field() if nvar == NVAR_GLM else None
    if nvar == NVAR_MHD:
        return conserved_mhd(rho, vel[0], vel[1], vel[2], pr, B[0], B[1], B[2], gamma)
    return conserved_glm(rho, vel[0], vel[1], vel[2], pr, B[0], B[1], B[2], psi, gamma)


def two_level_box(Nc=16, fine_lo=(4, 4, 4), fine_n=(8, 8, 8), ng=3, gamma=5.0 / 3.0, theta=1.0, seed=40,
                  ndim=3, amp=0.2, vamp=0.4, uniform=False, coarse_split=1, nvar=NVAR, bamp=0.3):
    """A periodic box of Nc^ndim root cells with one level-1 patch (refinement 2).

    The fine patch covers root cells [fine_lo, fine_lo + fine_n) (even bounds).
    The state is a smooth periodic field given on the level-1 grid of the whole
    domain; root cells are the means of their 2^ndim children, so the initial
    hierarchy is consistent.  Root patches: the box cut into coarse_split^ndim
    patches with EXTERNAL faces (periodic root domain); the fine patch has
    EXTERNAL faces everywhere (ghosts from the root level by prolongation).
    nvar 8 / 9: MHD / GLM-MHD, B (and psi) smooth fields of the same kind (see _mhd_fields).
    Returns (PatchSet, U, periodic_mask, domain).
    """
    Nf = 2 * Nc
    rng = np.random.default_rng(seed)
    shape_f = tuple(Nf if d < ndim else 1 for d in (2, 1, 0))
    xs = [(np.arange(Nf if d < ndim else 1) + 0.5) / Nf for d in range(3)]
    Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    pos = [X, Y, Z]

    def field():
        tot = np.zeros(shape_f)
        for _ in range(3):
            k = rng.integers(-2, 3, size=3)
            k[ndim:] = 0
            if not k.any():
                k[0] = 1
            ph = rng.uniform(0, 2 * np.pi)
            tot += np.sin(2 * np.pi * (k[0] * pos[0] + k[1] * pos[1] + k[2] * pos[2]) + ph)
        return tot / 3.0

    if uniform:
        rho = np.full(shape_f, 1.3)
        vel = [np.full(shape_f, 0.3), np.full(shape_f, -0.2 if ndim > 1 else 0.0), np.full(shape_f, 0.1 if ndim > 2 else 0.0)]
        pr = np.full(shape_f, 0.8)
    else:
        rho = 1.0 + amp * field()
        vel = [vamp * field() if d < ndim else np.zeros(shape_f) for d in range(3)]
        pr = 1.0 + amp * field()
    Uf = _with_fields(rho, vel, pr, gamma, nvar, field, bamp, uniform)
    # root field: mean of the 2^ndim children
    Uc = Uf
    for ax in range(ndim):
        axis = 3 - ax
        sl0 = [slice(None)] * 4
        sl1 = [slice(None)] * 4
        sl0[axis] = slice(0, None, 2)
        sl1[axis] = slice(1, None, 2)
        Uc = Uc[tuple(sl0)] + Uc[tuple(sl1)]
    Uc = Uc / float(2 ** ndim)
    m = coarse_split
    Pc = Nc // m
    los, ns, levels, bcs = [], [], [], []
    rng_idx = [range(m) if d < ndim else range(1) for d in range(3)]
    for kz in rng_idx[2]:
        for jy in rng_idx[1]:
            for ix in rng_idx[0]:
                los.append([ix * Pc if ndim > 0 else 0, jy * Pc if ndim > 1 else 0, kz * Pc if ndim > 2 else 0])
                ns.append([Pc if d < ndim else 1 for d in range(3)])
                levels.append(0)
    flo = [2 * fine_lo[d] if d < ndim else 0 for d in range(3)]
    fn = [2 * fine_n[d] if d < ndim else 1 for d in range(3)]
    los.append(flo)
    ns.append(fn)
    levels.append(1)
    dx0 = tuple(1.0 / Nc if d < ndim else 1.0 for d in range(3))
    ps = make_patchset(ndim, ns, ng, [BC_EXTERNAL] * 6, level=levels, lo=los, gamma=gamma, theta=theta, dx0=dx0,
                       nvar=nvar)
    U = new_arena(ps)
    for p in range(ps.npatch):
        lo, n = ps.lo[p], ps.n[p]
        src = Uc if ps.level[p] == 0 else Uf
        ps.active(U, p)[...] = src[:, lo[2]:lo[2] + n[2], lo[1]:lo[1] + n[1], lo[0]:lo[0] + n[0]]
    periodic = (1 << ndim) - 1
    domain = tuple(Nc if d < ndim else 0 for d in range(3))
    return ps, U, periodic, domain


def composite_totals(ps, U):
    """Totals of the conserved variables over the composite grid (cells not covered
    by a finer patch), each cell weighted by its volume."""
    nd = ps.ndim
    tot = np.zeros(ps.nvar)
    lo = ps.lo.astype(np.int64)
    hi = lo + ps.n.astype(np.int64)
    for p in range(ps.npatch):
        l = int(ps.level[p])
        vol = np.prod([ps.dx0[d] / 2 ** l for d in range(nd)])
        a = ps.active(U, p)
        mask = np.ones(a.shape[1:], bool)
        fine = np.nonzero(ps.level == l + 1)[0]
        if len(fine):
            flo = lo[fine] // 2
            fhi = hi[fine] // 2
            olo = np.maximum(flo, lo[p])
            ohi = np.minimum(fhi, hi[p])
            hit = np.all((ohi[:, :nd] > olo[:, :nd]), axis=1)
            for q in np.nonzero(hit)[0]:
                sl = [slice(int(olo[q, d] - lo[p, d]), int(ohi[q, d] - lo[p, d])) if d < nd else slice(None)
                      for d in range(3)]
                mask[sl[2], sl[1], sl[0]] = False
        tot += vol * np.array([math.fsum(a[k][mask].ravel()) for k in range(ps.nvar)])
    return tot


def nested_box(Nc=16, boxes=((4, 12), (12, 20)), ng=3, gamma=5.0 / 3.0, theta=1.0, seed=48, ndim=3, amp=0.2,
               vamp=0.4, nvar=NVAR, bamp=0.3):
    """A periodic root box of Nc^ndim cells with a chain of nested refined patches.

    boxes[i] = (lo, hi): level i+1 patch covering level-i cells [lo, hi) in every
    active dimension (hi - lo even).  The state is a smooth periodic field given on
    the finest grid of the whole domain; coarser cells are means of their children.
    The root level is one patch with EXTERNAL faces (periodic root domain).
    Returns (PatchSet, U, periodic_mask, domain).
    """
    nlev = len(boxes) + 1
    Nf = Nc << (nlev - 1)
    rng = np.random.default_rng(seed)
    shape_f = tuple(Nf if d < ndim else 1 for d in (2, 1, 0))
    xs = [(np.arange(Nf if d < ndim else 1) + 0.5) / Nf for d in range(3)]
    Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")

    def field():
        tot = np.zeros(shape_f)
        for _ in range(3):
            k = rng.integers(-2, 3, size=3)
            k[ndim:] = 0
            if not k.any():
                k[0] = 1
            tot += np.sin(2 * np.pi * (k[0] * X + k[1] * Y + k[2] * Z) + rng.uniform(0, 2 * np.pi))
        return tot / 3.0

    rho = 1.0 + amp * field()
    vel = [vamp * field() if d < ndim else np.zeros(shape_f) for d in range(3)]
    pr = 1.0 + amp * field()
    fields = [_with_fields(rho, vel, pr, gamma, nvar, field, bamp, False)]  # finest first
    for _ in range(nlev - 1):
        Uc = fields[-1]
        for ax in range(ndim):
            axis = 3 - ax
            s0 = [slice(None)] * 4
            s1 = [slice(None)] * 4
            s0[axis] = slice(0, None, 2)
            s1[axis] = slice(1, None, 2)
            Uc = Uc[tuple(s0)] + Uc[tuple(s1)]
        fields.append(Uc / float(2 ** ndim))
    fields = fields[::-1]  # level 0 first
    los, ns, levels = [[0, 0, 0]], [[Nc if d < ndim else 1 for d in range(3)]], [0]
    for i, (lo, hi) in enumerate(boxes):
        los.append([2 * lo if d < ndim else 0 for d in range(3)])
        ns.append([2 * (hi - lo) if d < ndim else 1 for d in range(3)])
        levels.append(i + 1)
    dx0 = tuple(1.0 / Nc if d < ndim else 1.0 for d in range(3))
    ps = make_patchset(ndim, ns, ng, [BC_EXTERNAL] * 6, level=levels, lo=los, gamma=gamma, theta=theta, dx0=dx0,
                       nvar=nvar)
    U = new_arena(ps)
    for p in range(ps.npatch):
        lo, n = ps.lo[p], ps.n[p]
        src = fields[int(ps.level[p])]
        ps.active(U, p)[...] = src[:, lo[2]:lo[2] + n[2], lo[1]:lo[1] + n[1], lo[0]:lo[0] + n[0]]
    return ps, U, (1 << ndim) - 1, tuple(Nc if d < ndim else 0 for d in range(3))


# ---------------------------------------------------------------- Sedov-Taylor blast
class SedovSolution:
    """Self-similar point explosion in a uniform gas (Sedov 1959), spherical.

    Parametric closed form in the similarity variable V (velocity v = 2 r V / (5 t)),
    running from V = 2/(gamma+1) at the shock (xi = r/R = 1) to V -> 1/gamma at
    the centre:
      xi^5 = [(g+1)V/2]^-2 [(g+1)(5-(3g-1)V)/(7-g)]^n1 [(g+1)(gV-1)/(g-1)]^n2
      rho/rho1 = (g+1)/(g-1) [(g+1)(gV-1)/(g-1)]^n3 [(g+1)(5-(3g-1)V)/(7-g)]^n4
                 [(g+1)(1-V)/(g-1)]^n5
      c^2 = (4 r^2 / 25 t^2) g (g-1) (1-V) V^2 / (2 (gV-1)),  p = rho c^2 / g
    with n1 = -(13g^2-7g+12)/((3g-1)(2g+1)), n2 = 5(g-1)/(2g+1), n3 = 3/(2g+1),
    n4 = -n1/(2-g), n5 = -2/(2-g).  The shock radius is R = xi0 (E t^2/rho1)^(1/5)
    with xi0^5 = 25 / (16 pi I), I = int_0^1 (rho/rho1) xi^4 (V^2/2 + Z/(g(g-1))) dxi.
    """

    def __init__(self, gamma=5.0 / 3.0, npts=40000):
        g = gamma
        self.gamma = g
        n1 = -(13 * g * g - 7 * g + 12) / ((3 * g - 1) * (2 * g + 1))
        n2 = 5 * (g - 1) / (2 * g + 1)
        n3 = 3 / (2 * g + 1)
        n4 = -n1 / (2 - g)
        n5 = -2 / (2 - g)
        Vs, Vc = 2 / (g + 1), 1 / g
        u = np.linspace(0.0, 1.0, npts + 1)[1:]
        V = Vc + (Vs - Vc) * np.maximum(u ** 6, 1e-12)  # dense towards the centre (V > 1/gamma)
        a = (g + 1) * V / 2
        b = (g + 1) * (5 - (3 * g - 1) * V) / (7 - g)
        c = (g + 1) * (g * V - 1) / (g - 1)
        d = (g + 1) * (1 - V) / (g - 1)
        xi = (a ** -2 * b ** n1 * c ** n2) ** 0.2
        G = (g + 1) / (g - 1) * c ** n3 * b ** n4 * d ** n5
        Z = g * (g - 1) * (1 - V) * V * V / (2 * (g * V - 1))
        order = np.argsort(xi)
        self.xi, self.G, self.V, self.Z = xi[order], G[order], V[order], Z[order]
        f = self.G * self.xi ** 4 * (self.V ** 2 / 2 + self.Z / (g * (g - 1)))
        xs = np.concatenate([[0.0], self.xi])
        fs = np.concatenate([[0.0], f])
        self.I = float(np.trapezoid(fs, xs))
        self.xi0 = (25.0 / (16.0 * np.pi * self.I)) ** 0.2

    def radius(self, E, t, rho1=1.0):
        return self.xi0 * (E * t * t / rho1) ** 0.2

    def state(self, r, E, t, rho1=1.0, p1=1e-5, rho_floor=0.0):
        """(rho, radial velocity, p) at radii r (array), ambient outside the shock."""
        R = self.radius(E, t, rho1)
        r = np.asarray(r, np.float64)
        xi = r / R
        inside = xi < 1.0
        xq = np.clip(xi, self.xi[0], 1.0)
        G = np.interp(xq, self.xi, self.G)
        V = np.interp(xq, self.xi, self.V)
        Z = np.interp(xq, self.xi, self.Z)
        rho = np.where(inside, rho1 * G, rho1)
        vel = np.where(inside, 2 * r / (5 * t) * V, 0.0)
        c2 = 4 * r * r / (25 * t * t) * Z
        p = np.where(inside, np.maximum(rho1 * G * c2 / self.gamma, p1), p1)
        if rho_floor > 0:
            rho = np.maximum(rho, rho_floor)
        return rho, vel, p


def sedov_uniform(N=64, t0=0.01, E=1.0, gamma=5.0 / 3.0, rho1=1.0, p1=1e-5, nvar=NVAR, B0=0.0, ng=2, sub=2):
    """Point explosion on a uniform N^3 grid of the cube [-1/2, 1/2]^3 (one patch, outflow faces),
    initialised with the self-similar profile at time t0 (blast energy E at the centre), each cell
    the mean of sub^3 samples.  nvar 8 makes an ideal-MHD set-up with the uniform field (B0, 0, 0)
    (the uniform-grid MHD blast of the paper's MHD section), nvar 9 the same with psi = 0; B0 = 0
    keeps the hydro solution.
    Returns (PatchSet, U, SedovSolution)."""
    sol = SedovSolution(gamma)
    ps = make_patchset(3, [[N, N, N]], ng, [BC_OUTFLOW] * 6, gamma=gamma, dx0=(1.0 / N,) * 3, nvar=nvar)
    off = (np.arange(sub) + 0.5) / sub - 0.5
    xc = (np.arange(N) + 0.5) / N - 0.5
    rho = np.zeros((N, N, N))
    mom = np.zeros((3, N, N, N))
    En = np.zeros((N, N, N))
    for oz in off:
        for oy in off:
            for ox in off:
                Z, Y, X = np.meshgrid(xc + oz / N, xc + oy / N, xc + ox / N, indexing="ij")
                r = np.sqrt(X * X + Y * Y + Z * Z)
                d, vr, p = sol.state(r, E, t0, rho1, p1)
                rs = np.maximum(r, 1e-300)
                rho += d
                for k, c in enumerate((X, Y, Z)):
                    mom[k] += d * vr * c / rs
                En += p / (gamma - 1.0) + 0.5 * d * vr * vr
    n = float(sub ** 3)
    rho, mom, En = rho / n, mom / n, En / n
    U = new_arena(ps)
    a = ps.active(U, 0)
    a[0], a[1], a[2], a[3], a[4] = rho, mom[0], mom[1], mom[2], En
    if nvar >= NVAR_MHD:
        a[4] += 0.5 * B0 * B0
        a[5], a[6], a[7] = B0, 0.0, 0.0
    if nvar == NVAR_GLM:
        a[8] = 0.0
    return ps, U, sol


def shock_radius(ps, U):
    """Shock radius of a centred blast on a single-patch cube: the shell-averaged density profile
    (shells one cell wide) is followed outward from its peak to where it falls half way to the
    ambient density, interpolated linearly between shells."""
    a = ps.active(U, 0)
    N = int(ps.n[0, 0])
    xc = (np.arange(N) + 0.5) / N - 0.5
    Z, Y, X = np.meshgrid(xc, xc, xc, indexing="ij")
    r = np.sqrt(X * X + Y * Y + Z * Z).ravel()
    k = np.minimum((r * N).astype(int), N)
    cnt = np.bincount(k, minlength=N + 1).astype(float)
    prof = np.bincount(k, weights=a[0].ravel(), minlength=N + 1) / np.maximum(cnt, 1.0)
    rmid = (np.arange(N + 1) + 0.5) / N
    valid = np.nonzero(rmid < 0.5)[0]
    i0 = int(valid[np.argmax(prof[valid])])
    amb = prof[valid[-1]]
    half = 0.5 * (prof[i0] + amb)
    for i in range(i0, valid[-1]):
        if prof[i] >= half > prof[i + 1]:
            return float(rmid[i] + (prof[i] - half) / (prof[i] - prof[i + 1]) / N)
    return float("nan")


# Floors on recovered primitives for the Sedov set-up (ambient specific internal energy is
# 1.5e-5).  A fixed hierarchy lets the Mach > 1000 shock cross coarse/fine interfaces,
# where prolongation and refluxing can leave a cell with negative internal energy; the
# floor keeps the wave speeds and fluxes of such a cell defined, as pressure floors do
# in production AMR codes.  Floors never modify U.
SEDOV_FLOORS = dict(rho_floor=1e-6, e_floor=1e-9)


def sedov_hierarchy(root=64, levels=6, t=0.05, E_octant=1.0, gamma=5.0 / 3.0, eps=0.3, ng=3, rho_floor=1e-2,
                    p1=1e-5, block=32, brick=8, samples=2, with_state=True):
    """Octant Sedov blast on [0,1]^3 (blast at the corner origin), root^3 cells plus
    `levels` levels of factor-2 refinement placed by a density-gradient criterion on
    the analytic profile at time t (E = E_octant in the octant, i.e. 8 E_octant in the
    full sphere; rho = 1, p = p1 ambient; density floored at rho_floor).

    Level l+1 is built from level l: a covered level-l cell is flagged where the
    largest relative density jump to a face neighbour, |d rho| / min rho, exceeds
    eps; fine 8^3 bricks holding children of flagged cells (dilated by one cell) are
    kept if their footprint, dilated by one coarse cell, is covered by level l (proper
    nesting: ghost cells and their prolongation stencils stay on level l).  Kept
    bricks are grouped into aligned 32^3 blocks; a block's patch is the bounding box
    of its bricks (8..32 cells per dimension), split into 16^3 sub-blocks or single
    bricks where the box would break the nesting.  Faces on x=0, y=0, z=0 reflect,
    far faces are outflow, faces between patches are EXTERNAL.
    Returns (PatchSet, U or None, periodic=0, domain).
    """
    sol = SedovSolution(gamma)
    E = 8.0 * E_octant

    def rho_at(x, y, z):
        r = np.sqrt(x * x + y * y + z * z)
        return sol.state(r, E, t, 1.0, p1, rho_floor)[0]

    def nested(cov, lo, hi, N):
        """Fine box [lo, hi) of level l+1 (cells): its footprint dilated by one coarse cell,
        clipped to the domain, lies in level-l coverage (a set of level-l bricks)."""
        clo = [max(lo[d] // 2 - 1, 0) for d in range(3)]
        chi = [min((hi[d] + 1) // 2 + 1, N) for d in range(3)]
        for bk in range(clo[2] // brick, (chi[2] - 1) // brick + 1):
            for bj in range(clo[1] // brick, (chi[1] - 1) // brick + 1):
                for bi in range(clo[0] // brick, (chi[0] - 1) // brick + 1):
                    if (bi, bj, bk) not in cov:
                        return False
        return True

    nb_root = root // brick
    bricks = [set((i, j, k) for i in range(nb_root) for j in range(nb_root) for k in range(nb_root))]
    boxes = [[((0, 0, 0), (root, root, root))]]
    per = block // brick
    for l in range(levels):
        N = root << l
        dx = 1.0 / N
        cov = bricks[l]
        cand = set()
        for (bi, bj, bk) in cov:
            ii = (np.arange(-1, brick + 1) + bi * brick + 0.5) * dx
            jj = (np.arange(-1, brick + 1) + bj * brick + 0.5) * dx
            kk = (np.arange(-1, brick + 1) + bk * brick + 0.5) * dx
            Zc, Yc, Xc = np.meshgrid(kk, jj, ii, indexing="ij")
            rho = rho_at(Xc, Yc, Zc)
            c = rho[1:-1, 1:-1, 1:-1]
            jump = np.zeros_like(c)
            for sl in ((slice(2, None), slice(1, -1), slice(1, -1)), (slice(0, -2), slice(1, -1), slice(1, -1)),
                       (slice(1, -1), slice(2, None), slice(1, -1)), (slice(1, -1), slice(0, -2), slice(1, -1)),
                       (slice(1, -1), slice(1, -1), slice(2, None)), (slice(1, -1), slice(1, -1), slice(0, -2))):
                nbv = rho[sl]
                jump = np.maximum(jump, np.abs(nbv - c) / np.minimum(nbv, c))
            fk, fj, fi = np.nonzero(jump > eps)
            if len(fi) == 0:
                continue
            ci = np.concatenate([fi + d for d in (-1, 0, 1)]) + bi * brick
            cj = np.concatenate([fj + d for d in (-1, 0, 1)]) + bj * brick
            ck = np.concatenate([fk + d for d in (-1, 0, 1)]) + bk * brick
            for a in range(3):  # dilation by one cell along each axis (cross), then to fine bricks
                arrs = [fi + bi * brick, fj + bj * brick, fk + bk * brick]
                for dd in (-1, 0, 1):
                    q = [x.copy() for x in arrs]
                    q[a] = q[a] + dd
                    ok = (q[0] >= 0) & (q[1] >= 0) & (q[2] >= 0) & (q[0] < N) & (q[1] < N) & (q[2] < N)
                    for x, y, z in zip(q[0][ok], q[1][ok], q[2][ok]):
                        cand.add(((2 * x) // brick, (2 * y) // brick, (2 * z) // brick))
            del ci, cj, ck
        Nf = N * 2
        keep = set(b for b in cand
                   if nested(cov, [b[d] * brick for d in range(3)], [(b[d] + 1) * brick for d in range(3)], N))
        # patches of level l+1
        groups = {}
        for b in keep:
            groups.setdefault((b[0] // per, b[1] // per, b[2] // per), []).append(b)
        lvl_boxes, lvl_bricks = [], set()

        def emit(bs):
            arr = np.array(bs)
            lo = tuple(int(x) for x in arr.min(axis=0) * brick)
            hi = tuple(int(x) for x in (arr.max(axis=0) + 1) * brick)
            if nested(cov, lo, hi, N):
                lvl_boxes.append((lo, hi))
                for bk in range(lo[2] // brick, hi[2] // brick):
                    for bj in range(lo[1] // brick, hi[1] // brick):
                        for bi in range(lo[0] // brick, hi[0] // brick):
                            lvl_bricks.add((bi, bj, bk))
                return True
            return False

        for key in sorted(groups):
            bs = groups[key]
            if emit(bs):
                continue
            sub = {}
            for b in bs:
                sub.setdefault(tuple((b[d] % per) // (per // 2) for d in range(3)), []).append(b)
            for sk in sorted(sub):
                if not emit(sub[sk]):
                    for b in sorted(sub[sk]):
                        emit([b])
        if not lvl_boxes:
            break
        del Nf
        bricks.append(lvl_bricks)
        boxes.append(sorted(lvl_boxes))
    # root patches: 2x2x2 blocks of (root/2)^3
    h = root // 2
    los, ns, lvls = [], [], []
    for k in range(2):
        for j in range(2):
            for i in range(2):
                los.append([i * h, j * h, k * h])
                ns.append([h, h, h])
                lvls.append(0)
    for l in range(1, len(boxes)):
        for lo, hi in boxes[l]:
            los.append(list(lo))
            ns.append([hi[d] - lo[d] for d in range(3)])
            lvls.append(l)
    los = np.array(los, np.int32)
    ns = np.array(ns, np.int32)
    lvls = np.array(lvls, np.int32)
    bcs = np.full((len(lvls), 6), BC_EXTERNAL, np.int32)
    for p in range(len(lvls)):
        N = root << int(lvls[p])
        for d in range(3):
            if los[p, d] == 0:
                bcs[p, 2 * d] = BC_REFLECT
            if los[p, d] + ns[p, d] == N:
                bcs[p, 2 * d + 1] = BC_OUTFLOW
    ps = make_patchset(3, ns, ng, bcs, level=lvls, lo=los, gamma=gamma, theta=1.0, dx0=(1.0 / root,) * 3)
    if not with_state:
        return ps, None, 0, (root, root, root)
    U = new_arena(ps)
    offs = (np.arange(samples) + 0.5) / samples - 0.5
    for p in range(ps.npatch):
        l = int(ps.level[p])
        dx = 1.0 / (root << l)
        n = ps.n[p]
        lo = ps.lo[p]
        acc = np.zeros((5, n[2], n[1], n[0]))
        for oz in offs:
            for oy in offs:
                for ox in offs:
                    x = (lo[0] + np.arange(n[0]) + 0.5 + ox) * dx
                    y = (lo[1] + np.arange(n[1]) + 0.5 + oy) * dx
                    z = (lo[2] + np.arange(n[2]) + 0.5 + oz) * dx
                    Zc, Yc, Xc = np.meshgrid(z, y, x, indexing="ij")
                    r = np.sqrt(Xc * Xc + Yc * Yc + Zc * Zc)
                    rho, vr, pr = sol.state(r, E, t, 1.0, p1, rho_floor)
                    rs = np.maximum(r, 1e-300)
                    acc += conserved(rho, vr * Xc / rs, vr * Yc / rs, vr * Zc / rs, pr, gamma)
        ps.active(U, p)[...] = acc / samples ** 3
    return ps, U, 0, (root, root, root)
