"""Exact solutions used to pin the oracle (test infrastructure only).

* :func:`riemann_star` / :func:`riemann_sample` - the exact solution of the
  Riemann problem for the 1D Euler equations with an ideal gas (the Sod tube of
  Sec. 6.1 is one).  The star pressure solves f_L(p) + f_R(p) + (u_R - u_L) = 0,
  where f_K is the shock (Rankine-Hugoniot) branch for p > p_K and the
  rarefaction (isentropic, Riemann invariant) branch otherwise; it is found by
  Newton's method with a bisection safeguard.  The self-similar solution is then
  sampled at x/t.
* :func:`riemann_cell_averages` - exact cell averages by composite Gauss-Legendre
  quadrature inside each cell, splitting cells at every wave position so that
  each piece is smooth.
* :func:`wave_cell_average` - exact cell averages of 1 + a sin(2 pi (x - t)).
"""
from __future__ import annotations

import math

import numpy as np


def _fK(p, rho, pK, g):
    """Velocity jump across the K-wave as a function of the star pressure, and its derivative."""
    c = math.sqrt(g * pK / rho)
    if p > pK:  # shock: Rankine-Hugoniot
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pK
        s = math.sqrt(A / (p + B))
        return (p - pK) * s, s * (1.0 - 0.5 * (p - pK) / (p + B))
    # rarefaction: isentropic, constant Riemann invariant
    e = (g - 1.0) / (2.0 * g)
    return 2.0 * c / (g - 1.0) * ((p / pK) ** e - 1.0), (p / pK) ** (-(g + 1.0) / (2.0 * g)) / (rho * c)


def riemann_star(rhoL, uL, pL, rhoR, uR, pR, g, tol=1e-15):
    """Star-region pressure and velocity (p*, u*)."""
    du = uR - uL
    lo, hi = 0.0, max(pL, pR)
    while _fK(hi, rhoL, pL, g)[0] + _fK(hi, rhoR, pR, g)[0] + du < 0:
        hi *= 2.0
    p = 0.5 * (pL + pR)
    for _ in range(200):
        fL, dL = _fK(p, rhoL, pL, g)
        fR, dR = _fK(p, rhoR, pR, g)
        f = fL + fR + du
        if f > 0:
            hi = p
        else:
            lo = p
        pn = p - f / (dL + dR)
        if not (lo < pn < hi):
            pn = 0.5 * (lo + hi)
        if abs(pn - p) <= tol * p:
            p = pn
            break
        p = pn
    fL, _ = _fK(p, rhoL, pL, g)
    fR, _ = _fK(p, rhoR, pR, g)
    u = 0.5 * (uL + uR) + 0.5 * (fR - fL)
    return p, u


class RiemannSolution:
    """The self-similar exact solution of one Riemann problem."""

    def __init__(self, rhoL, uL, pL, rhoR, uR, pR, g):
        self.L = (rhoL, uL, pL)
        self.R = (rhoR, uR, pR)
        self.g = g
        self.p, self.u = riemann_star(rhoL, uL, pL, rhoR, uR, pR, g)
        p, u = self.p, self.u
        gm = (g - 1.0) / (g + 1.0)
        cL = math.sqrt(g * pL / rhoL)
        cR = math.sqrt(g * pR / rhoR)
        if p > pL:
            self.rhoL = rhoL * (p / pL + gm) / (gm * p / pL + 1.0)
            sL = uL - cL * math.sqrt((g + 1) / (2 * g) * p / pL + (g - 1) / (2 * g))
            self.left_waves = (sL, sL)
        else:
            self.rhoL = rhoL * (p / pL) ** (1.0 / g)
            cs = cL * (p / pL) ** ((g - 1) / (2 * g))
            self.left_waves = (uL - cL, u - cs)
        if p > pR:
            self.rhoR = rhoR * (p / pR + gm) / (gm * p / pR + 1.0)
            sR = uR + cR * math.sqrt((g + 1) / (2 * g) * p / pR + (g - 1) / (2 * g))
            self.right_waves = (sR, sR)
        else:
            self.rhoR = rhoR * (p / pR) ** (1.0 / g)
            cs = cR * (p / pR) ** ((g - 1) / (2 * g))
            self.right_waves = (u + cs, uR + cR)

    def wave_speeds(self):
        return sorted(set(self.left_waves + (self.u,) + self.right_waves))

    def sample(self, s):
        """(rho, u, p) at similarity coordinate s = (x - x0)/t (numpy array)."""
        s = np.asarray(s, np.float64)
        g = self.g
        rhoL, uL, pL = self.L
        rhoR, uR, pR = self.R
        out = np.zeros((3,) + s.shape)
        left = s < self.u
        # left side
        head, tail = self.left_waves
        cL = math.sqrt(g * pL / rhoL)
        m = left & (s < head)
        out[:, m] = np.array([rhoL, uL, pL])[:, None]
        m = left & (s >= tail)
        out[:, m] = np.array([self.rhoL, self.u, self.p])[:, None]
        m = left & (s >= head) & (s < tail)
        if m.any():  # inside the left rarefaction fan
            uf = 2.0 / (g + 1) * (cL + (g - 1) / 2 * uL + s[m])
            cf = 2.0 / (g + 1) * (cL + (g - 1) / 2 * (uL - s[m]))
            rf = rhoL * (cf / cL) ** (2.0 / (g - 1))
            out[0, m], out[1, m], out[2, m] = rf, uf, pL * (cf / cL) ** (2 * g / (g - 1))
        # right side
        tail, head = self.right_waves
        cR = math.sqrt(g * pR / rhoR)
        right = ~left
        m = right & (s > head)
        out[:, m] = np.array([rhoR, uR, pR])[:, None]
        m = right & (s <= tail)
        out[:, m] = np.array([self.rhoR, self.u, self.p])[:, None]
        m = right & (s > tail) & (s <= head)
        if m.any():
            uf = 2.0 / (g + 1) * (-cR + (g - 1) / 2 * uR + s[m])
            cf = 2.0 / (g + 1) * (cR - (g - 1) / 2 * (uR - s[m]))
            rf = rhoR * (cf / cR) ** (2.0 / (g - 1))
            out[0, m], out[1, m], out[2, m] = rf, uf, pR * (cf / cR) ** (2 * g / (g - 1))
        return out

    def cell_averages(self, N, t, x0=0.5, a=0.0, b=1.0, order=8):
        """Exact averages of (rho, rho u, rho E) over N equal cells of [a, b] at time t."""
        xg, wg = np.polynomial.legendre.leggauss(order)
        edges = np.linspace(a, b, N + 1)
        breaks = [x0 + s * t for s in self.wave_speeds()]
        out = np.zeros((3, N))
        for i in range(N):
            lo, hi = edges[i], edges[i + 1]
            pts = [lo] + [x for x in breaks if lo < x < hi] + [hi]
            acc = np.zeros(3)
            for u0, u1 in zip(pts[:-1], pts[1:]):
                x = 0.5 * (u1 - u0) * xg + 0.5 * (u1 + u0)
                r, u, p = self.sample((x - x0) / t)
                E = p / (self.g - 1) + 0.5 * r * u * u
                acc += 0.5 * (u1 - u0) * np.array([np.dot(wg, r), np.dot(wg, r * u), np.dot(wg, E)])
            out[:, i] = acc / (hi - lo)
        return out


def wave_cell_average(N, t, amp=0.2):
    """Exact cell averages of rho(x, t) = 1 + amp sin(2 pi (x - t)) on N cells of [0,1]."""
    e = np.arange(N + 1) / N
    h = 1.0 / N
    return 1.0 + amp * (np.cos(2 * np.pi * (e[:-1] - t)) - np.cos(2 * np.pi * (e[1:] - t))) / (2 * np.pi * h)
