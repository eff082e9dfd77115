"""ctypes front end of the FP64 CPU oracle (``oracle/liboracle.so``).

TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the CPU
baseline of the benchmark.  The product path never imports this module.

The arithmetic lives in ``oracle.c`` (serial FP64, one IEEE operation per
source operation, no FMA contraction); this file marshals a
:class:`paper_0910_5547_amd.workloads.PatchSet` into the oracle's own
metadata rows and drives time loops.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

FLUX_PAPER, FLUX_HLL2 = 0, 1


class Phys(C.Structure):
    _fields_ = [("nvar", C.c_int32), ("ndim", C.c_int32), ("gamma", C.c_double), ("theta", C.c_double),
                ("dx0", C.c_double * 3), ("flux", C.c_int32), ("periodic", C.c_int32),
                ("domain", C.c_int32 * 3), ("pad", C.c_int32),
                ("rho_floor", C.c_double), ("e_floor", C.c_double)]


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b  # noqa: F401  (plain build of the C source)
            _b.build()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        lp = C.POINTER(C.c_int64)
        pp = C.POINTER(Phys)
        L.or_minmod3.restype = C.c_double
        L.or_minmod3.argtypes = [C.c_double] * 3
        L.or_prim.argtypes = [pp, dp, dp]
        L.or_face_flux.argtypes = [pp, C.c_int, dp, dp, dp]
        L.or_face_flux.restype = None
        L.or_phys_flux.argtypes = [pp, C.c_int, dp, dp]
        L.or_phys_flux.restype = None
        L.or_fill_ghosts.argtypes = [C.c_int32, ip, lp, pp, dp, C.c_int32]
        L.or_patch_L.argtypes = [ip, C.c_int64, pp, dp, dp]
        L.or_stage.argtypes = [C.c_int32, ip, lp, pp, dp, dp, dp, C.c_double, C.c_int32, C.c_int32]
        L.or_rk2_step.argtypes = [C.c_int32, ip, lp, pp, dp, dp, C.c_double, C.c_int32]
        L.or_max_speed.restype = C.c_double
        L.or_max_speed.argtypes = [C.c_int32, ip, lp, pp, dp, C.c_int32, C.POINTER(C.c_int)]
        L.or_cfl_dt.restype = C.c_double
        L.or_cfl_dt.argtypes = [C.c_int32, ip, lp, pp, dp, C.c_double, C.c_int32]
        _LIB = L
    return _LIB


def _dp(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def phys(gamma=1.4, theta=1.0, ndim=3, dx0=(1.0, 1.0, 1.0), flux=FLUX_PAPER, rho_floor=0.0, e_floor=0.0,
         periodic=0, domain=(0, 0, 0)):
    ph = Phys()
    ph.nvar, ph.ndim, ph.gamma, ph.theta = 5, ndim, gamma, theta
    ph.periodic = periodic
    for d in range(3):
        ph.dx0[d] = dx0[d]
        ph.domain[d] = int(domain[d])
    ph.flux, ph.rho_floor, ph.e_floor = flux, rho_floor, e_floor
    return ph


def minmod3(a, b, c):
    return lib().or_minmod3(a, b, c)


def prim(ph, U5):
    U5 = np.ascontiguousarray(U5, np.float64)
    q = np.zeros(6)
    bad = lib().or_prim(C.byref(ph), _dp(U5), _dp(q))
    return q, bad


def face_flux(ph, d, qL, qR):
    qL = np.ascontiguousarray(qL, np.float64)
    qR = np.ascontiguousarray(qR, np.float64)
    F = np.zeros(5)
    lib().or_face_flux(C.byref(ph), d, _dp(qL), _dp(qR), _dp(F))
    return F


def phys_flux(ph, d, q):
    q = np.ascontiguousarray(q, np.float64)
    F = np.zeros(5)
    lib().or_phys_flux(C.byref(ph), d, _dp(q), _dp(F))
    return F


class Oracle:
    """Oracle bound to one patch table.  All arrays are FP64 arenas laid out as ``ps``."""

    def __init__(self, ps, flux=FLUX_PAPER, rho_floor=0.0, e_floor=0.0, theta=None, periodic=0, domain=(0, 0, 0)):
        self.ps = ps
        self.ph = phys(ps.gamma, ps.theta if theta is None else theta, ps.ndim, ps.dx0, flux, rho_floor, e_floor,
                       periodic, domain)
        self.meta = np.ascontiguousarray(ps.meta(), np.int32)
        self.off = np.ascontiguousarray(ps.offset, np.int64)
        self._W = None

    def _args(self):
        return (self.ps.npatch, self.meta.ctypes.data_as(C.POINTER(C.c_int32)),
                self.off.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(self.ph))

    def fill_ghosts(self, U, level=-1):
        lib().or_fill_ghosts(*self._args(), _dp(U), level)

    def stage(self, V, U0, out, dt, stage, level=-1):
        return lib().or_stage(*self._args(), _dp(V), _dp(U0) if U0 is not None else None, _dp(out), dt, stage,
                              level)

    def rk2_step(self, U, dt, level=-1):
        if self._W is None or self._W.shape != U.shape:
            self._W = np.full_like(U, np.nan)
        return lib().or_rk2_step(*self._args(), _dp(U), _dp(self._W), dt, level)

    def max_speed(self, U, level=-1):
        flag = C.c_int(0)
        s = lib().or_max_speed(*self._args(), _dp(U), level, C.byref(flag))
        return s, flag.value

    def cfl_dt(self, U, cfl, level=-1):
        return lib().or_cfl_dt(*self._args(), _dp(U), cfl, level)

    def run(self, U, t_end, cfl=0.8, max_steps=10 ** 7):
        """Advance U (in place) to t_end with dt = cfl_dt, the last step clipped to t_end."""
        t, steps = 0.0, 0
        while t < t_end and steps < max_steps:
            dt = self.cfl_dt(U, cfl)
            if t + dt > t_end:
                dt = t_end - t
            bad = self.rk2_step(U, dt)
            if bad:
                raise FloatingPointError(f"oracle met an unphysical state at step {steps}")
            t += dt
            steps += 1
        return steps
