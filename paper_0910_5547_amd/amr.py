"""Python binding of the C ABI in ``include/amr_hydro.h`` (argument marshalling only).

Every function here has the name of the C entry point it calls; all of the
update's arithmetic runs in the HIP library ``libamrhydro.so`` built in-tree by
``paper_0910_5547_amd/build.py``.  PyTorch provides device memory (the U arena
and the dt scalar are CUDA/HIP tensors passed by ``data_ptr()``) and streams.
There is no fallback: if the library is missing or cannot be loaded, importing
it raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library then shares)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libamrhydro.so")

AMR_OK, AMR_EINVAL, AMR_ENOMEM, AMR_EHIP, AMR_EUNPHYSICAL, AMR_ESTATE = 0, -1, -2, -3, -4, -5
AMR_BC_OUTFLOW, AMR_BC_PERIODIC, AMR_BC_REFLECT, AMR_BC_EXTERNAL = 0, 1, 2, 3
AMR_FLUX_PAPER, AMR_FLUX_HLL2 = 0, 1
AMR_PREC_FP64, AMR_PREC_MIXED = 0, 1
AMR_EXEC_PLAIN, AMR_EXEC_BATCHED = 0, 1
AMR_RECON_E, AMR_RECON_P = 0, 1
AMR_STEP_FUSE_DT = 0x1
AMR_STEP_TIMED = 0x2
AMR_STEP_SUBSTEP1 = 0x4

EXPORTED = ("amr_patch_table_create", "amr_patch_table_destroy", "amr_table_arena_elems", "amr_cfl_dt",
            "amr_hydro_rk2_step", "amr_flux_correct", "amr_table_status", "amr_table_num_tilings",
            "amr_table_set_tiling", "amr_table_get_tiling", "amr_table_tiling_shape", "amr_autotune",
            "amr_table_last_stage_ms", "amr_hydro_advance", "amr_status_string", "amr_table_cells",
            "amr_flag_cells", "amr_cluster_flags", "amr_regrid_fill", "amr_patch_rk2_step_noalloc",
            "amr_stream_ceiling")
AMR_NOALLOC_SCRATCH_BYTES = 134217728


class amr_patch_desc(C.Structure):
    _fields_ = [("level", C.c_int32), ("lo", C.c_int32 * 3), ("n", C.c_int32 * 3), ("ng", C.c_int32),
                ("offset", C.c_int64), ("bc", C.c_int32 * 6), ("reserved", C.c_int32 * 2)]


class amr_physics(C.Structure):
    _fields_ = [("nvar", C.c_int32), ("ndim", C.c_int32), ("gamma", C.c_double), ("theta", C.c_double),
                ("dx0", C.c_double * 3), ("flux", C.c_int32), ("precision", C.c_int32), ("exec", C.c_int32),
                ("periodic", C.c_int32), ("domain", C.c_int32 * 3), ("recon", C.c_int32),
                ("rho_floor", C.c_double), ("e_floor", C.c_double), ("ch", C.c_double)]


class AmrError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {amr_status_string(status)}")


_LIB = None


def lib():
    """The loaded HIP library (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_0910_5547_amd/build.py (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        vp, dp, i32, i64 = C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_int64
        L.amr_patch_table_create.argtypes = [C.POINTER(amr_patch_desc), i32, C.POINTER(amr_physics), vp,
                                             C.POINTER(vp)]
        L.amr_patch_table_destroy.argtypes = [vp]
        L.amr_table_arena_elems.argtypes = [vp]
        L.amr_table_arena_elems.restype = i64
        L.amr_cfl_dt.argtypes = [vp, vp, C.c_double, i32, vp, dp, vp]
        L.amr_hydro_rk2_step.argtypes = [vp, vp, vp, i32, C.c_uint32, vp]
        L.amr_flux_correct.argtypes = [vp, vp, i32, vp]
        L.amr_hydro_advance.argtypes = [vp, vp, vp, C.c_uint32, vp]
        L.amr_table_status.argtypes = [vp, vp]
        L.amr_table_num_tilings.argtypes = [vp]
        L.amr_table_set_tiling.argtypes = [vp, i32, i32]
        L.amr_table_get_tiling.argtypes = [vp, C.POINTER(i32), C.POINTER(i32)]
        L.amr_table_tiling_shape.argtypes = [vp, i32, C.POINTER(i32), C.POINTER(i32)]
        L.amr_autotune.argtypes = [vp, vp, vp, i32, i32, vp, C.POINTER(C.c_float)]
        L.amr_table_last_stage_ms.argtypes = [vp, C.POINTER(C.c_float)]
        L.amr_status_string.argtypes = [i32]
        L.amr_status_string.restype = C.c_char_p
        L.amr_table_cells.argtypes = [vp, i32]
        L.amr_table_cells.restype = i64
        L.amr_flag_cells.argtypes = [vp, vp, i32, C.c_double, vp, vp]
        L.amr_regrid_fill.argtypes = [vp, vp, vp, vp, vp]
        L.amr_stream_ceiling.argtypes = [vp, vp, vp, i64, i32, vp]
        L.amr_patch_rk2_step_noalloc.argtypes = [C.POINTER(amr_patch_desc), C.POINTER(amr_physics), vp, vp, vp, vp]
        L.amr_cluster_flags.argtypes = [C.POINTER(amr_patch_desc), i32, i32, C.POINTER(i32), i32,
                                         C.POINTER(C.c_uint8), i32, i32, C.POINTER(i32), i32, C.POINTER(i32)]
        for name in EXPORTED:
            if name not in ("amr_table_arena_elems", "amr_status_string", "amr_table_cells"):
                getattr(L, name).restype = i32
        _LIB = L
    return _LIB


def amr_status_string(status: int) -> str:
    return lib().amr_status_string(int(status)).decode()


def _check(st, where):
    if st != AMR_OK:
        raise AmrError(st, where)
    return st


def _stream(stream):
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("device arrays must be contiguous float64 GPU tensors")
        return C.c_void_p(t.data_ptr())
    return C.c_void_p(int(t))


def _arena(h, U):
    """_ptr of an arena tensor, checked to hold the table's arena (U indexes up to it)."""
    if isinstance(U, torch.Tensor) and U.numel() < int(lib().amr_table_arena_elems(h)):
        raise ValueError("the arena tensor is smaller than the table's arena (amr_table_arena_elems)")
    return _ptr(U)


def descriptors(ps):
    """amr_patch_desc array of a :class:`paper_0910_5547_amd.workloads.PatchSet`."""
    arr = (amr_patch_desc * ps.npatch)()
    for p in range(ps.npatch):
        d = arr[p]
        d.level = int(ps.level[p])
        for k in range(3):
            d.lo[k] = int(ps.lo[p, k])
            d.n[k] = int(ps.n[p, k])
        d.ng = int(ps.ng[p])
        d.offset = int(ps.offset[p])
        for f in range(6):
            d.bc[f] = int(ps.bc[p, f])
    return arr


def physics(ps, precision=AMR_PREC_FP64, exec_form=AMR_EXEC_BATCHED, flux=AMR_FLUX_PAPER, theta=None,
            periodic=0, domain=(0, 0, 0), rho_floor=0.0, e_floor=0.0, recon=AMR_RECON_E, ch=0.0):
    ph = amr_physics()
    ph.nvar, ph.ndim = int(getattr(ps, "nvar", 5)), ps.ndim
    ph.gamma = ps.gamma
    ph.theta = ps.theta if theta is None else theta
    for d in range(3):
        ph.dx0[d] = ps.dx0[d]
        ph.domain[d] = int(domain[d])
    ph.flux, ph.precision, ph.exec, ph.periodic = flux, precision, exec_form, periodic
    ph.rho_floor, ph.e_floor = rho_floor, e_floor
    ph.recon = recon
    ph.ch = ch
    return ph


# ------------------------------------------------------------------ C ABI, one function each
def amr_patch_table_create(descs, phys, stream=None):
    h = C.c_void_p()
    _check(lib().amr_patch_table_create(descs, len(descs), C.byref(phys), _stream(stream), C.byref(h)),
           "amr_patch_table_create")
    return h


def amr_patch_table_destroy(h):
    return _check(lib().amr_patch_table_destroy(h), "amr_patch_table_destroy")


def amr_table_arena_elems(h):
    return int(lib().amr_table_arena_elems(h))


def amr_cfl_dt(h, U, cfl, level, dt_dev, host=False, stream=None):
    """dt into dt_dev; with host=True also returns it (synchronising)."""
    out = C.c_double(0.0)
    _check(lib().amr_cfl_dt(h, _arena(h, U), float(cfl), int(level), _ptr(dt_dev), C.byref(out) if host else None,
                            _stream(stream)), "amr_cfl_dt")
    return out.value if host else None


def amr_hydro_rk2_step(h, U, dt_dev, level=-1, flags=0, stream=None):
    return _check(lib().amr_hydro_rk2_step(h, _arena(h, U), _ptr(dt_dev), int(level), int(flags), _stream(stream)),
                  "amr_hydro_rk2_step")


def amr_flux_correct(h, U, coarse_level, stream=None):
    return _check(lib().amr_flux_correct(h, _arena(h, U), int(coarse_level), _stream(stream)), "amr_flux_correct")


def amr_hydro_advance(h, U, dt0_dev, flags=0, stream=None):
    return _check(lib().amr_hydro_advance(h, _arena(h, U), _ptr(dt0_dev), int(flags), _stream(stream)),
                  "amr_hydro_advance")


def amr_table_status(h, stream=None):
    return lib().amr_table_status(h, _stream(stream))


def amr_table_num_tilings(h):
    return int(lib().amr_table_num_tilings(h))


def amr_table_set_tiling(h, tid, zslab=0):
    return _check(lib().amr_table_set_tiling(h, int(tid), int(zslab)), "amr_table_set_tiling")


def amr_table_get_tiling(h):
    a, b = C.c_int32(), C.c_int32()
    _check(lib().amr_table_get_tiling(h, C.byref(a), C.byref(b)), "amr_table_get_tiling")
    return a.value, b.value


def amr_table_tiling_shape(h, tid):
    a, b = C.c_int32(), C.c_int32()
    _check(lib().amr_table_tiling_shape(h, int(tid), C.byref(a), C.byref(b)), "amr_table_tiling_shape")
    return a.value, b.value


def amr_autotune(h, U, dt_dev, level=-1, reps=3, stream=None):
    ms = C.c_float(0.0)
    _check(lib().amr_autotune(h, _arena(h, U), _ptr(dt_dev), int(level), int(reps), _stream(stream), C.byref(ms)),
           "amr_autotune")
    return ms.value


def amr_table_cells(h, level=-1):
    return int(lib().amr_table_cells(h, level))


def amr_flag_cells(h, U, level, eps, flags, stream=None):
    """Refinement flags of `level` into the uint8 device tensor `flags` (amr_table_cells(level) bytes)."""
    if not (flags.dtype == torch.uint8 and flags.is_cuda and flags.is_contiguous()
            and flags.numel() >= amr_table_cells(h, level)):
        raise ValueError("flags must be a contiguous uint8 GPU tensor of amr_table_cells(level) bytes")
    _check(lib().amr_flag_cells(h, _arena(h, U), level, float(eps), C.c_void_p(flags.data_ptr()), _stream(stream)),
           "amr_flag_cells")


def amr_regrid_fill(h_old, U_old, h_new, U_new, stream=None):
    _check(lib().amr_regrid_fill(h_old, _arena(h_old, U_old), h_new, _arena(h_new, U_new), _stream(stream)),
           "amr_regrid_fill")


def amr_cluster_flags(descs, ndim, domain, level, flags, brick=8, block=32):
    """Boxes (lo[3], n[3]) of level+1 clustered from the host uint8 flags of `level` (host work)."""
    flags = np.ascontiguousarray(flags, np.uint8)
    need = sum(int(d.n[0]) * int(d.n[1]) * int(d.n[2]) for d in descs if d.level == level)
    if flags.size < need:
        raise ValueError(f"flags hold {flags.size} cells, the level-{level} patches {need}")
    dom = (C.c_int32 * 3)(*[int(x) for x in domain])
    n = C.c_int32(0)
    cap = 1024
    while True:
        out = np.zeros(6 * cap, np.int32)
        st = lib().amr_cluster_flags(descs, len(descs), ndim, dom, level,
                                     flags.ctypes.data_as(C.POINTER(C.c_uint8)), brick, block,
                                     out.ctypes.data_as(C.POINTER(C.c_int32)), cap, C.byref(n))
        if st == AMR_OK:
            return out[:6 * n.value].reshape(-1, 6)
        if n.value > cap:
            cap = n.value
            continue
        _check(st, "amr_cluster_flags")


def amr_patch_rk2_step_noalloc(desc, phys, U, dt_dev, flag_dev, stream=None):
    """One RK2 step of the lone patch `desc` (an amr_patch_desc) with the library's static
    scratch; flag_dev is an int32 device tensor the step sets nonzero on an unphysical state."""
    if not (flag_dev.dtype == torch.int32 and flag_dev.is_cuda and flag_dev.numel() >= 1):
        raise ValueError("flag_dev must be an int32 GPU tensor")
    return _check(lib().amr_patch_rk2_step_noalloc(C.byref(desc), C.byref(phys), _ptr(U), _ptr(dt_dev),
                                                   C.c_void_p(flag_dev.data_ptr()), _stream(stream)),
                  "amr_patch_rk2_step_noalloc")


def amr_stream_ceiling(a, b, out, n, wg_per_cu=0, stream=None):
    """out[:n] = (a[:n] + b[:n]) / 2 on the device (the streaming ceiling's kernel)."""
    for t in (a, b, out):
        if t.numel() < n:
            raise ValueError("arrays shorter than n")
    return _check(lib().amr_stream_ceiling(_ptr(a), _ptr(b), _ptr(out), int(n), int(wg_per_cu), _stream(stream)),
                  "amr_stream_ceiling")


def amr_table_last_stage_ms(h):
    ms = (C.c_float * 2)()
    _check(lib().amr_table_last_stage_ms(h, ms), "amr_table_last_stage_ms")
    return float(ms[0]), float(ms[1])


# ------------------------------------------------------------------ convenience
class Table:
    """Owns one amr_table for a PatchSet; U arenas are float64 device tensors."""

    def __init__(self, ps, precision=AMR_PREC_FP64, exec_form=AMR_EXEC_BATCHED, flux=AMR_FLUX_PAPER, theta=None,
                 periodic=0, domain=(0, 0, 0), rho_floor=0.0, e_floor=0.0, recon=AMR_RECON_E, ch=0.0,
                 device="cuda"):
        self.ps = ps
        self.device = torch.device(device)
        self.descs = descriptors(ps)
        self.phys = physics(ps, precision, exec_form, flux, theta, periodic, domain, rho_floor, e_floor, recon, ch)
        self.h = amr_patch_table_create(self.descs, self.phys)
        self.arena = amr_table_arena_elems(self.h)
        self.dt = torch.zeros(1, dtype=torch.float64, device=self.device)

    def upload(self, U_host: np.ndarray) -> torch.Tensor:
        assert U_host.dtype == np.float64 and U_host.size >= self.arena
        return torch.from_numpy(np.ascontiguousarray(U_host)).to(self.device)

    def cfl_dt(self, U, cfl=0.8, level=-1, host=True):
        return amr_cfl_dt(self.h, U, cfl, level, self.dt, host=host)

    def step(self, U, dt=None, level=-1, flags=0):
        if dt is not None:
            self.dt.fill_(float(dt))
        amr_hydro_rk2_step(self.h, U, self.dt, level, flags)

    def advance(self, U, dt0=None):
        """One subcycled root step of the hierarchy (dt0 from the last cfl_dt unless given)."""
        if dt0 is not None:
            self.dt.fill_(float(dt0))
        amr_hydro_advance(self.h, U, self.dt)

    def status(self):
        return amr_table_status(self.h)

    def close(self):
        if self.h is not None:
            amr_patch_table_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
