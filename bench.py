#!/usr/bin/env python3
"""Benchmark of the per-patch hydro update: cell-updates/s of full TVD-RK2 steps.

One "step" is the whole hot path over the workload: the CFL time step (a
device-side reduction; fused into the previous step's second stage) and one
TVD-RK2 step (two stage kernels: conserved->primitive, PLM, face fluxes,
divergence, RK combine).  Inputs are resident in HBM before the timed region.

Workloads (seeded, synthetic; see paper_0910_5547_amd.workloads):
  patches4000  4000 independent patches, sizes 8..32 per dimension, 3 ghost
               layers, smooth states with random planar shocks in 20% (the
               default headline: the batched form's thousands of uneven patches)
  box256       256^3 periodic box, gamma 5/3, GRF density (k^-2, 1<=|k|<=16),
               Mach 0.5 GRF velocities, p = 1 (one patch; timed by default as an
               extra key of the same line)
  patches4000-g0  the same 4000 patches stored without ghost layers (ng = 0, their
               faces applied by index maps): timed by default as an extra key
  (boxes store no ghost layers by default; a "-g3" suffix stores three, "-g0" none)
  sedov        deep-AMR octant Sedov hierarchy (7 levels, subcycled root steps)
  glm192       the mhd192 box with the GLM cleaning field (9 variables, c_h = 3)
  sedovN       centred blast on a uniform N^3 grid (one patch); mhdsedovN: the same
               with 8 MHD variables and a uniform field (the MHD blast timing series)
  mhd192       ideal MHD (8 variables), 192^3 periodic box as 216 patches of 32^3
               with EXTERNAL faces: Orszag-Tang-like vortex velocity, B = curl of
               a seeded GRF vector potential (divergence-free), plasma beta 1.7

Three forms are timed on identical inputs: plain FP64 (one launch per patch
per stage), batched FP64 (persistent launch per stage, graph-replayed step) and
batched mixed (FP32 reconstruction and flux, FP64 accumulation).  `value` is
the batched mixed form of the headline workload.  Each form also reports its
relative L1 error against the FP64 oracle and the difference of its totals
from the oracle's, on a sample the oracle computes in seconds (a subset of the
patches, or blocks of a periodic box recomputed with their domain of
dependence), after a few steps fed the GPU's own time steps.  The line carries
the stage kernels' roofline against the 8 TB/s HBM peak and against the
measured streaming ceiling (amr_stream_ceiling: two arrays read, one written),
and the oracle's rate on one host core and on all of them.  Prints one JSON
line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0           # MI355X HBM3E
# algorithmic HBM bytes per cell-update: 5 passes x nvar variables x 8 B (stage 1: read U,
# write U1; stage 2: read U1 and U, write U^{n+1}); 200 B for hydro, 320 B for MHD
def bytes_per_cell(nvar):
    return 5 * nvar * 8


def bytes_stage(nvar):  # per active cell, stage 1 and stage 2
    return (2 * nvar * 8, 3 * nvar * 8)
METRIC = "cell-updates/s per RK2 step (batched FP32/FP64 vs plain FP64); % HBM peak"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stage_kernel_traffic.json")
COPY_BYTES = 1 << 30  # calibration copy: 1 GiB read + 1 GiB written


STAGE_SOURCES = ("amr_device.h", "amr_internal.h", "amr_stage.h", "amr_stage_hydro_f32.hip",
                 "amr_stage_hydro_f64.hip", "amr_stage_mhd.hip", "amr_stage_glm.hip", "amr_api.hip")


def kernel_source_sha():
    """Hash of the stage kernel's sources and of the host code that lays out its tiles:
    a traffic measurement is only valid for the kernels it was taken on."""
    import hashlib
    h = hashlib.sha256()
    cdir = os.path.join(ROOT, "paper_0910_5547_amd", "csrc")
    for f in STAGE_SOURCES:
        with open(os.path.join(cdir, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def traffic_for(workload, form, cells, tile):
    """Measured HBM bytes per stage launch (average of the two stages), or None when no
    measurement was taken on these kernel sources, this workload and this tile shape."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    e = t.get("entries", {}).get(f"{workload}/{form}")
    if (not e or e.get("kernel_source_sha") != kernel_source_sha() or e.get("cells") != cells
            or e.get("tile") != tile):
        return None
    return e["hbm_bytes_per_launch"]


def stage_tile(kernel_name):
    """'TXxTY' from a stage kernel's template arguments (type, variables, TX, TY, ...)."""
    import re
    m = re.search(r"stage_kernel<\w+, \d+, (\d+), (\d+),", kernel_name)
    return f"{m.group(1)}x{m.group(2)}" if m else None


def summarize_pmc(fetch_csv, write_csv, workload, form, cells, nvar=5):
    """Turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch) into HBM
    bytes per stage launch, each counter scaled by what it reads for the 1 GiB copy."""
    import csv
    import statistics

    def per_kernel(path, counter):
        vals = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return vals
    fetch, write = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    copy_f = [v for k, vs in fetch.items() if "copy" in k.lower() or "elementwise" in k.lower() for v in vs]
    copy_w = [v for k, vs in write.items() if "copy" in k.lower() or "elementwise" in k.lower() for v in vs]
    big_f = max(copy_f)
    big_w = max(copy_w)
    sf = COPY_BYTES / (big_f * 1024.0)
    sw = COPY_BYTES / (big_w * 1024.0)
    # the timed run's kernels: the tile shape with the most dispatches (the autotuner
    # tries every shape a few times first)
    counts = {}
    for k, vs in fetch.items():
        if "stage_kernel" in k:
            counts[stage_tile(k)] = counts.get(stage_tile(k), 0) + len(vs)
    main_tile = max(counts, key=counts.get)
    out = {}
    for k in fetch:
        if "stage_kernel" not in k or stage_tile(k) != main_tile:
            continue
        f = statistics.median(fetch[k]) * 1024.0 * sf
        w = statistics.median(write.get(k, [0.0])) * 1024.0 * sw
        out[k] = {"fetch_bytes": f, "write_bytes": w, "dispatches": len(fetch[k])}
    per_launch = sum(v["fetch_bytes"] + v["write_bytes"] for v in out.values()) / max(1, len(out))
    tiles = {stage_tile(k) for k in out}
    entry = {"kernel_source_sha": kernel_source_sha(), "cells": cells, "hbm_bytes_per_launch": per_launch,
             "tile": tiles.pop() if len(tiles) == 1 else None,
             "algorithmic_bytes_per_launch": bytes_per_cell(nvar) * cells / 2, "copy_scale_fetch": sf,
             "copy_scale_write": sw, "kernels": out}
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        t = {"what": "HBM bytes per stage-kernel launch from rocprofv3 FETCH_SIZE/WRITE_SIZE, scaled by a 1 GiB copy",
             "entries": {}}
    t["entries"][f"{workload}/{form}"] = entry
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(t, fh, indent=1)
    return entry


# Ghost layers stored per patch face: the 4000-patch configuration states three; the
# boxes (one periodic patch, or patches whose faces read their siblings directly) need
# none stored, their ghost cells being index maps or sibling reads.
DEFAULT_NG = {"patches4000": 3, "box256": 0, "mhd192": 0, "glm192": 0}


def make_workload(name):
    """(PatchSet, U, description, extra Table arguments) of a named workload.  A name ending
    in "-g0" or "-g3" stores the same patches without ghost layers (ng = 0: faces applied
    by index maps or read from same-shaped siblings) or with three per side."""
    if name.endswith(("-g0", "-g3")):
        ng = int(name[-1])
        ps, U, desc, kw = make_workload_ng(name[:-3], ng)
    else:
        ps, U, desc, kw = make_workload_ng(name, DEFAULT_NG.get(name))
    return ps, U, desc, kw


def make_workload_ng(name, ng):
    from paper_0910_5547_amd import workloads as W
    kw = {}
    g = {} if ng is None else {"ng": ng}
    if ng is not None and not (name in DEFAULT_NG or name.startswith("box")):
        raise SystemExit(f"workload {name} takes no ghost-layer count")
    if name == "box256":
        ps, U = W.periodic_turbulent_box(N=256, seed=20, **g)
        desc = ("periodic box 256^3, gamma=5/3, rho=1+0.1 GRF(k^-2, 1<=|k|<=16, seed 20), Mach 0.5 GRF velocities, "
                f"p=1, one patch, ng={ps.ng[0]}")
    elif name == "patches4000":
        ps, U = W.uneven_patches(npatch=4000, seed=30, **g)
        desc = (f"4000 patches, n_d in {{8,16,24,32}} (seed 30), ng={ps.ng[0]} stored ghost layers, outflow, "
                "smooth states + 20% planar shocks")
    elif name == "sedov":
        ps, U, _, _ = W.sedov_hierarchy()
        kw = dict(W.SEDOV_FLOORS)
        desc = ("octant Sedov blast (E=1 in the octant, rho=1, p=1e-5, gamma=5/3, t=0.05): 64^3 root + 6 levels "
                "of factor-2 refinement on the analytic profile, density-gradient flags (eps 0.3), "
                f"{ps.npatch} patches of 8..32 cells per dimension, subcycled with refluxing, "
                f"floors rho {kw['rho_floor']:g} e {kw['e_floor']:g}")
    elif name == "mhd192":
        ps, U = W.mhd_vortex_box(N=192, patch=32, seed=50, **g)
        kw = dict(periodic=7, domain=(192, 192, 192))
        desc = (f"ideal MHD (8 variables), 192^3 periodic as 216 patches of 32^3 (EXTERNAL faces, ng={ps.ng[0]}), "
                "gamma=5/3, rho=25/(36 pi), p=5/(12 pi), v=(-sin 2 pi y, sin 2 pi x, 0), B=curl A with "
                "A=GRF(k^-2, 1<=|k|<=4, seeds 50-52), beta=1.7")
    elif name == "glm192":
        ps8, U8 = W.mhd_vortex_box(N=192, patch=32, seed=50, **g)
        ps = W.make_patchset(3, ps8.n, ps8.ng, ps8.bc, lo=ps8.lo, gamma=ps8.gamma, dx0=ps8.dx0, nvar=W.NVAR_GLM)
        U = W.new_arena(ps)
        for p in range(ps.npatch):
            ps.active(U, p)[:8] = ps8.active(U8, p)
            ps.active(U, p)[8] = 0.0
        del U8
        kw = dict(periodic=7, domain=(192, 192, 192), ch=3.0)
        desc = ("GLM-MHD (9 variables, cleaning speed c_h = 3), the mhd192 vortex box with psi = 0: 192^3 "
                f"periodic as 216 patches of 32^3 (EXTERNAL faces, ng={ps.ng[0]})")
    elif name.startswith("sedov") or name.startswith("mhdsedov"):
        # sedovN / mhdsedovN: the centred blast on a uniform N^3 grid (one patch), from the
        # self-similar profile at t = 0.01; the MHD form carries the uniform field (0.01, 0, 0)
        mhd = name.startswith("mhd")
        N = int(name[8:] if mhd else name[5:])
        ps, U, _ = W.sedov_uniform(N, t0=0.01, nvar=W.NVAR_MHD if mhd else W.NVAR, B0=0.01 if mhd else 0.0)
        desc = (f"{'ideal-MHD ' if mhd else ''}blast on a uniform {N}^3 grid of [-1/2,1/2]^3, outflow faces, "
                f"E=1, rho=1, p=1e-5, gamma=5/3, self-similar profile at t=0.01"
                + (", B=(0.01,0,0)" if mhd else ""))
    elif name.startswith("box") and "p" in name[3:]:
        # boxNpP: the N^3 periodic box as (N/P)^3 patches of P^3 with EXTERNAL faces
        N, P = (int(x) for x in name[3:].split("p"))
        ps, U = W.periodic_turbulent_box(N=N, seed=20, kmax=min(16.0, N / 4), patch=P, ng=g.get("ng", 3))
        kw = dict(periodic=7, domain=(N, N, N))
        desc = f"periodic box {N}^3 as {(N // P) ** 3} patches of {P}^3 (EXTERNAL faces, ng=3)"
    elif name.startswith("box"):
        N = int(name[3:])
        ps, U = W.periodic_turbulent_box(N=N, seed=20, kmax=min(16.0, N / 4), **g)
        desc = f"periodic box {N}^3"
    else:
        raise SystemExit(f"unknown workload {name}")
    return ps, U, desc, kw


def time_hierarchy(A, torch, ps, U, precision, exec_form, steps, warmup, kw, shape=None, zslab=0):
    """Root steps of a subcycled hierarchy: CFL reduction (all levels) + amr_hydro_advance.
    The stage split is not measured here (a root step launches every level's stages);
    stage_ms halves the whole step."""
    T = A.Table(ps, precision=precision, exec_form=exec_form, **kw)
    if shape is not None:
        A.amr_table_set_tiling(T.h, shape, zslab)
    Ud = T.upload(U)
    for _ in range(warmup):
        A.amr_cfl_dt(T.h, Ud, 0.8, -1, T.dt)
        A.amr_hydro_advance(T.h, Ud, T.dt)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        A.amr_cfl_dt(T.h, Ud, 0.8, -1, T.dt)
        A.amr_hydro_advance(T.h, Ud, T.dt)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    status = T.status()
    tiling = A.amr_table_get_tiling(T.h)
    tile = "%dx%d" % A.amr_table_tiling_shape(T.h, tiling[0])
    T.close()
    if status != A.AMR_OK:
        raise SystemExit(f"unphysical state during the benchmark: {A.amr_status_string(status)}")
    ms = 1e3 * wall / steps
    return {"ms_per_step": ms, "event_ms_per_step": e0.elapsed_time(e1) / steps, "stage_ms": [ms / 2, ms / 2],
            "tiling": list(tiling), "tile": tile}


def time_form(A, torch, ps, U, precision, exec_form, steps, warmup, kw, tune=True, shape=None, zslab=0):
    if int(ps.level.max()) > 0:
        return time_hierarchy(A, torch, ps, U, precision, exec_form, steps, warmup, kw, shape, zslab)
    T = A.Table(ps, precision=precision, exec_form=exec_form, **kw)
    if shape is not None:
        A.amr_table_set_tiling(T.h, shape, zslab)
    Ud = T.upload(U)
    T.cfl_dt(Ud, 0.8)
    if tune and shape is None and exec_form == A.AMR_EXEC_BATCHED:
        ms = A.amr_autotune(T.h, Ud, T.dt, -1, 3)
        log(f"  autotune: best {A.amr_table_get_tiling(T.h)} at {ms:.3f} ms/step")
    fuse = A.AMR_STEP_FUSE_DT
    for _ in range(warmup):
        A.amr_cfl_dt(T.h, Ud, 0.8, -1, T.dt)
        A.amr_hydro_rk2_step(T.h, Ud, T.dt, -1, fuse)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        A.amr_cfl_dt(T.h, Ud, 0.8, -1, T.dt)
        A.amr_hydro_rk2_step(T.h, Ud, T.dt, -1, fuse)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    # kernel durations: the same launches, eagerly enqueued with HIP events around each stage
    st = [0.0, 0.0]
    for _ in range(steps):
        A.amr_cfl_dt(T.h, Ud, 0.8, -1, T.dt)
        A.amr_hydro_rk2_step(T.h, Ud, T.dt, -1, fuse | A.AMR_STEP_TIMED)
        a, b = A.amr_table_last_stage_ms(T.h)
        st[0] += a
        st[1] += b
    status = T.status()
    tiling = A.amr_table_get_tiling(T.h)
    tile = "%dx%d" % A.amr_table_tiling_shape(T.h, tiling[0])
    T.close()
    if status != A.AMR_OK:
        raise SystemExit(f"unphysical state during the benchmark: {A.amr_status_string(status)}")
    return {"ms_per_step": 1e3 * wall / steps, "event_ms_per_step": ev_ms / steps,
            "stage_ms": [st[0] / steps, st[1] / steps], "tiling": list(tiling), "tile": tile}



# ------------------------------------------------------------------ accuracy against the oracle
def _rel_stats(g, r):
    """Relative L1 per variable, the max per-cell error relative to each variable's largest
    magnitude, and the largest difference of totals relative to the variable's L1 norm."""
    import numpy as np
    l1 = [float(np.sum(np.abs(g[k] - r[k])) / max(np.sum(np.abs(r[k])), 1e-300)) for k in range(len(r))]
    mx = [float(np.max(np.abs(g[k] - r[k])) / max(np.max(np.abs(r[k])), 1e-300)) for k in range(len(r))]
    tot = [abs(math.fsum(g[k]) - math.fsum(r[k])) / max(math.fsum(np.abs(r[k])), 1e-300) for k in range(len(r))]
    return {"l1_rho_vs_oracle": l1[0], "l1_vs_oracle": l1, "max_rel_err_vs_oracle": max(mx),
            "totals_rel_diff_vs_oracle": max(tot)}


def _gpu_steps(A, torch, ps, U, precision, exec_form, kw, steps):
    """`steps` RK2 steps of the whole workload from U with the table's own CFL dt (read back
    each step); returns the final arena and the dt sequence."""
    T = A.Table(ps, precision=precision, exec_form=exec_form, **kw)
    Ud = T.upload(U)
    dts = []
    for _ in range(steps):
        dts.append(T.cfl_dt(Ud, 0.8))
        T.step(Ud)
    torch.cuda.synchronize()
    st = T.status()
    Ug = Ud.cpu().numpy()
    T.close()
    if st != A.AMR_OK:
        raise SystemExit(f"unphysical state in the accuracy run: {A.amr_status_string(st)}")
    return Ug, dts


def _oracle_kw(kw):
    return {k: v for k, v in kw.items() if k in ("rho_floor", "e_floor", "ch")}


def check_patches(A, torch, O, ps, U, precision, exec_form, kw, steps=10, nsample=40):
    """Independent patches: the oracle advances an evenly spread sample of them with the
    GPU run's time steps (the global dt couples the patches only through its value)."""
    import numpy as np
    from paper_0910_5547_amd import workloads as W
    Ug, dts = _gpu_steps(A, torch, ps, U, precision, exec_form, kw, steps)
    sel = sorted(set(np.linspace(0, ps.npatch - 1, min(nsample, ps.npatch)).astype(int).tolist()))
    # (the oracle stores its ghost layers: at least two)
    sub = W.make_patchset(ps.ndim, ps.n[sel], np.maximum(ps.ng[sel], 2), ps.bc[sel], gamma=ps.gamma,
                          theta=ps.theta, dx0=ps.dx0, nvar=ps.nvar)
    Us = W.new_arena(sub)
    for i, p in enumerate(sel):
        sub.active(Us, i)[...] = ps.active(U, p)
    o = O.Oracle(sub, parallel=True, **_oracle_kw(kw))
    for dt in dts:
        if o.rk2_step(Us, dt):
            raise SystemExit("the oracle met an unphysical state in the accuracy run")
    g = np.concatenate([ps.active(Ug, p).reshape(ps.nvar, -1) for p in sel], axis=1)
    r = np.concatenate([sub.active(Us, i).reshape(ps.nvar, -1) for i in range(len(sel))], axis=1)
    out = _rel_stats(g, r)
    out.update({"steps": steps, "sample": f"{len(sel)} of {ps.npatch} patches ({r.shape[1]} cells)"})
    return out


def _global_field(ps, U):
    """(nvar, Nz, Ny, Nx) active field of a single-level periodic box (one patch or many)."""
    import numpy as np
    hi = (ps.lo + ps.n).max(axis=0)
    G = np.empty((ps.nvar, int(hi[2]), int(hi[1]), int(hi[0])))
    for p in range(ps.npatch):
        lo, n = ps.lo[p], ps.n[p]
        G[:, lo[2]:lo[2] + n[2], lo[1]:lo[1] + n[1], lo[0]:lo[0] + n[0]] = ps.active(U, p)
    return G


def check_box(A, torch, O, ps, U, precision, exec_form, kw, steps=2, B=32):
    """Periodic box: four B^3 blocks (two across the periodic seam) recomputed by the oracle
    on the block plus a halo of 4 cells per step (one RK2 step reads 4 cells each way), fed
    the GPU's time steps; the conservation drift of the whole box is the GPU's own."""
    import numpy as np
    from paper_0910_5547_amd import workloads as W
    Ug, dts = _gpu_steps(A, torch, ps, U, precision, exec_form, kw, steps)
    G0, G1 = _global_field(ps, U), _global_field(ps, Ug)
    N = G0.shape[1:]
    h = 4 * steps
    origins = [(0, 0, 0), (N[0] // 3, N[1] // 2, N[2] // 5), (N[0] - B // 2, N[1] - B // 2, N[2] - B // 2),
               (N[0] // 2, 7, N[2] - 9)]
    gs, rs = [], []
    for oz, oy, ox in origins:
        idx = [(o - h + np.arange(B + 2 * h)) % N[a] for a, o in enumerate((oz, oy, ox))]
        blk = G0[:, idx[0]][:, :, idx[1]][:, :, :, idx[2]]
        sub = W.make_patchset(3, [[B + 2 * h] * 3], 2, [W.BC_OUTFLOW] * 6, gamma=ps.gamma, theta=ps.theta,
                              dx0=ps.dx0, nvar=ps.nvar)
        Us = W.new_arena(sub)
        sub.active(Us, 0)[...] = blk
        o = O.Oracle(sub, **_oracle_kw(kw))
        for dt in dts:
            if o.rk2_step(Us, dt):
                raise SystemExit("the oracle met an unphysical state in the accuracy run")
        rs.append(sub.active(Us, 0)[:, h:h + B, h:h + B, h:h + B].reshape(ps.nvar, -1))
        inner = [(o + np.arange(B)) % N[a] for a, o in enumerate((oz, oy, ox))]
        gs.append(G1[:, inner[0]][:, :, inner[1]][:, :, :, inner[2]].reshape(ps.nvar, -1))
    out = _rel_stats(np.concatenate(gs, axis=1), np.concatenate(rs, axis=1))
    # (a variable that starts at zero everywhere, v_z of the MHD vortex, takes its developed field's scale)
    drift = [abs(math.fsum(G1[k].ravel()) - math.fsum(G0[k].ravel()))
             / max(math.fsum(np.abs(G0[k]).ravel()), math.fsum(np.abs(G1[k]).ravel()), 1e-300) for k in range(ps.nvar)]
    out.update({"steps": steps, "totals_drift": max(drift),
                "sample": f"4 blocks of {B}^3 (oracle on {B + 2 * h}^3 with their domain of dependence)"})
    return out


def check_form(A, torch, ps, U, precision, exec_form, kw, plain_many):
    """Accuracy of one form against the oracle, or None where no cheap sample exists
    (hierarchies, whose subcycled step the test suite checks; single large patches)."""
    from oracle import oracle as O
    if int(ps.level.max()) > 0:
        return None
    periodic_box = kw.get("periodic", 0) == (1 << ps.ndim) - 1 or (ps.npatch == 1 and (ps.bc == 1).all())
    if periodic_box and ps.ndim == 3:
        return check_box(A, torch, O, ps, U, precision, exec_form, kw, steps=1 if plain_many else 2)
    if (ps.bc == 3).any() or ps.npatch < 8:
        return None
    return check_patches(A, torch, O, ps, U, precision, exec_form, kw, steps=3 if plain_many else 10)


# ------------------------------------------------------------------ streaming ceiling
def stream_ceiling(A, torch, n=1 << 28, reps=5):
    """GB/s of amr_stream_ceiling over 3 arrays of n doubles (2 GiB each, far beyond the
    256 MB Infinity Cache), the best of a few launch shapes, timed with events on the
    launch stream."""
    a = torch.full((n,), 1.0, dtype=torch.float64, device="cuda")
    b = torch.full((n,), 3.0, dtype=torch.float64, device="cuda")
    c = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    best = None
    for wpc in (0, 4, 8, 16):
        A.amr_stream_ceiling(a, b, c, n, wpc)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            A.amr_stream_ceiling(a, b, c, n, wpc)
        e1.record(stream)
        torch.cuda.synchronize()
        gbps = 24.0 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
        if best is None or gbps > best[0]:
            best = (gbps, wpc)
    ok = bool(torch.all(c == 2.0).item())
    del a, b, c
    torch.cuda.empty_cache()
    if not ok:
        raise SystemExit("amr_stream_ceiling produced a wrong result")
    return {"value": best[0], "unit": "GB/s", "frac_of_peak": best[0] / HBM_PEAK_GBPS,
            "kernel": f"amr_stream_ceiling: out=(a+b)/2, 3 x {n * 8 >> 30} GiB, 24 B per element, "
                      f"{'one pass' if best[1] == 0 else f'{best[1]} workgroups per CU'}"}


# ------------------------------------------------------------------ CPU baseline
def host_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def _oracle_rate(O, ps, U, kw, parallel, budget_s):
    o = O.Oracle(ps, parallel=parallel, **kw)
    V = U.copy()
    cells = ps.active_cells()
    steps, t = 0, 0.0
    while t < budget_s and steps < 1000:
        t0 = time.perf_counter()
        dt = o.cfl_dt(V, 0.8)
        o.rk2_step(V, dt)
        t += time.perf_counter() - t0
        steps += 1
    return cells * steps / t, steps, t


def cpu_baseline(ps_full, U_full, kw, budget_s=8.0):
    """The FP64 oracle on a bounded sample of the same workload: the serial build pinned to
    one core, and its OpenMP build (same results) on every core this process may use."""
    import numpy as np

    from oracle import oracle as O
    from paper_0910_5547_amd import workloads as W
    nv = ps_full.nvar
    kw = _oracle_kw(kw)
    if ps_full.npatch == 1:
        B = min(64, int(ps_full.n[0].min()))
        a = ps_full.active(U_full, 0)[:, :B, :B, :B]
        ps = W.make_patchset(3, [[B, B, B]], 2, ps_full.bc[0], gamma=ps_full.gamma, dx0=ps_full.dx0, nvar=nv)
        U = W.new_arena(ps)
        ps.active(U, 0)[...] = a
        what = f"{B}^3 corner sub-box of the workload's field (its boundary conditions)"
    else:
        k = 64 if nv == W.NVAR else 8
        sel = list(range(k))
        ps = W.make_patchset(3, ps_full.n[sel], np.maximum(ps_full.ng[sel], 2), [W.BC_OUTFLOW] * 6,
                             gamma=ps_full.gamma, dx0=ps_full.dx0, nvar=nv)
        U = W.new_arena(ps)
        for i, p in enumerate(sel):
            ps.active(U, i)[...] = ps_full.active(U_full, p)
        what = f"first {k} of the workload's patches (outflow faces)"
    info = host_info()
    try:
        cpus = sorted(os.sched_getaffinity(0))
        os.sched_setaffinity(0, {cpus[0]})
    except (AttributeError, OSError):
        cpus = None
    try:
        v1, s1, t1 = _oracle_rate(O, ps, U, kw, False, budget_s)
    finally:
        if cpus:
            os.sched_setaffinity(0, set(cpus))
    threads = int(O.lib(True).or_threads())
    vn, sn, tn = _oracle_rate(O, ps, U, kw, True, budget_s)
    return {"value": v1, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{what}: {ps.active_cells()} cells x {s1} RK2 steps (+ CFL) in {t1:.1f} s, serial FP64 "
                      f"pinned to one core",
            "all_cores": {"value": vn, "cores": threads, "build": "the same source with -fopenmp (patch loops)",
                          "sample": f"{sn} RK2 steps (+ CFL) in {tn:.1f} s"},
            "host": info}


# ------------------------------------------------------------------ one workload
FORMS = ("plain_fp64", "batched_fp64", "batched_mixed")


def run_workload(A, torch, name, forms, args):
    t0 = time.time()
    ps, U, desc, kw = make_workload(name)
    hierarchy = int(ps.level.max()) > 0
    bpc = bytes_per_cell(ps.nvar)
    # cell-updates per step: sum over levels of 2^l N_l (level l takes 2^l steps per root step)
    cells = int(sum((1 << int(ps.level[p])) * int(ps.n[p].prod()) for p in range(ps.npatch)))
    log(f"workload {name}: {cells} cells, {ps.npatch} patches, arena {ps.arena * 8 / 1e9:.2f} GB "
        f"(built in {time.time() - t0:.1f} s)")
    kinds = {"plain_fp64": (A.AMR_PREC_FP64, A.AMR_EXEC_PLAIN), "batched_fp64": (A.AMR_PREC_FP64, A.AMR_EXEC_BATCHED),
             "batched_mixed": (A.AMR_PREC_MIXED, A.AMR_EXEC_BATCHED)}
    res = {}
    for form in forms:
        prec, exe = kinds[form]
        steps, warmup = args.steps, args.warmup
        plain_many = exe == A.AMR_EXEC_PLAIN and ps.npatch > 64
        if hierarchy and exe == A.AMR_EXEC_PLAIN:
            # one launch per patch, stage, level substep: ~10^5 launches per root step
            steps, warmup = min(steps, 2), min(warmup, 1)
        elif plain_many:
            # one launch per patch and stage: thousands of launches per step
            steps, warmup = min(steps, 5), min(warmup, 2)
        log(f"form {form} ({steps} steps)")
        r = time_form(A, torch, ps, U, prec, exe, steps, warmup, kw, tune=args.tune, shape=args.shape,
                      zslab=args.zslab)
        r["steps"] = steps
        r["value"] = cells / (r["ms_per_step"] * 1e-3)
        r["hbm_frac_step"] = bpc * cells / (r["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBPS
        kern_ms = sum(r["stage_ms"])
        r["stage_kernel_GBps"] = bpc * cells / (kern_ms * 1e-3) / 1e9
        log(f"  {form}: {r['ms_per_step']:.3f} ms/step, {r['value'] / 1e9:.2f} G cell-updates/s, "
            f"stages {r['stage_ms'][0]:.3f}+{r['stage_ms'][1]:.3f} ms, {r['stage_kernel_GBps']:.0f} GB/s")
        if args.check:
            c = check_form(A, torch, ps, U, prec, exe, kw, plain_many)
            if c is not None:
                log(f"  {form} vs oracle: L1(rho) {c['l1_rho_vs_oracle']:.2e}, max rel {c['max_rel_err_vs_oracle']:.2e}, "
                    f"totals {c['totals_rel_diff_vs_oracle']:.2e} ({c['sample']}, {c['steps']} steps)")
            r["accuracy"] = c
        res[form] = r
    main_form = "batched_mixed" if "batched_mixed" in res else list(res)[-1]
    m = res[main_form]
    achieved = bpc * cells / (sum(m["stage_ms"]) * 1e-3) / 1e9
    block = {
        "workload": desc, "nvar": ps.nvar, "cells": cells, "patches": ps.npatch, "form": main_form,
        "value": m["value"], "ms_per_step": m["ms_per_step"], "hbm_frac": m["hbm_frac_step"],
        "forms": {k: {"value": v["value"], "ms_per_step": v["ms_per_step"], "hbm_frac": v["hbm_frac_step"],
                      "steps": v["steps"], "stage_ms": v["stage_ms"], "tiling": v["tiling"],
                      **({"l1_rho_vs_oracle": v["accuracy"]["l1_rho_vs_oracle"],
                          "accuracy": v["accuracy"]} if v.get("accuracy") else {})}
                  for k, v in res.items()},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic_for(name, main_form, cells, m["tile"]),
                     "kernel": (f"whole root step of all levels ({main_form}): stage, ghost, register, refluxing "
                                f"and restriction kernels, {bpc} B per cell-update" if hierarchy else
                                f"stage_kernel ({main_form}, {m['tile']} tiles), 2 launches/step, "
                                f"{bytes_stage(ps.nvar)[0]}+{bytes_stage(ps.nvar)[1]} "
                                f"B/cell, avg {sum(m['stage_ms']) / 2:.4f} ms/launch")},
        "config": {"cfl": 0.8, "theta": ps.theta, "flux": "paper (Sec. 4)", "tiling": m["tiling"]},
    }
    return block, ps, U, kw


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="patches4000")
    ap.add_argument("--extra", default="box256,patches4000-g0",
                    help="comma-separated workloads timed as extra keys of the same line ('' = none)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-check", dest="check", action="store_false",
                    help="skip the accuracy runs against the oracle")
    ap.add_argument("--no-ceiling", dest="ceiling", action="store_false",
                    help="skip the streaming-ceiling measurement")
    ap.add_argument("--no-tune", dest="tune", action="store_false",
                    help="skip the library's autotuner (tile shape and z-slab) and keep its default tiling")
    ap.add_argument("--forms", default=",".join(FORMS))
    ap.add_argument("--shape", type=int, default=None,
                    help="tile shape id (default: the library's choice for the workload; --tune overrides)")
    ap.add_argument("--zslab", type=int, default=0, help="z-slab length with --shape (0 = automatic)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 1 GiB device copy (counter calibration for --summarize-pmc)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the traffic summary from two rocprofv3 --pmc counter_collection CSVs and exit")
    args = ap.parse_args()
    if args.summarize_pmc:
        cells, nvar = {"box256": (256 ** 3, 5), "mhd192": (192 ** 3, 8), "glm192": (192 ** 3, 9)}.get(args.workload, (None, 5))
        if cells is None:
            cells = make_workload(args.workload)[0].active_cells()
        form = args.forms.split(",")[-1]
        e = summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.workload, form, cells, nvar)
        print(json.dumps(e, indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py: the update runs on one GPU; --gpus {args.gpus} is not supported "
              "(sharding the patch table over several GPUs is designed, not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_0910_5547_amd import amr as A
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    A.lib()

    if args.calibrate_copy:
        a = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    forms = args.forms.split(",")
    head, ps, U, kw = run_workload(A, torch, args.workload, forms, args)
    extras = {}
    for name in [x for x in args.extra.split(",") if x and x != args.workload]:
        extras[name], _, _, _ = run_workload(A, torch, name, forms, args)
    ceiling = stream_ceiling(A, torch) if args.ceiling else None
    if ceiling:
        log(f"streaming ceiling: {ceiling['value']:.0f} GB/s ({ceiling['kernel']})")
        for blk in [head, *extras.values()]:
            blk["roofline"]["ceiling"] = ceiling["value"]
            blk["roofline"]["frac_of_ceiling"] = blk["roofline"]["achieved"] / ceiling["value"]
    main_form = head["form"]
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if main_form == "batched_mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": head["workload"], "nvar": head["nvar"], "cells": head["cells"],
                   "patches": head["patches"], "form": main_form, **head["config"]},
        "hbm_frac": head["hbm_frac"],
        "forms": head["forms"],
        "roofline": head["roofline"],
    }
    if ceiling:
        out["ceiling"] = ceiling
    for name, blk in extras.items():
        out[name] = blk
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(ps, U, kw)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
