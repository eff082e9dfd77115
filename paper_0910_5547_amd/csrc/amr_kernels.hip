// amr_kernels.hip - gfx950 kernels around the stage kernel of the per-patch MOL
// update (Wang, Abel & Kaehler, Secs. 4-5): the CFL reduction, same-level ghost
// copies, the per-level dt and graph-safe clears, and the launch dispatch to the
// stage kernel's instantiations (amr_stage.h).
#include "amr_device.h"
#include "amr_internal.h"

namespace amr {
// ------------------------------------------------------------------ CFL
// Max signal speed over the active cells of the tile list (one plane of a tile
// per workgroup iteration); the block max is merged into smax[level] with a
// 64-bit atomicMax on the bit pattern (non-negative doubles order as integers).
template <bool FAST, int NV>
__global__ __launch_bounds__(NT) void cfl_kernel(CflArgs a) {
  const Consts C = a.c;
  int bad = 0;
  for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
    const Tile T = a.tiles[t];
    const PatchDev P = a.patches[T.patch];
    const int tx = a.tx > 0 ? a.tx : T.tx, ty = a.tx > 0 ? a.ty : NT / tx;  // tx 0: the tile's own width
    const int nxT = min(tx, P.n[0] - T.x0), nyT = min(ty, P.n[1] - T.y0);
    const int per_plane = nxT * nyT;
    const int ncell = per_plane * (T.z1 - T.z0);
    double smax = 0.0;
    for (int c = threadIdx.x; c < ncell; c += NT) {
      const int kk = c / per_plane, r = c - kk * per_plane;
      const int jj = r / nxT, ii = r - jj * nxT;
      const int64_t e = cell_elem(P, T.x0 + ii, T.y0 + jj, T.z0 + kk);
      double u[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) u[v] = a.U[e + v * P.S];
      smax = fmax(smax, cell_speed<FAST, NV>(u, C, P, bad));
    }
    block_max_to(a.smax + P.level, smax);
  }
  if (bad) atomicOr(a.flag, 1);
}

// dt from the per-level maxima: one level l -> cfl / smax_l; all levels (root) ->
// the root step of factor-2 subcycling, dt0 = cfl * min_l 2^l / smax_l, computed as
// cfl / max_l (smax_l 2^-l) (the power-of-two scaling is exact).
__global__ void cfl_finalize(const unsigned long long* smax, int lmin, int lmax, int root, double cfl, double* dt) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double S = 0.0;
    for (int l = lmin; l <= lmax; ++l) {
      const double s = __longlong_as_double((long long)smax[l]);
      S = fmax(S, root ? ldexp(s, -l) : s);
    }
    dt[0] = cfl / S;
  }
}

// ------------------------------------------------------------------ ghosts
// Same-level EXTERNAL ghost fill, one ghost cell (all NV variables) per lane; every
// variable is read before the first store (one round trip, not one per variable).
template <int NV>
__global__ __launch_bounds__(NT) void copy_ghosts(const CopyOp* __restrict__ ops, Work w,
                                                  const PatchDev* __restrict__ patches, double* A) {
  int c;
  const int o = work_item(w, c);
  if (o < 0) return;
  const CopyOp op = ops[o];
  const PatchDev& D = patches[op.dst];
  const PatchDev& S = patches[op.src];
  int b[3];
  box_cell(op.sz, c, b);
  const int i = op.lo[0] + b[0], j = op.lo[1] + b[1], k = op.lo[2] + b[2];
  const int64_t ed = cell_elem(D, i, j, k);
  const int64_t es = cell_elem(S, i + op.sh[0], j + op.sh[1], k + op.sh[2]);
  double u[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = A[es + v * S.S];
#pragma unroll
  for (int v = 0; v < NV; ++v) A[ed + v * D.S] = u[v];
}

// dt_l = dt0 / 2^l: factor-2 subcycling of a block-structured hierarchy.
__global__ void scale_dt(const double* dt0, double* dtl, int nlev) {
  const int l = threadIdx.x;
  if (l < nlev) dtl[l] = ldexp(dt0[0], -l);
}

// Graph-safe clears (no memset nodes in captured work).
__global__ void fill_u64(unsigned long long* p, int n, unsigned long long v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void fill_i32(int* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ launchers
// The stage kernel's instantiations live in one translation unit per variable count
// (and, for hydro, per reconstruction precision): amr_stage_*.hip.
hipError_t launch_stage(int nv, int mixed, int shape, int stage, int grid, hipStream_t s, const StageArgs& a) {
  if (nv == NVAR_MHD) return launch_stage_mhd8(mixed, shape, stage, grid, s, a);
  if (nv == NVAR_GLM) return launch_stage_glm9(mixed, shape, stage, grid, s, a);
  return mixed ? launch_stage_hydro_f32(shape, stage, grid, s, a) : launch_stage_hydro_f64(shape, stage, grid, s, a);
}

const void* stage_kernel_ptr(int nv, int mixed, int shape, int stage, bool rec) {
  if (nv == NVAR_MHD) return stage_kernel_ptr_mhd8(mixed, shape, stage, rec);
  if (nv == NVAR_GLM) return stage_kernel_ptr_glm9(mixed, shape, stage, rec);
  return mixed ? stage_kernel_ptr_hydro_f32(shape, stage, rec) : stage_kernel_ptr_hydro_f64(shape, stage, rec);
}

hipError_t launch_cfl(int grid, hipStream_t s, const CflArgs& a) {
  if (a.nv == NVAR_MHD) {
    if (a.fast) hipLaunchKernelGGL((cfl_kernel<true, NVAR_MHD>), dim3(grid), dim3(NT), 0, s, a);
    else hipLaunchKernelGGL((cfl_kernel<false, NVAR_MHD>), dim3(grid), dim3(NT), 0, s, a);
  } else if (a.nv == NVAR_GLM) {
    if (a.fast) hipLaunchKernelGGL((cfl_kernel<true, NVAR_GLM>), dim3(grid), dim3(NT), 0, s, a);
    else hipLaunchKernelGGL((cfl_kernel<false, NVAR_GLM>), dim3(grid), dim3(NT), 0, s, a);
  } else {
    if (a.fast) hipLaunchKernelGGL((cfl_kernel<true, NVAR>), dim3(grid), dim3(NT), 0, s, a);
    else hipLaunchKernelGGL((cfl_kernel<false, NVAR>), dim3(grid), dim3(NT), 0, s, a);
  }
  return hipGetLastError();
}
hipError_t launch_cfl_finalize(hipStream_t s, const unsigned long long* smax, int lmin, int lmax, int root,
                               double cfl, double* dt) {
  hipLaunchKernelGGL(cfl_finalize, dim3(1), dim3(64), 0, s, smax, lmin, lmax, root, cfl, dt);
  return hipGetLastError();
}
hipError_t launch_copy_ghosts(hipStream_t s, const CopyOp* ops, const Work& w, const PatchDev* p, double* A, int nv) {
  if (nv == NVAR_MHD) hipLaunchKernelGGL(copy_ghosts<NVAR_MHD>, dim3(w.nblk), dim3(NT), 0, s, ops, w, p, A);
  else if (nv == NVAR_GLM) hipLaunchKernelGGL(copy_ghosts<NVAR_GLM>, dim3(w.nblk), dim3(NT), 0, s, ops, w, p, A);
  else hipLaunchKernelGGL(copy_ghosts<NVAR>, dim3(w.nblk), dim3(NT), 0, s, ops, w, p, A);
  return hipGetLastError();
}
hipError_t launch_fill_u64(hipStream_t s, unsigned long long* p, int n, unsigned long long v) {
  hipLaunchKernelGGL(fill_u64, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_scale_dt(hipStream_t s, const double* dt0, double* dtl, int nlev) {
  hipLaunchKernelGGL(scale_dt, dim3(1), dim3(64), 0, s, dt0, dtl, nlev);
  return hipGetLastError();
}
hipError_t launch_fill_i32(hipStream_t s, int* p, int n, int v) {
  hipLaunchKernelGGL(fill_i32, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace amr
