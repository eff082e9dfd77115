// amr_internal.h - kernel argument blocks and launcher declarations shared by
// the kernels (amr_kernels.hip, amr_stage*.hip, amr_refine.hip, amr_regrid.hip) and the
// host library (amr_api.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/amr_hydro.h"
#include "amr_device.h"

namespace amr {

struct StageArgs {
  const double* V;               // stage input arena (EXTERNAL ghosts filled)
  const double* U0;              // U^n (stage 2 only)
  double* out;                   // stage output arena (U^(1), or U^{n+1} in place over U^n)
  const double* dt;              // device scalar, read when the stage runs
  const PatchDev* patches;
  const Tile* tiles;
  int ntiles;
  int pad;
  int* flag;                     // unphysical-state latch
  unsigned long long* smax;      // stage 2: per-level max signal speed of U^{n+1}, or nullptr
  double* reg;                   // fine-face flux registers (+= dt/2 F on recorded faces), or nullptr
  Consts c;
};

struct CflArgs {
  const double* U;
  const PatchDev* patches;
  const Tile* tiles;
  int ntiles, tx, ty, fast;         // tx 0: each tile carries its width (Tile::tx); fast: the mixed CFL rule
  int nv;                           // conserved variables (5 hydro, 8 MHD)
  int* flag;
  unsigned long long* smax;      // per-level maxima
  Consts c;
};

// Block-wide max of a non-negative double merged into *dst with a 64-bit
// atomicMax on its bit pattern.  Must be called by every lane of the block.
__device__ __forceinline__ void block_max_to(unsigned long long* dst, double v) {
  __shared__ double red[16];  // one per wavefront, up to 1024 threads
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();  // red[] may still be read by a previous call
  if (lane == 0) red[wv] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, red[w]);
    if (m > 0) atomicMax(dst, (unsigned long long)__double_as_longlong(m));
  }
}

// Wavefront max of a non-negative double merged into *dst (no workgroup barrier).
__device__ __forceinline__ void wave_max_to(unsigned long long* dst, double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  if ((threadIdx.x & 63) == 0 && v > 0) atomicMax(dst, (unsigned long long)__double_as_longlong(v));
}

hipError_t launch_stage(int nv, int mixed, int shape, int stage, int grid, hipStream_t s, const StageArgs& a);
const void* stage_kernel_ptr(int nv, int mixed, int shape, int stage, bool rec);
// per translation unit of the stage kernel (amr_stage_*.hip)
hipError_t launch_stage_hydro_f32(int shape, int stage, int grid, hipStream_t s, const StageArgs& a);
hipError_t launch_stage_hydro_f64(int shape, int stage, int grid, hipStream_t s, const StageArgs& a);
hipError_t launch_stage_mhd8(int mixed, int shape, int stage, int grid, hipStream_t s, const StageArgs& a);
hipError_t launch_stage_glm9(int mixed, int shape, int stage, int grid, hipStream_t s, const StageArgs& a);
const void* stage_kernel_ptr_hydro_f32(int shape, int stage, bool rec);
const void* stage_kernel_ptr_hydro_f64(int shape, int stage, bool rec);
const void* stage_kernel_ptr_mhd8(int mixed, int shape, int stage, bool rec);
const void* stage_kernel_ptr_glm9(int mixed, int shape, int stage, bool rec);
hipError_t launch_cfl(int grid, hipStream_t s, const CflArgs& a);
hipError_t launch_cfl_finalize(hipStream_t s, const unsigned long long* smax, int lmin, int lmax, int root,
                               double cfl, double* dt);
hipError_t launch_copy_ghosts(hipStream_t s, const CopyOp* ops, const Work& w, const PatchDev* p, double* A, int nv);
hipError_t launch_fill_u64(hipStream_t s, unsigned long long* p, int n, unsigned long long v);
hipError_t launch_fill_i32(hipStream_t s, int* p, int n, int v);

hipError_t launch_prolong(hipStream_t s, const ProlongOp* ops, const Work& w, const PatchDev* p, double* A,
                          const double* Cold, const double* Cnew, double alpha, int ndim, int nv);
hipError_t launch_phys(hipStream_t s, const PhysOp* ops, const Work& w, const PatchDev* p, double* A, int nv);
hipError_t launch_flux_fix(int mixed, int nv, hipStream_t s, const FixOp* ops, const Work& w, const PatchDev* p,
                           double* U, const double* S1, const double* S2, const double* reg, const double* dtc,
                           const Consts& C, int* flag);
hipError_t launch_restrict(hipStream_t s, const RestrictOp* ops, const Work& w, const PatchDev* p, double* U,
                           int ndim, int nv);
hipError_t launch_scale_dt(hipStream_t s, const double* dt0, double* dtl, int nlev);
hipError_t launch_copy_cells_x(hipStream_t s, const CopyOp* ops, const Work& w, const PatchDev* pdst,
                               const PatchDev* psrc, double* Adst, const double* Asrc, int nv);
hipError_t launch_flag_cells(hipStream_t s, const int* plist, const int64_t* cofs, int npl, int64_t ncells,
                             const PatchDev* patches, const double* U, double eps, uint8_t* flags, int ndim);

// Compiled tile shapes; shape 0 is the 1D shape.  TX x TY = workgroup size: one
// tile per workgroup (256 threads; 512 for 32 x 16, shape 5, and 384 for 32 x 12,
// shape 6, which cut the y-halo share of a tile); 8 x 8 (shape 4, small patches):
// one tile per wavefront, four per workgroup.  Every shape has at most one halo
// cell and one edge face per lane.
// Shape 7 (patch-fit, SHAPE_TX = SHAPE_TY = 0): 256-lane tiles whose width follows the
// patch, tx = 8, 16 or 32 for n_x up to 8, 16 or more, height 256 / tx, so that patches
// 8 or 16 cells wide fill the lanes that 32-wide tiles leave idle.
constexpr int NSHAPES = 8;
constexpr int SHAPE_TX[NSHAPES] = {256, 32, 64, 16, 8, 32, 32, 0};
constexpr int SHAPE_TY[NSHAPES] = {1, 8, 4, 16, 8, 16, 12, 0};
constexpr int SHAPE_NT[NSHAPES] = {256, 256, 256, 256, 256, 512, 384, 256};
constexpr int SHAPE_SMALL = 4;
constexpr int SHAPE_FIT = 7;
constexpr int shape_tiles_per_wg(int shape) {
  return shape == SHAPE_FIT ? 1 : SHAPE_NT[shape] / (SHAPE_TX[shape] * SHAPE_TY[shape]);
}
// Tile width and height of a shape on a patch n_x cells wide.
inline void tile_dims(int shape, int nx, int& tx, int& ty) {
  if (shape == SHAPE_FIT) {
    tx = nx <= 8 ? 8 : nx <= 16 ? 16 : 32;
    ty = NT / tx;
  } else {
    tx = SHAPE_TX[shape];
    ty = SHAPE_TY[shape];
  }
}
// Shapes compiled for MHD (8 variables): 1D, 32 x 8, 8 x 8 and patch-fit in both precisions;
// 32 x 16 and 32 x 12 in FP32 only (in FP64 the primitive plane and face states of
// eight variables exceed the LDS of a workgroup, or leave one workgroup per CU
// that spills registers).
constexpr bool mhd_shape_ok(int mixed, int shape) {
  return shape == 0 || shape == 1 || shape == 4 || shape == SHAPE_FIT || ((shape == 5 || shape == 6) && mixed);
}

// Host helpers shared by the table (amr_api.hip) and the allocation-free step
// (amr_noalloc.hip).
// Descriptor and physics validation of amr_patch_table_create (AMR_EINVAL rules of
// the public header).
amr_status validate_patches(const amr_patch_desc* P, int32_t np, const amr_physics* ph);
// Kernel constants of a physics block.
Consts consts_of_phys(const amr_physics& ph);
// z-slab length that balances a persistent launch: per-tile time taken as
// proportional to its planes + 4 (the z prologue reads 4 planes); with txy column
// blocks, nz planes and G tiles in flight, the slab count that minimises
// rounds x (slab + 4).  Enough column blocks keep whole patches.
inline int balanced_zslab(int64_t txy, int nz, int64_t G) {
  if (txy >= 4 * G) return nz;
  int64_t best = -1;
  int bz = nz;
  for (int ns = 1; ns <= (nz / 8 > 1 ? nz / 8 : 1); ++ns) {
    const int zs = (nz + ns - 1) / ns;
    const int64_t rounds = (txy * ((nz + zs - 1) / zs) + G - 1) / G;
    const int64_t c = rounds * (zs + 4);
    if (best < 0 || c < best) {
      best = c;
      bz = zs;
    }
  }
  return bz;
}

}  // namespace amr
