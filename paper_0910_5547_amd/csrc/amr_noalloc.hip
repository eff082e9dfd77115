// amr_noalloc.hip - the allocation-free RK2 step of one patch (amr_patch_rk2_step_noalloc
// in include/amr_hydro.h), for callers that cannot allocate device memory.
//
// Its device scratch - the stage output U^(1), the patch's device descriptor and its
// tile list - lives in `scratch`, a file-scope device array that each GPU holds from
// the library's first use on it until the process ends.  The host never passes the
// array's name to a kernel or a copy (in host code it names a host-side stand-in):
// on the first call on a device, with that device current, hipGetSymbolAddress gives
// that device's address of the array, kept per device and used from then on.  The
// tile list and descriptor are written by a small kernel from its arguments, so one
// call enqueues kernels only (no allocation, no host-to-device copy) and can be
// captured into a HIP graph.  Calls that overlap on one GPU share its scratch and race.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <mutex>

#include "../../include/amr_hydro.h"
#include "amr_internal.h"

using namespace amr;

namespace {

constexpr size_t SCRATCH_BYTES = AMR_NOALLOC_SCRATCH_BYTES;
constexpr size_t HDR_BYTES = 512;  // descriptor slot; the tile list follows
static_assert(sizeof(PatchDev) <= HDR_BYTES, "descriptor slot too small");
static_assert(sizeof(Tile) == 32, "tile layout");

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
unsigned char* g_scratch[MAX_DEVICES] = {};  // device address of `scratch`, per device
int g_ncu[MAX_DEVICES] = {};
int g_occ[3][2][NSHAPES][2] = {};            // resident workgroups per CU: [variables][mixed][shape][stage]

// Tile list of one patch in the persistent launch's order: the column blocks (x
// fastest, then y, then z slab) are cut into 8 contiguous chunks of units of W tiles
// (W = tiles per workgroup), the larger chunks last, and dealt unit by unit over the
// chunks, so that workgroup b (run on XCD b mod 8) walks one compact region and the
// unit holding the list's ragged end comes last.
__global__ void noalloc_tiles(PatchDev P, PatchDev* pd, Tile* tiles, int L, int W, int ntx, int nty, int TX,
                              int TY, int zs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *pd = P;
  if (i >= L) return;
  const int NU = (L + W - 1) / W, fl = NU / 8, r = NU % 8;
  const int j = i / W, q = i % W;
  int c, m;
  if (j < 8 * fl) {
    c = j % 8;
    m = j / 8;
  } else {
    c = 8 - r + (j - 8 * fl);
    m = fl;
  }
  const int start = c * fl + max(0, c - (8 - r));
  const int u = (start + m) * W + q;  // index in x, y, z-slab order; < L by construction
  const int xb = u % ntx, yb = (u / ntx) % nty, zb = u / (ntx * nty);
  Tile T{};
  T.patch = 0;
  T.x0 = xb * TX;
  T.y0 = yb * TY;
  T.z0 = zb * zs;
  T.z1 = min(T.z0 + zs, P.n[2]);
  T.tx = TX;
  tiles[i] = T;
}

int occupancy(int nv, int mixed, int shape, int stage) {
  const int vk = nv == NVAR_MHD ? 1 : nv == NVAR_GLM ? 2 : 0;
  int& per_cu = g_occ[vk][mixed][shape][stage - 1];
  if (per_cu <= 0) {
    const void* k = stage_kernel_ptr(nv, mixed, shape, stage, false);
    if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, SHAPE_NT[shape], 0) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
  }
  return per_cu;
}

// The table's default tile shape for a lone patch: 32 x 16 where those tiles are
// nearly full (3D hydro, and MHD in mixed precision), else 8 x 8 wavefront tiles
// when 32 x 8 tiles would leave more than half their lanes idle, else 32 x 8.
int lone_patch_shape(const amr_physics& ph, const int n[3]) {
  if (ph.ndim == 1) return 0;
  auto lane_use = [&](int shape) {
    const double TX = SHAPE_TX[shape], TY = SHAPE_TY[shape];
    return (double)n[0] * n[1] / (std::ceil(n[0] / TX) * TX * std::ceil(n[1] / TY) * TY);
  };
  if (ph.ndim == 3 && (ph.nvar == NVAR || ph.precision == AMR_PREC_MIXED) && lane_use(5) >= 0.9) return 5;
  const double u1 = lane_use(1), us = lane_use(SHAPE_SMALL);
  return (u1 < 0.5 && us > u1) ? SHAPE_SMALL : 1;
}

}  // namespace

extern "C" amr_status amr_patch_rk2_step_noalloc(const amr_patch_desc* patch, const amr_physics* phys, double* U,
                                                 const double* dt_dev, int32_t* flag_dev, hipStream_t stream) {
  if (!patch || !phys || !U || !dt_dev || !flag_dev) return AMR_EINVAL;
  amr_status st = validate_patches(patch, 1, phys);
  if (st != AMR_OK) return st;
  if (patch->level != 0) return AMR_EINVAL;
  for (int f = 0; f < 2 * phys->ndim; ++f)
    if (patch->bc[f] == AMR_BC_EXTERNAL) return AMR_EINVAL;  // a lone patch has no source for them

  PatchDev P{};
  P.off = patch->offset;
  P.level = 0;
  int64_t S = 1;
  for (int d = 0; d < 3; ++d) {
    P.n[d] = patch->n[d];
    P.g[d] = d < phys->ndim ? patch->ng : 0;
    P.s[d] = P.n[d] + 2 * P.g[d];
    P.dx[d] = phys->dx0[d];
    P.rdx[d] = 1.0 / P.dx[d];
    S *= P.s[d];
  }
  P.S = S;
  for (int f = 0; f < 6; ++f) {
    P.bc[f] = patch->bc[f];
    P.reg[f] = -1;
  }
  // U^(1) in the scratch: the active cells alone, from its start
  P.off1 = 0;
  P.S1 = (int64_t)P.n[0] * P.n[1] * P.n[2];
  for (int d = 0; d < 3; ++d) {
    P.s1[d] = P.n[d];
    P.g1[d] = 0;
  }

  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return AMR_EHIP;
  if (dev < 0 || dev >= MAX_DEVICES) return AMR_EINVAL;
  const int mixed = phys->precision == AMR_PREC_MIXED;
  const int shape = lone_patch_shape(*phys, P.n);
  int occ1 = 0, occ2 = 0, ncu = 0;
  unsigned char* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
      void* ptr = nullptr;
      if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return AMR_EHIP;
      int cu = 0;
      if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu < 1)
        return AMR_EHIP;
      g_scratch[dev] = static_cast<unsigned char*>(ptr);
      g_ncu[dev] = cu;
    }
    base = g_scratch[dev];
    ncu = g_ncu[dev];
    occ1 = occupancy(phys->nvar, mixed, shape, 1);
    occ2 = occupancy(phys->nvar, mixed, shape, 2);
  }

  // tiles: column blocks of the shape, z slabs balanced as the table's automatic choice
  const int TX = SHAPE_TX[shape], TY = SHAPE_TY[shape], W = shape_tiles_per_wg(shape);
  const int ntx = (P.n[0] + TX - 1) / TX, nty = (P.n[1] + TY - 1) / TY;
  const int64_t G = (int64_t)std::min(occ2 * ncu, 2 * ncu) * W;
  const int zs = phys->ndim == 3 ? balanced_zslab((int64_t)ntx * nty, P.n[2], G) : 1;
  const int64_t nzs = (P.n[2] + zs - 1) / zs;
  const int64_t L64 = (int64_t)ntx * nty * nzs;
  const size_t tile_bytes = (size_t)((L64 * (int64_t)sizeof(Tile) + 255) / 256 * 256);
  const size_t need = HDR_BYTES + tile_bytes + sizeof(double) * (size_t)phys->nvar * (size_t)P.S1;
  if (L64 > (1 << 30) || need > SCRATCH_BYTES) {
    fprintf(stderr,
            "amr_patch_rk2_step_noalloc: the patch needs %zu bytes of scratch, more than the %zu the library "
            "holds per GPU\n",
            need, SCRATCH_BYTES);
    return AMR_EINVAL;
  }
  const int L = (int)L64;
  PatchDev* pd = reinterpret_cast<PatchDev*>(base);
  Tile* tiles = reinterpret_cast<Tile*>(base + HDR_BYTES);
  double* U1 = reinterpret_cast<double*>(base + HDR_BYTES + tile_bytes);

  hipLaunchKernelGGL(noalloc_tiles, dim3((L + 255) / 256), dim3(256), 0, stream, P, pd, tiles, L, W, ntx, nty, TX,
                     TY, zs);
  if (hipGetLastError() != hipSuccess) return AMR_EHIP;

  auto grid_of = [&](int per_cu) {
    const int g = std::max(1, std::min((L + W - 1) / W, per_cu * ncu));
    return g >= 8 ? g / 8 * 8 : g;
  };
  StageArgs a{};
  a.V = U;
  a.U0 = nullptr;
  a.out = U1;
  a.dt = dt_dev;
  a.patches = pd;
  a.tiles = tiles;
  a.ntiles = L;
  a.flag = flag_dev;
  a.smax = nullptr;
  a.reg = nullptr;
  a.c = consts_of_phys(*phys);
  if (launch_stage(phys->nvar, mixed, shape, 1, grid_of(occ1), stream, a) != hipSuccess) return AMR_EHIP;
  a.V = U1;
  a.U0 = U;
  a.out = U;
  if (launch_stage(phys->nvar, mixed, shape, 2, grid_of(occ2), stream, a) != hipSuccess) return AMR_EHIP;
  return AMR_OK;
}
