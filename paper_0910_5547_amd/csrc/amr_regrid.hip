// amr_regrid.hip - gfx950 kernels on either side of the per-patch update for a
// dynamic hierarchy (the paper creates its hierarchy on the host, Sec. 3):
//   flag_cells   refinement flags by the density-gradient criterion, one lane per
//                active cell of the flagged level;
//   copy_cells_x cells of a new table's patches copied from an old table's arena.
#include "amr_device.h"
#include "amr_internal.h"

namespace amr {

// Density of the face neighbour of active cell c along +-d (s = +1 or -1): the
// boundary condition's index map, a direct sibling's cell, or ghost storage.
__device__ __forceinline__ double rho_neighbour(const double* U, const PatchDev& P, int c0, int c1, int c2, int d,
                                               int s) {
  int c[3] = {c0, c1, c2};
  const int raw = c[d] + s;
  bool flip = false;
  c[d] = map_index(raw, P.n[d], P.bc[2 * d], P.bc[2 * d + 1], flip);
  int64_t e = cell_elem(P, c[0], c[1], c[2]);
  const int f = 2 * d + (s > 0 ? 1 : 0);
  if ((raw < 0 || raw >= P.n[d]) && ((P.dmask >> f) & 1)) e += P.nbo[f];
  return U[e];
}

// Cell g of the list (the active cells of the patches plist[0..npl), patch after patch,
// x fastest) lies in patch plist[b] with cofs[b] <= g < cofs[b + 1].  A cell is flagged
// where |rho_n - rho_c| / min(rho_n, rho_c) > eps for a face neighbour n.
__global__ __launch_bounds__(NT) void flag_cells(const int* __restrict__ plist, const int64_t* __restrict__ cofs,
                                                 int npl, const PatchDev* __restrict__ patches,
                                                 const double* __restrict__ U, double eps, uint8_t* flags,
                                                 int ndim) {
  const int64_t g = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (g >= cofs[npl]) return;
  int lo = 0, hi = npl;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (cofs[mid] <= g) lo = mid;
    else hi = mid;
  }
  const PatchDev& P = patches[plist[lo]];
  const int64_t c = g - cofs[lo];
  const int64_t plane = (int64_t)P.n[0] * P.n[1];
  const int k = (int)(c / plane);
  const int r = (int)(c - k * plane);
  const int j = r / P.n[0], i = r - j * P.n[0];
  const double rc = U[cell_elem(P, i, j, k)];
  int f = 0;
  for (int d = 0; d < ndim; ++d)
    for (int s = -1; s <= 1; s += 2) {
      const double rn = rho_neighbour(U, P, i, j, k, d, s);
      if (fabs(rn - rc) / fmin(rn, rc) > eps) f = 1;
    }
  flags[g] = (uint8_t)f;
}

hipError_t launch_flag_cells(hipStream_t s, const int* plist, const int64_t* cofs, int npl, int64_t ncells,
                             const PatchDev* patches, const double* U, double eps, uint8_t* flags, int ndim) {
  if (ncells <= 0) return hipSuccess;
  const int64_t nb = (ncells + NT - 1) / NT;
  hipLaunchKernelGGL(flag_cells, dim3((unsigned)nb), dim3(NT), 0, s, plist, cofs, npl, patches, U, eps, flags, ndim);
  return hipGetLastError();
}

}  // namespace amr

namespace amr {

// Cells of a new table's patches taken from an old table's patches at the same level:
// op.dst (new table) box [lo, lo+sz) (dst-local) <- op.src (old table) cells at + sh;
// every variable is read before the first store.
template <int NV>
__global__ __launch_bounds__(NT) void copy_cells_x(const CopyOp* __restrict__ ops, Work w,
                                                   const PatchDev* __restrict__ pdst,
                                                   const PatchDev* __restrict__ psrc, double* Adst,
                                                   const double* __restrict__ Asrc) {
  int c;
  const int o = work_item(w, c);
  if (o < 0) return;
  const CopyOp op = ops[o];
  const PatchDev& D = pdst[op.dst];
  const PatchDev& S = psrc[op.src];
  int b[3];
  box_cell(op.sz, c, b);
  const int i = op.lo[0] + b[0], j = op.lo[1] + b[1], k = op.lo[2] + b[2];
  const int64_t ed = cell_elem(D, i, j, k);
  const int64_t es = cell_elem(S, i + op.sh[0], j + op.sh[1], k + op.sh[2]);
  double u[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = Asrc[es + v * S.S];
#pragma unroll
  for (int v = 0; v < NV; ++v) Adst[ed + v * D.S] = u[v];
}

hipError_t launch_copy_cells_x(hipStream_t s, const CopyOp* ops, const Work& w, const PatchDev* pdst,
                               const PatchDev* psrc, double* Adst, const double* Asrc, int nv) {
  if (nv == NVAR_MHD)
    hipLaunchKernelGGL(copy_cells_x<NVAR_MHD>, dim3(w.nblk), dim3(NT), 0, s, ops, w, pdst, psrc, Adst, Asrc);
  else if (nv == NVAR_GLM)
    hipLaunchKernelGGL(copy_cells_x<NVAR_GLM>, dim3(w.nblk), dim3(NT), 0, s, ops, w, pdst, psrc, Adst, Asrc);
  else hipLaunchKernelGGL(copy_cells_x<NVAR>, dim3(w.nblk), dim3(NT), 0, s, ops, w, pdst, psrc, Adst, Asrc);
  return hipGetLastError();
}

}  // namespace amr
