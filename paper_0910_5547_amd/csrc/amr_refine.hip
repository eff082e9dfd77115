// amr_refine.hip - gfx950 kernels of the coarse/fine coupling of a factor-2
// block-structured hierarchy (Sec. 3: Berger & Colella AMR; the paper keeps the
// hierarchy on the host and runs the per-grid update on the GPU):
//   prolong_ghosts   coarse -> fine EXTERNAL ghosts, conservative minmod-linear in
//                    space, linear in time between the coarse old and new states;
//   fill_phys_ghosts physical boundary ghosts of a coarse level written into
//                    storage (the prolongation stencil reads one layer of them);
//   flux_fix         refluxing: each uncovered coarse cell next to a fine patch
//                    swaps its own interface flux (recomputed bit for bit from the
//                    two saved stage inputs) for the fine registers' average;
//   restrict_cells   covered coarse cells <- mean of their 2^d children.
// Each op is a box of cells; a work list spreads the cells of all ops of a launch
// over the workgroups' lanes, one cell per lane.
#include "amr_device.h"
#include "amr_internal.h"

namespace amr {

__device__ __forceinline__ int64_t stride_of(const PatchDev& P, int d) {
  return d == 0 ? 1 : (d == 1 ? (int64_t)P.s[0] : (int64_t)P.s[0] * P.s[1]);
}

// ---------------------------------------------------------------- prolongation
// Coarse state at time fraction alpha between the old and new states: linear in time.
__device__ __forceinline__ double at_time(const double* Cold, const double* Cnew, double alpha, int64_t e) {
  const double a = (1.0 - alpha) * Cold[e];
  const double b = alpha * Cnew[e];
  return a + b;
}

// Fine ghost cell = u(C) + sum_d (+-1/4) minmod(u(C+e_d) - u(C), u(C) - u(C-e_d)),
// u the time-interpolated coarse state, C the coarse cell holding the fine cell,
// + for the upper child along d.  The 2^d children of C average to u(C).
// Every coarse value is loaded before the first store (A, Cold and Cnew may share
// one arena, so a store between two loads would order them one round trip apart).
template <int NV>
__global__ __launch_bounds__(NT) void prolong_ghosts(const ProlongOp* __restrict__ ops, Work w,
                                                     const PatchDev* __restrict__ patches, double* A,
                                                     const double* Cold, const double* Cnew, double alpha,
                                                     int ndim) {
  int c;
  const int o = work_item(w, c);
  if (o < 0) return;
  const ProlongOp op = ops[o];
  const PatchDev& D = patches[op.dst];
  const PatchDev& Q = patches[op.src];
  int b[3];
  box_cell(op.sz, c, b);
  const int loc[3] = {op.lo[0] + b[0], op.lo[1] + b[1], op.lo[2] + b[2]};
  int L[3] = {0, 0, 0}, cq[3] = {0, 0, 0};
  for (int d = 0; d < ndim; ++d) {
    L[d] = loc[d] + op.foff[d];
    cq[d] = (L[d] >> 1) - op.clo[d];
  }
  const int64_t ed = cell_elem(D, loc[0], loc[1], loc[2]);
  const int64_t e0 = cell_elem(Q, cq[0], cq[1], cq[2]);
  const int64_t DS = D.S, QS = Q.S;
  // (an inactive dimension's neighbours are the cell itself: loaded, never used)
  const int64_t qs[3] = {1, ndim > 1 ? (int64_t)Q.s[0] : 0, ndim > 2 ? (int64_t)Q.s[0] * Q.s[1] : 0};
  double u0[NV], up[3][NV], um[3][NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int64_t ev = e0 + v * QS;
    u0[v] = at_time(Cold, Cnew, alpha, ev);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      up[d][v] = at_time(Cold, Cnew, alpha, ev + qs[d]);
      um[d][v] = at_time(Cold, Cnew, alpha, ev - qs[d]);
    }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double val = u0[v];
#pragma unroll
    for (int d = 0; d < 3; ++d)
      if (d < ndim) {
        const double sg = minmod2(up[d][v] - u0[v], u0[v] - um[d][v]);
        const double sgn = (L[d] & 1) ? 0.25 : -0.25;
        val = val + sgn * sg;
      }
    A[ed + v * DS] = val;
  }
}

// ---------------------------------------------------------------- physical ghosts
template <int NV>
__global__ __launch_bounds__(NT) void fill_phys_ghosts(const PhysOp* __restrict__ ops, Work w,
                                                       const PatchDev* __restrict__ patches, double* A) {
  int c;
  const int o = work_item(w, c);
  if (o < 0) return;
  const PhysOp op = ops[o];
  const PatchDev& P = patches[op.patch];
  int b[3];
  box_cell(op.sz, c, b);
  const int i = op.lo[0] + b[0], j = op.lo[1] + b[1], k = op.lo[2] + b[2];
  double u[NV];
  load_cons<NV>(A, P, i, j, k, u);  // the boundary condition's index map
  const int64_t e = cell_elem(P, i, j, k);
#pragma unroll
  for (int v = 0; v < NV; ++v) A[e + v * P.S] = u[v];
}

// ---------------------------------------------------------------- refluxing
// Face flux of coarse patch Q at face f along d (between Q-local cells f-1 and f),
// at the other coordinates of c, from stage input S: the same reconstruction and
// Riemann flux, with the same operations, as the stage kernel's face of that patch.
template <typename RT, int NV>
__device__ void coarse_face_flux(const double* S, const PatchDev& Q, int d, int f, const int c[3],
                                 const Consts& C, RT F[NV], int& bad) {
  const FaceConsts<RT> K{(RT)C.gamma, (RT)C.gm1, (RT)C.gg1, C.recon, (RT)C.ch, (RT)C.ch2};
  const RT theta = (RT)C.theta;
  RT q[4][NV];
  for (int m = 0; m < 4; ++m) {
    int x[3] = {c[0], c[1], c[2]};
    x[d] = f - 2 + m;
    double u[NV];
    load_cons<NV>(S, Q, x[0], x[1], x[2], u);
    bad |= cons2prim<RT, NV>(u, C, q[m]) ? 1 : 0;
  }
  RT qL[NV], qR[NV];
  const bool th1 = C.theta == 1.0;  // the stage kernel's limiter form (same values)
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const RT s1 = th1 ? plm_slope_t<RT, true>(q[0][v], q[1][v], q[2][v], theta)
                      : plm_slope_t<RT, false>(q[0][v], q[1][v], q[2][v], theta);
    const RT s2 = th1 ? plm_slope_t<RT, true>(q[1][v], q[2][v], q[3][v], theta)
                      : plm_slope_t<RT, false>(q[1][v], q[2][v], q[3][v], theta);
    qL[v] = madd(RT(0.5), s1, q[1][v]);
    qR[v] = madd(RT(-0.5), s2, q[2][v]);
  }
  if (d == 2) riemann_flux<RT, 2, NV>(qL, qR, K, C.flux, F);
  else riemann_flux_xy<RT, NV>(qL, qR, d == 1, K, C.flux, F);
}

// U_c += s (R_c - <R_f>) / dx_c with R_c = dt_c/2 (F(S1) + F(S2)) the coarse
// interface flux of the two stages and <R_f> the mean of the fine registers of the
// 2^(ndim-1) fine faces under it; s = +1 where the interface is the coarse cell's
// high face (side 0), -1 where it is its low face.
template <typename RT, int NV>
__global__ __launch_bounds__(NT) void flux_fix(const FixOp* __restrict__ ops, Work w,
                                               const PatchDev* __restrict__ patches, double* U,
                                               const double* S1, const double* S2, const double* __restrict__ reg,
                                               const double* dtc_ptr, Consts C, int* flag) {
  int c;
  const int o = work_item(w, c);
  if (o < 0) return;
  const double dtc = *dtc_ptr;
  int bad = 0;
  const FixOp op = ops[o];
  const PatchDev& Q = patches[op.coarse];
  const PatchDev& P = patches[op.fine];
  const int d = op.d, face = 2 * d + op.side;
  int b[3];
  box_cell(op.sz, c, b);
  const int cc[3] = {op.lo[0] + b[0], op.lo[1] + b[1], op.lo[2] + b[2]};
  const int fl = cc[d] + (op.side == 0 ? 1 : 0);
  RT F1[NV], F2[NV];
  coarse_face_flux<RT, NV>(S1, Q, d, fl, cc, C, F1, bad);
  coarse_face_flux<RT, NV>(S2, Q, d, fl, cc, C, F2, bad);
  // fine faces under this coarse face: 2 per active tangential dimension, summed
  // with dimension (d+2)%3 outer and (d+1)%3 inner; the register of a face is
  // laid out [v][upper tangential dim][lower tangential dim]
  const int da = (d + 1) % 3, db = (d + 2) % 3;
  const int tlo = da < db ? da : db;
  const int na = da < C.ndim ? 2 : 1, nb = db < C.ndim ? 2 : 1;
  const int fa0 = da < C.ndim ? 2 * cc[da] + op.fo[da] : 0;
  const int fb0 = db < C.ndim ? 2 * cc[db] + op.fo[db] : 0;
  const int64_t st_a = da == tlo ? 1 : (int64_t)P.n[tlo];
  const int64_t st_b = db == tlo ? 1 : (int64_t)P.n[tlo];
  const int64_t rs_v = (int64_t)P.n[da] * P.n[db];
  // (constant indices into P: a runtime index would move it to scratch memory)
  const int64_t rbase = face == 0 ? P.reg[0] : face == 1 ? P.reg[1] : face == 2 ? P.reg[2]
                      : face == 3 ? P.reg[3] : face == 4 ? P.reg[4] : P.reg[5];
  const int64_t e = cell_elem(Q, cc[0], cc[1], cc[2]);
  const double sgn = op.side == 0 ? 1.0 : -1.0;
  // the coarse cell's values are read before the first store
  double u[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = U[e + v * Q.S];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double Rf = 0.0;
    for (int yb = 0; yb < nb; ++yb)
      for (int xa = 0; xa < na; ++xa)
        Rf = Rf + reg[rbase + v * rs_v + (int64_t)(fb0 + yb) * st_b + (int64_t)(fa0 + xa) * st_a];
    Rf = Rf / (double)(na * nb);
    double Rc = 0.5 * dtc * (double)F1[v];
    Rc = Rc + 0.5 * dtc * (double)F2[v];
    U[e + v * Q.S] = u[v] + sgn * (Rc - Rf) / Q.dx[d];
  }
  if (bad) atomicOr(flag, 1);
}

// ---------------------------------------------------------------- restriction
template <int NV>
__global__ __launch_bounds__(NT) void restrict_cells(const RestrictOp* __restrict__ ops, Work w,
                                                     const PatchDev* __restrict__ patches, double* U, int ndim) {
  int c;
  const int o = work_item(w, c);
  if (o < 0) return;
  const RestrictOp op = ops[o];
  const PatchDev& Q = patches[op.coarse];
  const PatchDev& P = patches[op.fine];
  const int mz = ndim > 2 ? 2 : 1, my = ndim > 1 ? 2 : 1;
  const double inv = (double)(1 << ndim);
  int b[3];
  box_cell(op.sz, c, b);
  const int cc[3] = {op.lo[0] + b[0], op.lo[1] + b[1], op.lo[2] + b[2]};
  int f0[3] = {0, 0, 0};
  for (int d = 0; d < ndim; ++d) f0[d] = 2 * cc[d] + op.fo[d];
  const int64_t e = cell_elem(Q, cc[0], cc[1], cc[2]);
  // every child is read before the first store (one round trip, not one per variable)
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    acc[v] = 0.0;
    for (int dz = 0; dz < mz; ++dz)
      for (int dy = 0; dy < my; ++dy)
        for (int dx = 0; dx < 2; ++dx)
          acc[v] = acc[v] + U[cell_elem(P, f0[0] + dx, f0[1] + dy, f0[2] + dz) + v * P.S];
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) U[e + v * Q.S] = acc[v] / inv;
}

// ---------------------------------------------------------------- launchers
hipError_t launch_prolong(hipStream_t s, const ProlongOp* ops, const Work& w, const PatchDev* p, double* A,
                          const double* Cold, const double* Cnew, double alpha, int ndim, int nv) {
  if (nv == NVAR_MHD)
    hipLaunchKernelGGL(prolong_ghosts<NVAR_MHD>, dim3(w.nblk), dim3(NT), 0, s, ops, w, p, A, Cold, Cnew, alpha, ndim);
  else if (nv == NVAR_GLM)
    hipLaunchKernelGGL(prolong_ghosts<NVAR_GLM>, dim3(w.nblk), dim3(NT), 0, s, ops, w, p, A, Cold, Cnew, alpha, ndim);
  else hipLaunchKernelGGL(prolong_ghosts<NVAR>, dim3(w.nblk), dim3(NT), 0, s, ops, w, p, A, Cold, Cnew, alpha, ndim);
  return hipGetLastError();
}
hipError_t launch_phys(hipStream_t s, const PhysOp* ops, const Work& w, const PatchDev* p, double* A, int nv) {
  if (nv == NVAR_MHD) hipLaunchKernelGGL(fill_phys_ghosts<NVAR_MHD>, dim3(w.nblk), dim3(NT), 0, s, ops, w, p, A);
  else if (nv == NVAR_GLM) hipLaunchKernelGGL(fill_phys_ghosts<NVAR_GLM>, dim3(w.nblk), dim3(NT), 0, s, ops, w, p, A);
  else hipLaunchKernelGGL(fill_phys_ghosts<NVAR>, dim3(w.nblk), dim3(NT), 0, s, ops, w, p, A);
  return hipGetLastError();
}
template <int NV>
static void launch_flux_fix_nv(int mixed, hipStream_t s, const FixOp* ops, const Work& w, const PatchDev* p,
                               double* U, const double* S1, const double* S2, const double* reg, const double* dtc,
                               const Consts& C, int* flag) {
  if (mixed)
    hipLaunchKernelGGL((flux_fix<float, NV>), dim3(w.nblk), dim3(NT), 0, s, ops, w, p, U, S1, S2, reg, dtc, C, flag);
  else
    hipLaunchKernelGGL((flux_fix<double, NV>), dim3(w.nblk), dim3(NT), 0, s, ops, w, p, U, S1, S2, reg, dtc, C, flag);
}
hipError_t launch_flux_fix(int mixed, int nv, hipStream_t s, const FixOp* ops, const Work& w, const PatchDev* p,
                           double* U, const double* S1, const double* S2, const double* reg, const double* dtc,
                           const Consts& C, int* flag) {
  if (nv == NVAR_MHD) launch_flux_fix_nv<NVAR_MHD>(mixed, s, ops, w, p, U, S1, S2, reg, dtc, C, flag);
  else if (nv == NVAR_GLM) launch_flux_fix_nv<NVAR_GLM>(mixed, s, ops, w, p, U, S1, S2, reg, dtc, C, flag);
  else launch_flux_fix_nv<NVAR>(mixed, s, ops, w, p, U, S1, S2, reg, dtc, C, flag);
  return hipGetLastError();
}
hipError_t launch_restrict(hipStream_t s, const RestrictOp* ops, const Work& w, const PatchDev* p, double* U,
                           int ndim, int nv) {
  if (nv == NVAR_MHD) hipLaunchKernelGGL(restrict_cells<NVAR_MHD>, dim3(w.nblk), dim3(NT), 0, s, ops, w, p, U, ndim);
  else if (nv == NVAR_GLM) hipLaunchKernelGGL(restrict_cells<NVAR_GLM>, dim3(w.nblk), dim3(NT), 0, s, ops, w, p, U, ndim);
  else hipLaunchKernelGGL(restrict_cells<NVAR>, dim3(w.nblk), dim3(NT), 0, s, ops, w, p, U, ndim);
  return hipGetLastError();
}

}  // namespace amr
