// amr_kernels.hip - gfx950 kernels of the per-patch MOL hydro update
// (Wang, Abel & Kaehler, Secs. 4-5).
//
// Stage kernel.  One workgroup of 256 lanes owns a TX x TY block of cell
// columns of one patch and marches it through the planes z0..z1-1 of its tile:
//   * the z direction lives in registers: each lane keeps, for its own column,
//     the conserved state and primitives of planes z and z+1, the limited
//     z-slope of plane z and the z-face flux F_{z-1/2}, and loads plane z+2
//     per step (so every cell of the column is read from HBM once per stage);
//   * the x-y plane lives in LDS: the primitives of plane z for the block plus
//     a 2-cell face halo (no corners: the MOL stencil is a cross, Sec. 4);
//     every x- and y-face of the block is computed ONCE by one lane and stored
//     in LDS, so the two cells sharing a face use the same bits (the flux
//     difference telescopes: conservation holds to round-off in both
//     precisions);
//   * L(U) is accumulated in FP64 in the order x, y, z (MOL equation), and the
//     TVD-RK2 stage combine is applied in FP64 before one store per variable.
// Stage 2 writes U^{n+1} over U^n in place: U^n is only read at the cell being
// written.  Boundary conditions other than EXTERNAL are index maps applied at
// load time; EXTERNAL ghosts are read from storage (filled by copy_ghosts).
//
// The same source serves the plain form (one launch per patch, one tile per
// workgroup) and the batched form (one persistent launch over the tile list of
// all patches, workgroups striding through it).
#include "amr_device.h"
#include "amr_internal.h"

namespace amr {

template <typename RT, int TX, int TY, int STAGE>
__global__ __launch_bounds__(NT) void stage_kernel(StageArgs a) {
  static_assert(TX * TY == NT, "one lane per column of the tile");
  constexpr bool HASY = TY > 1;               // 1D tiles carry no y rows
  constexpr int PR = HASY ? TY + 4 : 1;       // LDS rows of the primitive plane
  constexpr int RO = HASY ? 2 : 0;            // row offset of tile row 0
  constexpr int FYR = HASY ? TY + 1 : 1;
  __shared__ RT sP[NVAR][PR][TX + 4];
  __shared__ RT sFx[NVAR][TY][TX + 1];
  __shared__ RT sFy[NVAR][FYR][TX];

  const Consts C = a.c;
  const FaceConsts<RT> K{(RT)C.gamma, (RT)C.gm1};
  const RT theta = (RT)C.theta;
  const int kind = C.flux;
  const int tid = threadIdx.x;
  const int cx = tid % TX, cy = tid / TX;
  const double dt = *a.dt;
  int bad = 0;
  double smax = 0.0;

  for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
    const Tile T = a.tiles[t];
    const PatchDev P = a.patches[T.patch];
    const int nxT = min(TX, P.n[0] - T.x0);
    const int nyT = HASY ? min(TY, P.n[1] - T.y0) : 1;
    const bool act = cx < nxT && cy < nyT;
    const int i = T.x0 + cx, j = T.y0 + cy;
    const bool hasz = C.ndim == 3;
    const bool hasy = HASY && C.ndim >= 2;

    // z-direction register queue (3D only)
    double Vz[NVAR], Vz1[NVAR];
    RT qz[NVAR], qz1[NVAR], sgz[NVAR], Fzm[NVAR];
    if (hasz && act) {
      double u[NVAR];
      RT qa[NVAR], qb[NVAR];
      load_cons(a.V, P, i, j, T.z0 - 2, u);
      bad |= cons2prim<RT>(u, C, qa);
      load_cons(a.V, P, i, j, T.z0 - 1, u);
      bad |= cons2prim<RT>(u, C, qb);
      load_cons(a.V, P, i, j, T.z0, Vz);
      bad |= cons2prim<RT>(Vz, C, qz);
      load_cons(a.V, P, i, j, T.z0 + 1, Vz1);
      bad |= cons2prim<RT>(Vz1, C, qz1);
      RT qL[NVAR], qR[NVAR];
#pragma unroll
      for (int v = 0; v < NVAR; ++v) {
        const RT sa = plm_slope<RT>(qa[v], qb[v], qz[v], theta);
        sgz[v] = plm_slope<RT>(qb[v], qz[v], qz1[v], theta);
        qL[v] = qb[v] + RT(0.5) * sa;
        qR[v] = qz[v] - RT(0.5) * sgz[v];
      }
      riemann_flux<RT, 2>(qL, qR, K, kind, Fzm);
    }

    for (int k = T.z0; k < T.z1; ++k) {
      // issue this step's HBM reads early: plane k+2 of the column, U^n of the cell
      double Vn2[NVAR], U0c[NVAR];
      if (hasz && act) load_cons(a.V, P, i, j, k + 2, Vn2);
      if (STAGE == 2 && act) {
        const int64_t e = cell_elem(P, i, j, k);
#pragma unroll
        for (int v = 0; v < NVAR; ++v) U0c[v] = a.U0[e + v * P.S];
      }
      double Vc[NVAR];
      RT qc[NVAR];
      if (act) {
        if (hasz) {
#pragma unroll
          for (int v = 0; v < NVAR; ++v) { Vc[v] = Vz[v]; qc[v] = qz[v]; }
        } else {
          load_cons(a.V, P, i, j, k, Vc);
          bad |= cons2prim<RT>(Vc, C, qc);
        }
#pragma unroll
        for (int v = 0; v < NVAR; ++v) sP[v][cy + RO][cx + 2] = qc[v];
      }
      // face halo of plane k: x halo = cols -2,-1,nxT,nxT+1 of every row;
      // y halo = rows -2,-1,nyT,nyT+1 of every column.
      const int nhx = 4 * nyT, nhy = hasy ? 4 * nxT : 0;
      for (int h = tid; h < nhx + nhy; h += NT) {
        int col, row;
        if (h < nhx) {
          row = h >> 2;
          const int w = h & 3;
          col = w < 2 ? w - 2 : nxT + (w - 2);
        } else {
          const int h2 = h - nhx;
          col = h2 >> 2;
          const int w = h2 & 3;
          row = w < 2 ? w - 2 : nyT + (w - 2);
        }
        double u[NVAR];
        RT q[NVAR];
        load_cons(a.V, P, T.x0 + col, T.y0 + row, k, u);
        bad |= cons2prim<RT>(u, C, q);
#pragma unroll
        for (int v = 0; v < NVAR; ++v) sP[v][row + RO][col + 2] = q[v];
      }
      __syncthreads();

      // every x- and y-face of the block, once: face f lies between tile cells f-1 and f
      const int nfx = (nxT + 1) * nyT, nfy = hasy ? nxT * (nyT + 1) : 0;
      for (int w = tid; w < nfx + nfy; w += NT) {
        RT q0[NVAR], q1[NVAR], q2[NVAR], q3[NVAR], F[NVAR];
        if (w < nfx) {
          const int row = w / (nxT + 1), f = w - row * (nxT + 1);
#pragma unroll
          for (int v = 0; v < NVAR; ++v) {
            q0[v] = sP[v][row + RO][f];
            q1[v] = sP[v][row + RO][f + 1];
            q2[v] = sP[v][row + RO][f + 2];
            q3[v] = sP[v][row + RO][f + 3];
          }
          face_flux4<RT, 0>(q0, q1, q2, q3, theta, K, kind, F);
#pragma unroll
          for (int v = 0; v < NVAR; ++v) sFx[v][row][f] = F[v];
        } else {
          const int w2 = w - nfx;
          const int f = w2 / nxT, col = w2 - f * nxT;
#pragma unroll
          for (int v = 0; v < NVAR; ++v) {
            q0[v] = sP[v][f][col + 2];
            q1[v] = sP[v][f + 1][col + 2];
            q2[v] = sP[v][f + 2][col + 2];
            q3[v] = sP[v][f + 3][col + 2];
          }
          face_flux4<RT, 1>(q0, q1, q2, q3, theta, K, kind, F);
#pragma unroll
          for (int v = 0; v < NVAR; ++v) sFy[v][f][col] = F[v];
        }
      }
      __syncthreads();

      if (act) {
        double L[NVAR];
#pragma unroll
        for (int v = 0; v < NVAR; ++v) L[v] = 0.0 - ((double)sFx[v][cy][cx + 1] - (double)sFx[v][cy][cx]) / P.dx[0];
        if (hasy) {
#pragma unroll
          for (int v = 0; v < NVAR; ++v)
            L[v] = L[v] - ((double)sFy[v][cy + 1][cx] - (double)sFy[v][cy][cx]) / P.dx[1];
        }
        if (hasz) {
          RT qn2[NVAR], sg1[NVAR], qL[NVAR], qR[NVAR], Fzp[NVAR];
          bad |= cons2prim<RT>(Vn2, C, qn2);
#pragma unroll
          for (int v = 0; v < NVAR; ++v) {
            sg1[v] = plm_slope<RT>(qz[v], qz1[v], qn2[v], theta);
            qL[v] = qz[v] + RT(0.5) * sgz[v];
            qR[v] = qz1[v] - RT(0.5) * sg1[v];
          }
          riemann_flux<RT, 2>(qL, qR, K, kind, Fzp);
#pragma unroll
          for (int v = 0; v < NVAR; ++v) {
            L[v] = L[v] - ((double)Fzp[v] - (double)Fzm[v]) / P.dx[2];
            Vz[v] = Vz1[v];
            Vz1[v] = Vn2[v];
            qz[v] = qz1[v];
            qz1[v] = qn2[v];
            sgz[v] = sg1[v];
            Fzm[v] = Fzp[v];
          }
        }
        // TVD-RK2 (Sec. 4): stage 1 U1 = U + dt L(U); stage 2 U^{n+1} = U^n/2 + (U1 + dt L(U1))/2
        const int64_t e = cell_elem(P, i, j, k);
        double un[NVAR];
#pragma unroll
        for (int v = 0; v < NVAR; ++v) {
          const double u1 = Vc[v] + dt * L[v];
          un[v] = (STAGE == 1) ? u1 : 0.5 * U0c[v] + 0.5 * u1;
          a.out[e + v * P.S] = un[v];
        }
        if (STAGE == 2 && a.smax != nullptr) smax = fmax(smax, cell_speed(un, C, P.dx, bad));
      }
      __syncthreads();
    }
    if (STAGE == 2 && a.smax != nullptr) {  // fused next-dt reduction, per level
      block_max_to(a.smax + P.level, smax);
      smax = 0.0;
    }
  }
  if (bad) atomicOr(a.flag, 1);
}

// ------------------------------------------------------------------ CFL
// Max signal speed over the active cells of the tile list (one plane of a tile
// per workgroup iteration); the block max is merged into smax[level] with a
// 64-bit atomicMax on the bit pattern (non-negative doubles order as integers).
__global__ __launch_bounds__(NT) void cfl_kernel(CflArgs a) {
  const Consts C = a.c;
  int bad = 0;
  for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
    const Tile T = a.tiles[t];
    const PatchDev P = a.patches[T.patch];
    const int nxT = min(a.tx, P.n[0] - T.x0), nyT = min(a.ty, P.n[1] - T.y0);
    const int per_plane = nxT * nyT;
    const int ncell = per_plane * (T.z1 - T.z0);
    double smax = 0.0;
    for (int c = threadIdx.x; c < ncell; c += NT) {
      const int kk = c / per_plane, r = c - kk * per_plane;
      const int jj = r / nxT, ii = r - jj * nxT;
      const int64_t e = cell_elem(P, T.x0 + ii, T.y0 + jj, T.z0 + kk);
      double u[NVAR];
#pragma unroll
      for (int v = 0; v < NVAR; ++v) u[v] = a.U[e + v * P.S];
      smax = fmax(smax, cell_speed(u, C, P.dx, bad));
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
// Same-level EXTERNAL ghost fill: one workgroup per copy op.
__global__ __launch_bounds__(NT) void copy_ghosts(const CopyOp* __restrict__ ops, int nops,
                                                  const PatchDev* __restrict__ patches, double* A) {
  for (int o = blockIdx.x; o < nops; o += gridDim.x) {
    const CopyOp op = ops[o];
    const PatchDev D = patches[op.dst], S = patches[op.src];
    const int n = op.sz[0] * op.sz[1] * op.sz[2];
    for (int c = threadIdx.x; c < n; c += NT) {
      const int kk = c / (op.sz[0] * op.sz[1]), r = c - kk * op.sz[0] * op.sz[1];
      const int jj = r / op.sz[0], ii = r - jj * op.sz[0];
      const int i = op.lo[0] + ii, j = op.lo[1] + jj, k = op.lo[2] + kk;
      const int64_t ed = cell_elem(D, i, j, k);
      const int64_t es = cell_elem(S, i + op.sh[0], j + op.sh[1], k + op.sh[2]);
#pragma unroll
      for (int v = 0; v < NVAR; ++v) A[ed + v * D.S] = A[es + v * S.S];
    }
  }
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
template <typename RT, int TX, int TY>
static hipError_t launch_stage_t(int stage, dim3 grid, hipStream_t s, const StageArgs& a) {
  if (stage == 1) hipLaunchKernelGGL((stage_kernel<RT, TX, TY, 1>), grid, dim3(NT), 0, s, a);
  else hipLaunchKernelGGL((stage_kernel<RT, TX, TY, 2>), grid, dim3(NT), 0, s, a);
  return hipGetLastError();
}

template <typename RT>
static hipError_t launch_stage_rt(int shape, int stage, dim3 grid, hipStream_t s, const StageArgs& a) {
  switch (shape) {
    case 0: return launch_stage_t<RT, 256, 1>(stage, grid, s, a);
    case 1: return launch_stage_t<RT, 32, 8>(stage, grid, s, a);
    case 2: return launch_stage_t<RT, 64, 4>(stage, grid, s, a);
    case 3: return launch_stage_t<RT, 16, 16>(stage, grid, s, a);
    case 4: return launch_stage_t<RT, 128, 2>(stage, grid, s, a);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_stage(int mixed, int shape, int stage, int grid, hipStream_t s, const StageArgs& a) {
  if (mixed) return launch_stage_rt<float>(shape, stage, dim3(grid), s, a);
  return launch_stage_rt<double>(shape, stage, dim3(grid), s, a);
}

const void* stage_kernel_ptr(int mixed, int shape, int stage) {
#define AMR_KP(RT, TX, TY)                                                                          \
  (stage == 1 ? reinterpret_cast<const void*>(&stage_kernel<RT, TX, TY, 1>)                         \
              : reinterpret_cast<const void*>(&stage_kernel<RT, TX, TY, 2>))
  if (mixed) {
    switch (shape) {
      case 0: return AMR_KP(float, 256, 1);
      case 1: return AMR_KP(float, 32, 8);
      case 2: return AMR_KP(float, 64, 4);
      case 3: return AMR_KP(float, 16, 16);
      case 4: return AMR_KP(float, 128, 2);
    }
  } else {
    switch (shape) {
      case 0: return AMR_KP(double, 256, 1);
      case 1: return AMR_KP(double, 32, 8);
      case 2: return AMR_KP(double, 64, 4);
      case 3: return AMR_KP(double, 16, 16);
      case 4: return AMR_KP(double, 128, 2);
    }
  }
#undef AMR_KP
  return nullptr;
}

hipError_t launch_cfl(int grid, hipStream_t s, const CflArgs& a) {
  hipLaunchKernelGGL(cfl_kernel, dim3(grid), dim3(NT), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_cfl_finalize(hipStream_t s, const unsigned long long* smax, int lmin, int lmax, int root,
                               double cfl, double* dt) {
  hipLaunchKernelGGL(cfl_finalize, dim3(1), dim3(64), 0, s, smax, lmin, lmax, root, cfl, dt);
  return hipGetLastError();
}
hipError_t launch_copy_ghosts(int grid, hipStream_t s, const CopyOp* ops, int nops, const PatchDev* p, double* A) {
  hipLaunchKernelGGL(copy_ghosts, dim3(grid), dim3(NT), 0, s, ops, nops, p, A);
  return hipGetLastError();
}
hipError_t launch_fill_u64(hipStream_t s, unsigned long long* p, int n, unsigned long long v) {
  hipLaunchKernelGGL(fill_u64, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_i32(hipStream_t s, int* p, int n, int v) {
  hipLaunchKernelGGL(fill_i32, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace amr
