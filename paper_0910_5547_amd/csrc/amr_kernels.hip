// amr_kernels.hip - gfx950 kernels of the per-patch MOL hydro update
// (Wang, Abel & Kaehler, Secs. 4-5).
//
// Stage kernel.  One workgroup of 256 lanes owns a TX x TY block of cell
// columns of one patch and marches it through the planes z0..z1-1 of its tile:
//   * the z direction lives in registers: each lane keeps, for its own column,
//     the primitives of planes z and z+1, the limited z-slope of plane z and the
//     z-face flux F_{z-1/2}, and loads plane z+2 per step, so every cell of the
//     column is read from HBM once per stage (its conserved state waits in a
//     lane-private LDS ring until the update two planes later);
//   * the x-y plane lives in LDS: the primitives of plane z for the block plus
//     a 2-cell face halo (no corners: the MOL stencil is a cross, Sec. 4).
//     Per plane: (1) every cell's limited
//     slope in x and y is computed once and turned into the two face states it
//     contributes (q - sigma/2 on its low face, q + sigma/2 on its high face);
//     (2) every x- and y-face flux of the block is computed once, by one lane,
//     from its two face states, and written over them; (3) each cell reads its
//     two x and two y fluxes.  The two cells sharing a face use the same bits,
//     so the flux difference telescopes and totals are conserved to round-off
//     in both precisions.  The z-face flux of each column is computed between
//     (2) and (3), overlapping with the other waves' face work;
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

// Occupancy target: three 256-lane workgroups per CU for the FP32-reconstruction
// instantiations (<= 168 VGPRs), two for FP64 (LDS-bound at two per CU anyway).
// REC: record fine-face fluxes into the refluxing registers (patches of levels > 0).
// TH1: the limiter parameter is 1 (the two-argument minmod, see plm_slope_t).
template <typename RT, int TX, int TY, int STAGE, bool REC, bool TH1>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(Fast<RT>::value ? 3 : 2)))
void stage_kernel(StageArgs a) {
  static_assert(TX * TY == NT, "one lane per column of the tile");
  constexpr bool FAST = Fast<RT>::value;
  constexpr bool HASY = TY > 1;          // 1D tiles carry no y rows
  constexpr int PR = HASY ? TY + 4 : 1;  // LDS rows of the primitive plane
  constexpr int RO = HASY ? 2 : 0;       // row offset of tile row 0
  constexpr int YR = HASY ? TY + 1 : 1;  // y-face rows
  constexpr int HMAX = HASY ? (4 * (TX + TY) + NT - 1) / NT : 1;  // halo cells per lane
  // face slots: x faces first, slot row*(nxT+1) + f, then y faces, slot nfx + f*nxT + col
  constexpr int NSLOT = TY * (TX + 1) + (HASY ? YR * TX : 0);
  __shared__ RT sP[1][NVAR][PR][TX + 4];        // primitives of the plane (+ face halo)
  __shared__ RT sFL[NVAR][NSLOT], sFR[NVAR][NSLOT];  // left/right face states; sFL then holds the flux
  // conserved state of this lane's cell in planes k and k+1 (3D), for the update:
  // lane-private, kept in LDS rather than registers or a second read (FP32
  // instantiations; the FP64 ones re-read the cell, their LDS budget being spent)
  constexpr bool RING = FAST;
  __shared__ double sV[RING ? 2 : 1][NVAR][RING ? NT : 1];

  const Consts C = a.c;
  const FaceConsts<RT> K{(RT)C.gamma, (RT)C.gm1, (RT)C.gg1};
  const RT theta = (RT)C.theta;
  const int kind = C.flux;
  const int tid = threadIdx.x;
  const int cx = tid % TX, cy = tid / TX;
  const double dt = *a.dt;
  int bad = 0;
  double smax = 0.0;
  constexpr int buf = 0;

  for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
    const Tile T = a.tiles[t];
    const PatchDev P = a.patches[T.patch];
    const int nxT = min(TX, P.n[0] - T.x0);
    const int nyT = HASY ? min(TY, P.n[1] - T.y0) : 1;
    const bool act = cx < nxT && cy < nyT;
    const int i = T.x0 + cx, j = T.y0 + cy;
    const bool hasz = C.ndim == 3;
    const bool hasy = HASY && C.ndim >= 2;
    // element of this lane's column in plane 0 (the column is inside the patch) and
    // the stride between planes; plane k of the column is at col0 + kk * pstride,
    // kk being k after the z boundary map (uniform across the workgroup)
    const int64_t pstride = (int64_t)P.s[0] * P.s[1];
    // (inactive lanes of a ragged tile point at the tile's last active column, so that
    // every lane can issue the plane prefetch below unconditionally)
    const int ic = min(i, P.n[0] - 1), jc = min(j, P.n[1] - 1);
    const int64_t col0 = P.off + (int64_t)P.g[2] * pstride + (int64_t)(jc + P.g[1]) * P.s[0] + (ic + P.g[0]);
    // The REFLECT sign flip of the normal momentum is applied where loaded values
    // are used, not at the load: a flip right after the load would make the load
    // wait for its data, and the prefetches below would stop hiding latency.
    auto load_col_raw = [&](int kz, double u[NVAR]) -> bool {  // true: negate u[3]
      bool fz = false;
      const int kk = map_index(kz, P.n[2], P.bc[4], P.bc[5], fz);
      const int64_t e = col0 + (int64_t)kk * pstride;
#pragma unroll
      for (int v = 0; v < NVAR; ++v) u[v] = a.V[e + v * P.S];
      return fz;
    };
    auto load_col = [&](int kz, double u[NVAR]) {
      if (load_col_raw(kz, u)) u[3] = -u[3];
    };

    // z-direction register queue (3D only): primitives of planes k and k+1, the
    // z-slope of plane k and the flux F_{k-1/2}
    RT qz[NVAR], qz1[NVAR], sgz[NVAR], Fzm[NVAR];
    if (hasz) {
      double u[NVAR];
      RT qa[NVAR], qb[NVAR];
      load_col(T.z0 - 2, u);
      bad |= cons2prim<RT>(u, C, qa);
      load_col(T.z0 - 1, u);
      bad |= cons2prim<RT>(u, C, qb);
      load_col(T.z0, u);
      bad |= cons2prim<RT>(u, C, qz);
      if constexpr (RING) {
#pragma unroll
        for (int v = 0; v < NVAR; ++v) sV[T.z0 & 1][v][tid] = u[v];
      }
      load_col(T.z0 + 1, u);
      bad |= cons2prim<RT>(u, C, qz1);
      if constexpr (RING) {
#pragma unroll
        for (int v = 0; v < NVAR; ++v) sV[(T.z0 + 1) & 1][v][tid] = u[v];
      }
      RT qL[NVAR], qR[NVAR];
#pragma unroll
      for (int v = 0; v < NVAR; ++v) {
        const RT sa = plm_slope_t<RT, TH1>(qa[v], qb[v], qz[v], theta);
        sgz[v] = plm_slope_t<RT, TH1>(qb[v], qz[v], qz1[v], theta);
        qL[v] = madd(RT(0.5), sa, qb[v]);
        qR[v] = madd(RT(-0.5), sgz[v], qz[v]);
      }
      riemann_flux<RT, 2>(qL, qR, K, kind, Fzm);
    }
    // fine-face flux registers (Berger-Colella refluxing): faces on this patch's
    // boundary whose flux the coarse level must later see, dt/2 per stage
    const double hdt = 0.5 * dt;
    const bool rec = REC && P.level > 0;
    const bool rec_xy = rec && ((T.x0 == 0 && P.reg[0] >= 0) || (T.x0 + nxT == P.n[0] && P.reg[1] >= 0) ||
                                (hasy && T.y0 == 0 && P.reg[2] >= 0) ||
                                (hasy && T.y0 + nyT == P.n[1] && P.reg[3] >= 0));
    if (REC && hasz && act && rec && T.z0 == 0 && P.reg[4] >= 0) {
#pragma unroll
      for (int v = 0; v < NVAR; ++v) {
        double* r = a.reg + P.reg[4] + ((int64_t)v * P.n[1] + j) * P.n[0] + i;
        *r = *r + hdt * (double)Fzm[v];
      }
    }

    // Face halo of every plane: x halo = cols -2,-1,nxT,nxT+1 of every row, y halo =
    // rows -2,-1,nyT,nyT+1 of every column.  Lane tid owns halo cells tid + s*NT; their
    // conserved states are loaded one plane ahead so the loads' latency overlaps a
    // whole plane of work.
    const int nhx = 4 * nyT, nhy = hasy ? 4 * nxT : 0;
    int hrow[HMAX], hcol[HMAX], hflip[HMAX];
    int64_t hbase[HMAX];  // element of the halo cell's source in plane 0 (boundary maps applied)
    double Hn[HMAX][NVAR];
    auto load_halo = [&](int s, int kz, double u[NVAR]) {  // raw: hflip applied at use
      const int64_t e = hbase[s] + (int64_t)kz * pstride;
#pragma unroll
      for (int v = 0; v < NVAR; ++v) u[v] = a.V[e + v * P.S];
    };
#pragma unroll
    for (int s = 0; s < HMAX; ++s) {
      const int h = tid + s * NT;
      if (h < nhx) {
        hrow[s] = h >> 2;
        const int w = h & 3;
        hcol[s] = w < 2 ? w - 2 : nxT + (w - 2);
      } else {
        const int h2 = h - nhx;
        hcol[s] = h2 >> 2;
        const int w = h2 & 3;
        hrow[s] = w < 2 ? w - 2 : nyT + (w - 2);
      }
      bool fx = false, fy = false;
      const int ii = map_index(T.x0 + hcol[s], P.n[0], P.bc[0], P.bc[1], fx);
      const int jj = map_index(T.y0 + hrow[s], P.n[1], P.bc[2], P.bc[3], fy);
      hflip[s] = fx ? 1 : (fy ? 2 : 0);
      hbase[s] = P.off + (int64_t)P.g[2] * pstride + (int64_t)(jj + P.g[1]) * P.s[0] + (ii + P.g[0]);
      if (h < nhx + nhy) load_halo(s, T.z0, Hn[s]);
    }
    // lane -> (row, column) of the flattened slope and face index spaces: exact
    // float reciprocals (indices < 2^10, divisors <= 2^9) instead of integer division
    const float r_x1 = 1.0f / (float)(nxT + 1), r_x2 = 1.0f / (float)(nxT + 2), r_x0 = 1.0f / (float)nxT;
    auto idiv = [](int w, float r) { return (int)(((float)w + 0.5f) * r); };

    for (int k = T.z0; k < T.z1; ++k) {
      // this step's HBM read first: plane k+2 of the column in 3D (consumed by the z
      // flux after the x-y work), plane k itself in 1D/2D.  Issued by every lane
      // without a branch, so that nothing between here and the use waits for it.
      double Vn2[NVAR];
      const bool fz2 = load_col_raw(hasz ? k + 2 : k, Vn2);
      // halo of plane k (prefetched) into LDS, then prefetch the halo of plane k+1
#pragma unroll
      for (int s = 0; s < HMAX; ++s) {
        if (tid + s * NT < nhx + nhy) {
          RT q[NVAR];
          if (hflip[s] == 1) Hn[s][1] = -Hn[s][1];
          if (hflip[s] == 2) Hn[s][2] = -Hn[s][2];
          bad |= cons2prim<RT>(Hn[s], C, q);
#pragma unroll
          for (int v = 0; v < NVAR; ++v) sP[buf][v][hrow[s] + RO][hcol[s] + 2] = q[v];
          if (k + 1 < T.z1) load_halo(s, k + 1, Hn[s]);
        }
      }
      // (every lane computes; inactive lanes of ragged tiles hold a copy of an active
      // column and only skip the shared and global writes: a branch around loads or
      // their uses would leave loads pending on one path, and the next iteration would
      // wait for all memory at its first prefetch)
      {
        RT qc[NVAR];
        if (hasz) {
#pragma unroll
          for (int v = 0; v < NVAR; ++v) qc[v] = qz[v];
        } else {
          // (the empty asm keeps this use inside the 1D/2D branch: hoisted above it, the
          // conversion would make 3D wait here for its plane k+2 prefetch)
#pragma unroll
          for (int v = 0; v < NVAR; ++v) asm volatile("" : "+v"(Vn2[v]));
          if (fz2) Vn2[3] = -Vn2[3];
          bad |= cons2prim<RT>(Vn2, C, qc);
          if constexpr (RING) {
#pragma unroll
            for (int v = 0; v < NVAR; ++v) sV[k & 1][v][tid] = Vn2[v];
          }
        }
        if (act) {
#pragma unroll
          for (int v = 0; v < NVAR; ++v) sP[buf][v][cy + RO][cx + 2] = qc[v];
        }
      }
      __syncthreads();  // (A) plane primitives ready; previous plane's fluxes consumed

      // (1) slopes, once per cell: x for cells -1..nxT of every row, y for rows -1..nyT of
      // every column.  One code path for both: centre cell, neighbour stride, and the
      // two face slots the cell's states go to (its low face's right state and its
      // high face's left state).
      const int nsx = (nxT + 2) * nyT, nsy = hasy ? nxT * (nyT + 2) : 0;
      const int nfx = (nxT + 1) * nyT, nfy = hasy ? nxT * (nyT + 1) : 0;
      for (int w = tid; w < nsx + nsy; w += NT) {
        int pc, stride, slo, shi;  // LDS cell, stride to its neighbours, slots (-1: none)
        if (w < nsx) {
          const int row = idiv(w, r_x2), c = w - row * (nxT + 2) - 1;
          pc = (row + RO) * (TX + 4) + c + 2;
          stride = 1;
          slo = c >= 0 ? row * (nxT + 1) + c : -1;
          shi = c < nxT ? row * (nxT + 1) + c + 1 : -1;
        } else {
          const int w2 = w - nsx;
          const int r = idiv(w2, r_x0) - 1, col = w2 - (r + 1) * nxT;
          pc = (r + RO) * (TX + 4) + col + 2;
          stride = TX + 4;
          slo = r >= 0 ? nfx + r * nxT + col : -1;
          shi = r < nyT ? nfx + (r + 1) * nxT + col : -1;
        }
#pragma unroll
        for (int v = 0; v < NVAR; ++v) {
          const RT* pl = &sP[buf][v][0][0];
          const RT qm = pl[pc - stride], q0 = pl[pc], qp = pl[pc + stride];
          const RT sg = plm_slope_t<RT, TH1>(qm, q0, qp, theta);
          if (slo >= 0) sFR[v][slo] = madd(RT(-0.5), sg, q0);  // right state of the cell's low face
          if (shi >= 0) sFL[v][shi] = madd(RT(0.5), sg, q0);   // left state of its high face
        }
      }
      __syncthreads();  // (B) face states ready

      // the stage input (from the lane's LDS ring; FP64 instantiations re-read it) and
      // (stage 2) U^n of this cell, for the update: read here so the face pass hides
      // the latency
      double Vc[NVAR], U0c[NVAR];
      const int64_t ecell = col0 + (int64_t)k * pstride;
      {
        const int64_t e = ecell;
        if constexpr (RING) {
#pragma unroll
          for (int v = 0; v < NVAR; ++v) Vc[v] = sV[k & 1][v][tid];
        } else {
#pragma unroll
          for (int v = 0; v < NVAR; ++v) Vc[v] = a.V[e + v * P.S];
        }
        if (STAGE == 2) {
#pragma unroll
          for (int v = 0; v < NVAR; ++v) U0c[v] = a.U0[e + v * P.S];
        }
      }

      // (2) every x- and y-face flux of the block, once, written over its left state
      for (int w = tid; w < nfx + nfy; w += NT) {
        RT qL[NVAR], qR[NVAR], F[NVAR];
#pragma unroll
        for (int v = 0; v < NVAR; ++v) { qL[v] = sFL[v][w]; qR[v] = sFR[v][w]; }
        riemann_flux_xy<RT>(qL, qR, w >= nfx, K, kind, F);
#pragma unroll
        for (int v = 0; v < NVAR; ++v) sFL[v][w] = F[v];
        if (REC && rec_xy) {
          int64_t base = -1, stride = 0;
          // (constant indices into P: a runtime index would move P to scratch memory)
          if (w < nfx) {
            const int row = idiv(w, r_x1), f = w - row * (nxT + 1);
            const int gi = T.x0 + f, gj = T.y0 + row;
            const int64_t rg = gi == 0 ? P.reg[0] : (gi == P.n[0] ? P.reg[1] : -1);
            if (rg >= 0) {
              base = rg + (int64_t)k * P.n[1] + gj;
              stride = (int64_t)P.n[2] * P.n[1];
            }
          } else {
            const int w2 = w - nfx;
            const int f = idiv(w2, r_x0), col = w2 - f * nxT;
            const int gj = T.y0 + f, gi = T.x0 + col;
            const int64_t rg = gj == 0 ? P.reg[2] : (gj == P.n[1] ? P.reg[3] : -1);
            if (rg >= 0) {
              base = rg + (int64_t)k * P.n[0] + gi;
              stride = (int64_t)P.n[2] * P.n[0];
            }
          }
          if (base >= 0) {
#pragma unroll
            for (int v = 0; v < NVAR; ++v) {
              double* r = a.reg + base + v * stride;
              *r = *r + hdt * (double)F[v];
            }
          }
        }
      }
      // z-face flux F_{k+1/2} of this column from the register queue
      RT Fzp[NVAR], qn2[NVAR], sg1[NVAR];
      if (hasz) {
        RT qL[NVAR], qR[NVAR];
        if (fz2) Vn2[3] = -Vn2[3];
        bad |= cons2prim<RT>(Vn2, C, qn2);
#pragma unroll
        for (int v = 0; v < NVAR; ++v) {
          sg1[v] = plm_slope_t<RT, TH1>(qz[v], qz1[v], qn2[v], theta);
          qL[v] = madd(RT(0.5), sgz[v], qz[v]);
          qR[v] = madd(RT(-0.5), sg1[v], qz1[v]);
        }
        riemann_flux<RT, 2>(qL, qR, K, kind, Fzp);
        if (REC && act && rec && k == P.n[2] - 1 && P.reg[5] >= 0) {
#pragma unroll
          for (int v = 0; v < NVAR; ++v) {
            double* r = a.reg + P.reg[5] + ((int64_t)v * P.n[1] + j) * P.n[0] + i;
            *r = *r + hdt * (double)Fzp[v];
          }
        }
      }
      __syncthreads();  // (C) fluxes ready

      // (3) L(U) in the order x, y, z, then the TVD-RK2 stage combine
      {
        double L[NVAR];
        const int sx = cy * (nxT + 1) + cx, sy = nfx + cy * nxT + cx;
#pragma unroll
        for (int v = 0; v < NVAR; ++v) {
          const double d = (double)sFL[v][sx + 1] - (double)sFL[v][sx];
          if constexpr (FAST) L[v] = -d * P.rdx[0];
          else L[v] = 0.0 - d / P.dx[0];
        }
        if (hasy) {
#pragma unroll
          for (int v = 0; v < NVAR; ++v) {
            const double d = (double)sFL[v][sy + nxT] - (double)sFL[v][sy];
            if constexpr (FAST) L[v] = fma(-d, P.rdx[1], L[v]);
            else L[v] = L[v] - d / P.dx[1];
          }
        }
        if (hasz) {
#pragma unroll
          for (int v = 0; v < NVAR; ++v) {
            const double d = (double)Fzp[v] - (double)Fzm[v];
            if constexpr (FAST) L[v] = fma(-d, P.rdx[2], L[v]);
            else L[v] = L[v] - d / P.dx[2];
            if constexpr (RING) sV[k & 1][v][tid] = Vn2[v];  // plane k+2 takes plane k's slot
            qz[v] = qz1[v];
            qz1[v] = qn2[v];
            sgz[v] = sg1[v];
            Fzm[v] = Fzp[v];
          }
        }
        // TVD-RK2 (Sec. 4): stage 1 U1 = U + dt L(U); stage 2 U^{n+1} = U^n/2 + (U1 + dt L(U1))/2
        const int64_t e = ecell;
        double un[NVAR];
#pragma unroll
        for (int v = 0; v < NVAR; ++v) {
          double u1;
          if constexpr (FAST) u1 = fma(dt, L[v], Vc[v]);
          else u1 = Vc[v] + dt * L[v];
          un[v] = (STAGE == 1) ? u1 : 0.5 * U0c[v] + 0.5 * u1;
        }
        if (act) {
#pragma unroll
          for (int v = 0; v < NVAR; ++v) a.out[e + v * P.S] = un[v];
          if (STAGE == 2 && a.smax != nullptr) smax = fmax(smax, cell_speed<FAST>(un, C, P, bad));
        }
      }
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
template <bool FAST>
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
      smax = fmax(smax, cell_speed<FAST>(u, C, P, bad));
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
// Same-level EXTERNAL ghost fill, one ghost cell per lane.
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
#pragma unroll
  for (int v = 0; v < NVAR; ++v) A[ed + v * D.S] = A[es + v * S.S];
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
template <typename RT, int TX, int TY, int STAGE>
static hipError_t launch_stage_t(dim3 grid, hipStream_t s, const StageArgs& a) {
  const bool th1 = a.c.theta == 1.0;
  if (a.reg) {
    if (th1) hipLaunchKernelGGL((stage_kernel<RT, TX, TY, STAGE, true, true>), grid, dim3(NT), 0, s, a);
    else hipLaunchKernelGGL((stage_kernel<RT, TX, TY, STAGE, true, false>), grid, dim3(NT), 0, s, a);
  } else {
    if (th1) hipLaunchKernelGGL((stage_kernel<RT, TX, TY, STAGE, false, true>), grid, dim3(NT), 0, s, a);
    else hipLaunchKernelGGL((stage_kernel<RT, TX, TY, STAGE, false, false>), grid, dim3(NT), 0, s, a);
  }
  return hipGetLastError();
}

template <typename RT, int TX, int TY>
static hipError_t launch_stage_s(int stage, dim3 grid, hipStream_t s, const StageArgs& a) {
  return stage == 1 ? launch_stage_t<RT, TX, TY, 1>(grid, s, a) : launch_stage_t<RT, TX, TY, 2>(grid, s, a);
}

template <typename RT>
static hipError_t launch_stage_rt(int shape, int stage, dim3 grid, hipStream_t s, const StageArgs& a) {
  switch (shape) {
    case 0: return launch_stage_s<RT, 256, 1>(stage, grid, s, a);
    case 1: return launch_stage_s<RT, 32, 8>(stage, grid, s, a);
    case 2: return launch_stage_s<RT, 64, 4>(stage, grid, s, a);
    case 3: return launch_stage_s<RT, 16, 16>(stage, grid, s, a);
    case 4: return launch_stage_s<RT, 128, 2>(stage, grid, s, a);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_stage(int mixed, int shape, int stage, int grid, hipStream_t s, const StageArgs& a) {
  if (mixed) return launch_stage_rt<float>(shape, stage, dim3(grid), s, a);
  return launch_stage_rt<double>(shape, stage, dim3(grid), s, a);
}

// The non-recording, theta = 1 instantiation (the others share its resource class).
const void* stage_kernel_ptr(int mixed, int shape, int stage) {
#define AMR_KP(RT, TX, TY)                                                                          \
  (stage == 1 ? reinterpret_cast<const void*>(&stage_kernel<RT, TX, TY, 1, false, true>)            \
              : reinterpret_cast<const void*>(&stage_kernel<RT, TX, TY, 2, false, true>))
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
  if (a.fast) hipLaunchKernelGGL(cfl_kernel<true>, dim3(grid), dim3(NT), 0, s, a);
  else hipLaunchKernelGGL(cfl_kernel<false>, dim3(grid), dim3(NT), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_cfl_finalize(hipStream_t s, const unsigned long long* smax, int lmin, int lmax, int root,
                               double cfl, double* dt) {
  hipLaunchKernelGGL(cfl_finalize, dim3(1), dim3(64), 0, s, smax, lmin, lmax, root, cfl, dt);
  return hipGetLastError();
}
hipError_t launch_copy_ghosts(hipStream_t s, const CopyOp* ops, const Work& w, const PatchDev* p, double* A) {
  hipLaunchKernelGGL(copy_ghosts, dim3(w.nblk), dim3(NT), 0, s, ops, w, p, A);
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
