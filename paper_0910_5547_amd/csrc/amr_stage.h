// amr_stage.h - the gfx950 stage kernel of the per-patch MOL update
// (Wang, Abel & Kaehler, Secs. 4-5).
//
// Stage kernel.  One workgroup of 256 lanes owns a TX x TY block of cell
// columns of one patch and marches it through the planes z0..z1-1 of its tile:
//   * the z direction lives in registers: each lane keeps, for its own column,
//     the primitives of planes z and z+1, the limited z-slope of plane z and the
//     z-face flux F_{z-1/2}, and loads plane z+2 per step, so every cell of the
//     column is read from HBM once per stage (its conserved state waits in a
//     lane-private LDS ring, or in registers, until the update two planes later);
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
//     (2) and (3), overlapping with the other waves' face work.  On 32 x 16
//     tiles (one workgroup per CU, where every barrier drains the CU) and on the
//     FP32 patch-fit tiles (1) and (2) are one pass: the lane of a face forms both
//     its states from the primitive plane (the same slopes, evaluated once per
//     face side), and with the plane and the fluxes double-buffered one barrier
//     per plane remains;
//   * L(U) is accumulated in FP64 in the order x, y, z (MOL equation), and the
//     TVD-RK2 stage combine is applied in FP64 before one store per variable.
// Stage 2 writes U^{n+1} over U^n in place: U^n is only read at the cell being
// written.  Boundary conditions other than EXTERNAL are index maps applied at
// load time; EXTERNAL ghosts are read from storage (filled by copy_ghosts) or,
// on a direct sibling face of a single-level table, from the sibling's cells.
//
// The same source serves the plain form (one launch per patch, one tile per
// workgroup) and the batched form (one persistent launch over the tile list of
// all patches, workgroups striding through it).
//
// Included by the translation units that instantiate it (one per variable count and,
// for hydro, per reconstruction precision), which compile in parallel.
#pragma once
#include "amr_device.h"
#include "amr_internal.h"

namespace amr {

// A struct that the kernel only reads, at an address uniform across the wavefront:
// read word by word through the constant address space, which the compiler turns into
// scalar loads into scalar registers (a plain read would be a vector load holding the
// struct in every lane's registers).
template <typename S>
__device__ __forceinline__ S load_uniform(const S* p) {
  static_assert(sizeof(S) % 4 == 0 && alignof(S) >= 4, "whole words");
  typedef const __attribute__((address_space(4))) int ConstWord;
  const ConstWord* w = (const ConstWord*)p;
  S r;
  int* d = reinterpret_cast<int*>(&r);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(S) / 4); ++i) d[i] = w[i];
  return r;
}

// Occupancy target: three 256-lane workgroups per CU for the FP32-reconstruction
// instantiations (<= 168 VGPRs), two for FP64 (LDS-bound at two per CU anyway).
// REC: record fine-face fluxes into the refluxing registers (patches of levels > 0).
// TH1: the default scheme - limiter parameter 1 (the two-argument minmod, see
// plm_slope_t) and e reconstructed - known at compile time; the other instantiation
// takes theta and the reconstructed variable at run time.
// A tile of TX x TY = 256 columns is the whole workgroup's; a tile of 64 columns
// (small patches) is one wavefront's, each of the four wavefronts walking its own
// tiles and synchronising only with itself.
// NTH: threads per workgroup (256; 512 for the 32 x 16 tile, whose LDS allows one
// workgroup per CU; 384 for 32 x 12, two per CU).
// MHD (NV = 8, and 9 with the GLM field): two waves per SIMD in FP32; one in FP64, whose eight-variable LDS
// tiles leave one workgroup per CU, so the kernel may use the whole register file.
template <typename RT, int NV, int TX, int TY, int NTH, int STAGE, bool REC, bool TH1>
__global__ __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(
    NV >= NVAR_MHD ? (Fast<RT>::value ? 2 : 1) : (Fast<RT>::value && !REC && NTH != 512 ? 3 : 2))))
void stage_kernel(StageArgs a) {
  // TX = TY = 0: patch-fit tiles of 256 columns whose width tx (8, 16 or 32) each tile
  // carries (Tile::tx), its height 256 / tx; the LDS is sized for the largest plane
  constexpr bool VARW = TX == 0;
  static_assert(!VARW || NTH == NT, "patch-fit tiles are whole 256-lane workgroups");
  constexpr int TL = VARW ? NTH : TX * TY;  // lanes (columns) per tile
  static_assert(TL == NTH || TL == 64, "a tile is the workgroup or one wavefront");
  constexpr int WPB = NTH / TL;  // tiles in flight per workgroup
  constexpr bool FAST = Fast<RT>::value;
  constexpr bool HASY = VARW || TY > 1;  // 1D tiles carry no y rows
  constexpr int RO = HASY ? 2 : 0;       // row offset of tile row 0
  // LDS plane: (ty + 4) rows of tx + 4 cells (tx x ty = 8 x 32, 16 x 16 or 32 x 8 when VARW)
  constexpr int PLANE = VARW ? 36 * 12 : (HASY ? TY + 4 : 1) * (TX + 4);
  constexpr int HMAX = VARW ? (4 * 40 + TL - 1) / TL : HASY ? (4 * (TX + TY) + TL - 1) / TL : 1;  // halo cells per lane
  // face slots: x faces first, slot row*(nxT+1) + f, then y faces, slot nfx + f*nxT + col
  constexpr int NSLOT = VARW ? 32 * 9 + 33 * 8 : TY * (TX + 1) + (HASY ? (TY + 1) * TX : 0);
  // SB (512-lane tiles, one workgroup per CU: FP32 reconstruction, and FP64 hydro in
  // stage 1, its stage 2 being short of registers for it; FP32 hydro on patch-fit tiles,
  // three workgroups per CU with RREG): one workgroup barrier per plane instead of three.
  // Each lane forms both states of its low x and y faces from the primitive plane itself
  // (the limited slopes of the cells on either side), so no face states pass through LDS;
  // the primitive plane and the fluxes are double-buffered by plane parity, and plane
  // k+1's primitives go to LDS during plane k's face pass.
  // RREG: the conserved state of the lane's planes k and k+1 in registers (FP32
  // reconstruction): on patch-fit hydro tiles, so that the LDS holds two planes and their
  // fluxes and the single-barrier scheme keeps three workgroups per CU; on the 8- and
  // 9-variable 32 x 16 tiles and the wavefront tiles, instead of re-reading the cell from
  // global memory for the update.
  constexpr bool SB512 = WPB == 1 && NTH == 512 && (Fast<RT>::value || (NV == NVAR && STAGE == 1));
  constexpr bool RREG = FAST && ((VARW && NV == NVAR) || (SB512 && NV >= NVAR_MHD && !REC) || (WPB > 1 && NV == NVAR));
  constexpr bool SB = SB512 || (WPB == 1 && RREG);
  constexpr int PB = SB ? 2 : WPB;
  __shared__ RT sP[PB][NV][PLANE];  // primitives of the plane (+ face halo), rows of tx + 4
  // face states; sFL then holds the flux (SB: the flux only)
  __shared__ RT sFL[PB][NV][NSLOT], sFR[SB ? 1 : WPB][NV][SB ? 1 : NSLOT];
  // conserved state of this lane's cell in planes k and k+1 (3D), for the update:
  // lane-private, kept in LDS rather than registers or a second read (FP32 hydro on the
  // other workgroup tiles; RREG keeps it in registers; the FP64 kernels re-read the cell,
  // their LDS and register budgets being spent)
  constexpr bool RING = FAST && WPB == 1 && NV == NVAR && !RREG;
  __shared__ double sV[RING ? 2 : 1][NV][RING ? NTH : 1];

  Consts C = a.c;
  if constexpr (TH1) C.recon = RECON_E;  // (folds the reconstruction branches away)
  const FaceConsts<RT> K{(RT)C.gamma, (RT)C.gm1, (RT)C.gg1, C.recon, (RT)C.ch, (RT)C.ch2};
  const RT theta = (RT)C.theta;
  const int kind = C.flux;
  // this lane's tile slot in the workgroup: uniform across the wavefront (a tile is a
  // whole number of wavefronts), which readfirstlane tells the compiler, so that the
  // tile and its patch descriptor are scalar loads into scalar registers
  const int sub = WPB == 1 ? 0 : __builtin_amdgcn_readfirstlane((int)threadIdx.x / TL);
  const int tid = WPB == 1 ? (int)threadIdx.x : (int)threadIdx.x % TL;  // lane in the tile
  int cx = VARW ? 0 : tid % TX, cy = VARW ? 0 : tid / TX;
  auto tile_sync = [] {
    if constexpr (WPB == 1) {
      __syncthreads();
    } else {  // one wavefront: its LDS operations complete in order
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  };
  const double dt = *a.dt;
  int bad = 0;
  double smax = 0.0;
  const int buf = sub;

  for (int t = blockIdx.x * WPB + sub; t < a.ntiles; t += gridDim.x * WPB) {
    // (t is uniform across the wavefront; the tile list and the descriptors are read-only)
    const Tile T = load_uniform(a.tiles + t);
    const PatchDev P = load_uniform(a.patches + T.patch);
    const int tx = VARW ? T.tx : TX;        // tile width (a power of two when VARW)
    const int ty = VARW ? TL / tx : TY;
    const int pitch = tx + 4;                 // LDS row length of the plane
    if constexpr (VARW) {
      const int lg = __builtin_ctz(tx);
      cx = tid & (tx - 1);
      cy = tid >> lg;
    }
    const int nxT = min(tx, P.n[0] - T.x0);
    const int nyT = HASY ? min(ty, P.n[1] - T.y0) : 1;
    const bool act = cx < nxT && cy < nyT;
    const int i = T.x0 + cx, j = T.y0 + cy;
    const bool hasz = C.ndim == 3;
    const bool hasy = HASY && C.ndim >= 2;
    // Layouts: the stage input V (stage 1: the caller's U; stage 2: the scratch U^(1))
    // and the cell's own U^n and output (stage 1: U^(1); stage 2: U), each an element
    // offset, variable stride, row length, plane stride and ghost offsets.
    constexpr bool in_caller = STAGE == 1;
    const int64_t offV = in_caller ? P.off : P.off1, SV = in_caller ? P.S : P.S1;
    const int64_t offO = in_caller ? P.off1 : P.off, SO = in_caller ? P.S1 : P.S;
    const int rowV = in_caller ? P.s[0] : P.s1[0], rowO = in_caller ? P.s1[0] : P.s[0];
    const int gV0 = in_caller ? P.g[0] : P.g1[0], gV1 = in_caller ? P.g[1] : P.g1[1];
    const int gV2 = in_caller ? P.g[2] : P.g1[2];
    const int gO0 = in_caller ? P.g1[0] : P.g[0], gO1 = in_caller ? P.g1[1] : P.g[1];
    const int gO2 = in_caller ? P.g1[2] : P.g[2];
    // (constant indices only: a runtime index into P would move it to scratch memory)
#define NBO_V(f) (in_caller ? P.nbo[f] : P.nbo1[f])
    // element of this lane's column in plane 0 (the column is inside the patch) and
    // the stride between planes; plane k of the column is at col0 + kk * pstride,
    // kk being k after the z boundary map (uniform across the workgroup)
    const int64_t pstride = (int64_t)rowV * (in_caller ? P.s[1] : P.s1[1]);
    const int64_t pstrideO = (int64_t)rowO * (in_caller ? P.s1[1] : P.s[1]);
    // (inactive lanes of a ragged tile point at the tile's last active column, so that
    // every lane can issue the plane prefetch below unconditionally)
    const int ic = min(i, P.n[0] - 1), jc = min(j, P.n[1] - 1);
    const int64_t col0 = offV + (int64_t)gV2 * pstride + (int64_t)(jc + gV1) * rowV + (ic + gV0);
    const int64_t colO = offO + (int64_t)gO2 * pstrideO + (int64_t)(jc + gO1) * rowO + (ic + gO0);
    // The REFLECT sign flip of the normal momentum is applied where loaded values
    // are used, not at the load: a flip right after the load would make the load
    // wait for its data, and the prefetches below would stop hiding latency.
    // (a plane beyond a direct sibling face is read in the sibling: uniform branches)
    auto load_col_raw = [&](int kz, double u[NV]) -> bool {  // true: reflect in z
      bool fz = false;
      const int kk = map_index(kz, P.n[2], P.bc[4], P.bc[5], fz);
      int64_t e = col0 + (int64_t)kk * pstride;
      if (kz < 0 && (P.dmask & 16)) e += NBO_V(4);
      if (kz >= P.n[2] && (P.dmask & 32)) e += NBO_V(5);
#pragma unroll
      for (int v = 0; v < NV; ++v) u[v] = a.V[e + v * SV];
      return fz;
    };
    auto load_col = [&](int kz, double u[NV]) {
      if (load_col_raw(kz, u)) reflect_flip<NV>(u, 2);
    };

    // z-direction register queue (3D only): primitives of planes k and k+1, the
    // z-slope of plane k and the flux F_{k-1/2}
    RT qz[NV], qz1[NV], sgz[NV], Fzm[NV];
    double VcA[RREG ? NV : 1], VcB[RREG ? NV : 1];  // RREG: conserved state of planes k, k+1
    if (hasz) {
      double u[NV];
      RT qa[NV], qb[NV];
      load_col(T.z0 - 2, u);
      bad |= cons2prim<RT, NV>(u, C, qa);
      load_col(T.z0 - 1, u);
      bad |= cons2prim<RT, NV>(u, C, qb);
      load_col(T.z0, u);
      bad |= cons2prim<RT, NV>(u, C, qz);
      if constexpr (RING) {
#pragma unroll
        for (int v = 0; v < NV; ++v) sV[T.z0 & 1][v][threadIdx.x] = u[v];
      }
      if constexpr (RREG) {
#pragma unroll
        for (int v = 0; v < NV; ++v) VcA[v] = u[v];
      }
      load_col(T.z0 + 1, u);
      bad |= cons2prim<RT, NV>(u, C, qz1);
      if constexpr (RING) {
#pragma unroll
        for (int v = 0; v < NV; ++v) sV[(T.z0 + 1) & 1][v][threadIdx.x] = u[v];
      }
      if constexpr (RREG) {
#pragma unroll
        for (int v = 0; v < NV; ++v) VcB[v] = u[v];
      }
      RT qL[NV], qR[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const RT sa = plm_slope_t<RT, TH1>(qa[v], qb[v], qz[v], theta);
        sgz[v] = plm_slope_t<RT, TH1>(qb[v], qz[v], qz1[v], theta);
        qL[v] = madd(RT(0.5), sa, qb[v]);
        qR[v] = madd(RT(-0.5), sgz[v], qz[v]);
      }
      riemann_flux<RT, 2, NV>(qL, qR, K, kind, Fzm);
    }
    // fine-face flux registers (Berger-Colella refluxing): faces on this patch's
    // boundary whose flux the coarse level must later see, dt/2 per stage
    // (recorded in the update below, from the fluxes it reads anyway)
    const double hdt = 0.5 * dt;
    const bool rec = REC && P.level > 0;

    // Face halo of every plane: x halo = cols -2,-1,nxT,nxT+1 of every row, y halo =
    // rows -2,-1,nyT,nyT+1 of every column.  Lane tid owns halo cells tid + s*TL; their
    // conserved states are loaded one plane ahead so the loads' latency overlaps a
    // whole plane of work.
    const int nhx = 4 * nyT, nhy = hasy ? 4 * nxT : 0;
    int hrow[HMAX], hcol[HMAX], hflip[HMAX];
    int64_t hbase[HMAX];  // element of the halo cell's source in plane 0 (boundary maps applied)
    double Hn[HMAX][NV];
    auto load_halo = [&](int s, int kz, double u[NV]) {  // raw: hflip applied at use
      const int64_t e = hbase[s] + (int64_t)kz * pstride;
#pragma unroll
      for (int v = 0; v < NV; ++v) u[v] = a.V[e + v * SV];
    };
#pragma unroll
    for (int s = 0; s < HMAX; ++s) {
      const int h = tid + s * TL;
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
      const int iraw = T.x0 + hcol[s], jraw = T.y0 + hrow[s];
      const int ii = map_index(iraw, P.n[0], P.bc[0], P.bc[1], fx);
      const int jj = map_index(jraw, P.n[1], P.bc[2], P.bc[3], fy);
      hflip[s] = fx ? 1 : (fy ? 2 : 0);
      hbase[s] = offV + (int64_t)gV2 * pstride + (int64_t)(jj + gV1) * rowV + (ii + gV0);
      // a halo cell has at most one coordinate outside the patch (cross stencil)
      const int hf = iraw < 0 ? 0 : iraw >= P.n[0] ? 1 : jraw < 0 ? 2 : jraw >= P.n[1] ? 3 : -1;
      if (hf == 0 && (P.dmask & 1)) hbase[s] += NBO_V(0);
      if (hf == 1 && (P.dmask & 2)) hbase[s] += NBO_V(1);
      if (hf == 2 && (P.dmask & 4)) hbase[s] += NBO_V(2);
      if (hf == 3 && (P.dmask & 8)) hbase[s] += NBO_V(3);
      if (h < nhx + nhy) load_halo(s, T.z0, Hn[s]);
    }
    // Per-lane work of the slope and face passes, fixed for the tile:
    //  * the lane's own cell (active lanes): its x and y slopes, giving the right
    //    state of its low faces and the left state of its high faces, then the flux
    //    of its low x and low y faces;
    //  * one halo cell beside the tile (lanes < nhs): its slope across that side,
    //    giving the left state of the tile's first face or the right state of its
    //    last one;
    //  * one face on the tile's high x or high y edge (lanes < nfe).
    // Face slots: x faces row * (nxT + 1) + f, then y faces nfx + f * nxT + col.
    const int nfx = (nxT + 1) * nyT;
    const int pc_own = (cy + RO) * pitch + cx + 2;
    const int xs_own = cy * (nxT + 1) + cx, ys_own = nfx + cy * nxT + cx;
    const int nhs = 2 * nyT + (HASY ? 2 * nxT : 0);
    int pc_h = 0, st_h = 1, slot_h = 0;
    bool left_h = false;
    if (tid < nhs) {
      if (tid < 2 * nyT) {  // columns -1 and nxT
        const int row = tid >> 1, hi = tid & 1;
        pc_h = (row + RO) * pitch + (hi ? nxT : -1) + 2;
        slot_h = row * (nxT + 1) + (hi ? nxT : 0);
        left_h = !hi;
      } else {  // rows -1 and nyT
        const int q = tid - 2 * nyT, col = q >> 1, hi = q & 1;
        pc_h = ((hi ? nyT : -1) + RO) * pitch + col + 2;
        st_h = pitch;
        slot_h = nfx + (hi ? nyT : 0) * nxT + col;
        left_h = !hi;
      }
    }
    const int nfe = nyT + (HASY ? nxT : 0);
    int slot_e = 0, pc_e = 0, st_e = 1;  // (pc_e, st_e: the face's right cell in the plane, SB)
    bool ydir_e = false;
    if (tid < nfe) {
      if (tid < nyT) {
        slot_e = tid * (nxT + 1) + nxT;
        pc_e = (tid + RO) * pitch + nxT + 2;
      } else {
        slot_e = nfx + nyT * nxT + (tid - nyT);
        pc_e = (nyT + RO) * pitch + (tid - nyT) + 2;
        st_e = pitch;
        ydir_e = true;
      }
    }

    // halo of plane k (prefetched) into LDS, then prefetch the halo of plane k+1
    auto halo_to_lds = [&](int k, int pb) {
#pragma unroll
      for (int s = 0; s < HMAX; ++s) {
        if (tid + s * TL < nhx + nhy) {
          RT q[NV];
          if (hflip[s] == 1) reflect_flip<NV>(Hn[s], 0);
          if (hflip[s] == 2) reflect_flip<NV>(Hn[s], 1);
          bad |= cons2prim<RT, NV>(Hn[s], C, q);
#pragma unroll
          for (int v = 0; v < NV; ++v) sP[pb][v][(hrow[s] + RO) * pitch + hcol[s] + 2] = q[v];
          if (k + 1 < T.z1) load_halo(s, k + 1, Hn[s]);
        }
      }
    };
    auto own_to_lds = [&](const RT qc[NV], int pb) {
      if (act) {
#pragma unroll
        for (int v = 0; v < NV; ++v) sP[pb][v][(cy + RO) * pitch + cx + 2] = qc[v];
      }
    };
    if constexpr (SB) {  // plane z0 into LDS ahead of the plane loop
      halo_to_lds(T.z0, T.z0 & 1);
      if (hasz) {
        own_to_lds(qz, T.z0 & 1);
      } else {
        double u[NV];
        RT qc[NV];
        load_col(T.z0, u);
        bad |= cons2prim<RT, NV>(u, C, qc);
        if constexpr (RING) {
#pragma unroll
          for (int v = 0; v < NV; ++v) sV[T.z0 & 1][v][threadIdx.x] = u[v];
        }
        if constexpr (RREG) {
#pragma unroll
          for (int v = 0; v < NV; ++v) VcA[v] = u[v];
        }
        own_to_lds(qc, T.z0 & 1);
      }
      tile_sync();
    }

    for (int k = T.z0; k < T.z1; ++k) {
      const int fb = SB ? (k & 1) : buf;  // LDS buffer of this plane
      // this step's HBM read first: plane k+2 of the column in 3D (consumed by the z
      // flux after the x-y work), plane k itself in 1D/2D.  Issued by every lane
      // without a branch, so that nothing between here and the use waits for it.
      double Vn2[NV];
      const bool fz2 = load_col_raw(hasz ? k + 2 : k, Vn2);
      if constexpr (!SB) {
        halo_to_lds(k, buf);
        // (every lane computes; inactive lanes of ragged tiles hold a copy of an active
        // column and only skip the shared and global writes: a branch around loads or
        // their uses would leave loads pending on one path, and the next iteration would
        // wait for all memory at its first prefetch)
        RT qc[NV];
        if (hasz) {
#pragma unroll
          for (int v = 0; v < NV; ++v) qc[v] = qz[v];
        } else {
          // (the empty asm keeps this use inside the 1D/2D branch: hoisted above it, the
          // conversion would make 3D wait here for its plane k+2 prefetch)
#pragma unroll
          for (int v = 0; v < NV; ++v) asm volatile("" : "+v"(Vn2[v]));
          if (fz2) reflect_flip<NV>(Vn2, 2);
          bad |= cons2prim<RT, NV>(Vn2, C, qc);
          if constexpr (RING) {
#pragma unroll
            for (int v = 0; v < NV; ++v) sV[k & 1][v][threadIdx.x] = Vn2[v];
          }
          if constexpr (RREG) {
#pragma unroll
            for (int v = 0; v < NV; ++v) VcA[v] = Vn2[v];
          }
        }
        own_to_lds(qc, buf);
        tile_sync();  // (A) plane primitives ready; previous plane's fluxes consumed
      }

      // the stage input of this cell (from the lane's LDS ring, else re-read) and, in
      // stage 2, U^n: the global loads are issued before the face pass so that it
      // hides their latency (wavefront tiles, short of VGPRs, issue them after it)
      double Vc[NV], U0c[NV];
      const int64_t ecell = col0 + (int64_t)k * pstride;    // the cell in V
      const int64_t ecellO = colO + (int64_t)k * pstrideO;  // the cell in U^n and the output
      auto load_u0 = [&] {
        if (STAGE == 2) {
#pragma unroll
          for (int v = 0; v < NV; ++v) U0c[v] = a.U0[ecellO + v * SO];
        }
      };
      auto load_vc = [&] {
        if constexpr (RING) {
#pragma unroll
          for (int v = 0; v < NV; ++v) Vc[v] = sV[k & 1][v][threadIdx.x];
        } else if constexpr (RREG) {
#pragma unroll
          for (int v = 0; v < NV; ++v) Vc[v] = VcA[v];
        } else {
#pragma unroll
          for (int v = 0; v < NV; ++v) Vc[v] = a.V[ecell + v * SV];
        }
      };
      if constexpr (!SB) {
        // (1) slopes, once per cell, as face states
        if (act) {
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const RT* pl = &sP[fb][v][0];
            const RT q0 = pl[pc_own];
            const RT sx = plm_slope_t<RT, TH1>(pl[pc_own - 1], q0, pl[pc_own + 1], theta);
            sFR[fb][v][xs_own] = madd(RT(-0.5), sx, q0);     // right state of its low x face
            sFL[fb][v][xs_own + 1] = madd(RT(0.5), sx, q0);  // left state of its high x face
            if constexpr (HASY) {
              const RT sy = plm_slope_t<RT, TH1>(pl[pc_own - pitch], q0, pl[pc_own + pitch], theta);
              sFR[fb][v][ys_own] = madd(RT(-0.5), sy, q0);
              sFL[fb][v][ys_own + nxT] = madd(RT(0.5), sy, q0);
            }
          }
        }
        if (tid < nhs) {
          RT* dst = left_h ? &sFL[fb][0][slot_h] : &sFR[fb][0][slot_h];
          const RT hs = left_h ? RT(0.5) : RT(-0.5);
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const RT* pl = &sP[fb][v][0];
            const RT q0 = pl[pc_h];
            const RT sg = plm_slope_t<RT, TH1>(pl[pc_h - st_h], q0, pl[pc_h + st_h], theta);
            dst[v * NSLOT] = madd(hs, sg, q0);
          }
        }
        tile_sync();  // (B) face states ready
      }

      if constexpr (WPB == 1) {
        load_u0();
        if constexpr (!RING && !RREG) load_vc();
      }

      if constexpr (SB) {
        // (1+2) each lane's low x and low y face, and one face of the tile's high x or y
        // edge: both states from the cells on either side (the same limited slopes of
        // the same primitives as the slope pass of the other tilings), then the flux
        auto face_states = [&](int pc, int st, RT qL[NV], RT qR[NV]) {
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const RT* pl = &sP[fb][v][0];
            const RT a0 = pl[pc - 2 * st], a1 = pl[pc - st], a2 = pl[pc], a3 = pl[pc + st];
            qL[v] = madd(RT(0.5), plm_slope_t<RT, TH1>(a0, a1, a2, theta), a1);
            qR[v] = madd(RT(-0.5), plm_slope_t<RT, TH1>(a1, a2, a3, theta), a2);
          }
        };
        if (act) {
          RT qL[NV], qR[NV], F[NV];
          face_states(pc_own, 1, qL, qR);
          riemann_flux<RT, 0, NV>(qL, qR, K, kind, F);
#pragma unroll
          for (int v = 0; v < NV; ++v) sFL[fb][v][xs_own] = F[v];
          if constexpr (HASY) {
            face_states(pc_own, pitch, qL, qR);
            riemann_flux_xy<RT, NV>(qL, qR, true, K, kind, F);
#pragma unroll
            for (int v = 0; v < NV; ++v) sFL[fb][v][ys_own] = F[v];
          }
        }
        if (tid < nfe) {
          RT qL[NV], qR[NV], F[NV];
          face_states(pc_e, st_e, qL, qR);
          riemann_flux_xy<RT, NV>(qL, qR, ydir_e, K, kind, F);
#pragma unroll
          for (int v = 0; v < NV; ++v) sFL[fb][v][slot_e] = F[v];
        }
      } else {
        // (2) every x- and y-face flux of the block, once, written over its left state
        auto face_at = [&](int slot, RT qL[NV], RT qR[NV]) {
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            qL[v] = sFL[fb][v][slot];
            qR[v] = sFR[fb][v][slot];
          }
        };
        if (act) {
          RT qL[NV], qR[NV], F[NV];
          face_at(xs_own, qL, qR);
          riemann_flux<RT, 0, NV>(qL, qR, K, kind, F);
#pragma unroll
          for (int v = 0; v < NV; ++v) sFL[fb][v][xs_own] = F[v];
          if constexpr (HASY) {
            face_at(ys_own, qL, qR);
            // (the x-frame evaluation, as for every y face: riemann_flux<RT, 1> sums the
            // kinetic energy in another order, and in the mixed path its FP32 rounding
            // would differ from the coarse level's recomputed flux in refluxing)
            riemann_flux_xy<RT, NV>(qL, qR, true, K, kind, F);
#pragma unroll
            for (int v = 0; v < NV; ++v) sFL[fb][v][ys_own] = F[v];
          }
        }
        if (tid < nfe) {
          RT qL[NV], qR[NV], F[NV];
          face_at(slot_e, qL, qR);
          riemann_flux_xy<RT, NV>(qL, qR, ydir_e, K, kind, F);
#pragma unroll
          for (int v = 0; v < NV; ++v) sFL[fb][v][slot_e] = F[v];
        }
      }
      // z-face flux F_{k+1/2} of this column from the register queue
      RT Fzp[NV], qn2[NV], sg1[NV];
      if (hasz) {
        RT qL[NV], qR[NV];
        if (fz2) reflect_flip<NV>(Vn2, 2);
        bad |= cons2prim<RT, NV>(Vn2, C, qn2);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          sg1[v] = plm_slope_t<RT, TH1>(qz[v], qz1[v], qn2[v], theta);
          qL[v] = madd(RT(0.5), sgz[v], qz[v]);
          qR[v] = madd(RT(-0.5), sg1[v], qz1[v]);
        }
        riemann_flux<RT, 2, NV>(qL, qR, K, kind, Fzp);
      }
      // (a use of the prefetch on every path, before the next memory operation: 3D has
      // just waited for it, and 1D/2D in the one-barrier scheme does not read it at all.
      // Left pending on any path, it would be waited for where the loop's end moves it
      // between registers - after this plane's stores, which the same counter tracks.
      // On the three-barrier tilings the wait lands here and also takes the halo loads
      // issued at the start of the plane, which have had the face pass to arrive)
#pragma unroll
      for (int v = 0; v < NV; ++v) asm volatile("" ::"v"(Vn2[v]));
      if constexpr (SB) {  // plane k+1 into the other buffer (3D: 1D/2D tiles have one plane)
        if (k + 1 < T.z1) {
          halo_to_lds(k + 1, (k + 1) & 1);
          own_to_lds(qz1, (k + 1) & 1);
        }
      }
      tile_sync();  // (C) fluxes ready (SB: and the next plane's primitives)
      if constexpr (WPB > 1) {
        load_u0();
        load_vc();
      } else if constexpr (RING || RREG) {
        load_vc();
      }

      // (3) L(U) in the order x, y, z, then the TVD-RK2 stage combine; fluxes of
      // this cell's faces on a coarse/fine boundary of the patch also go to the
      // refluxing registers (+= dt/2 F, Berger-Colella)
      {
        double L[NV];
        const int sx = xs_own, sy = ys_own;
        // at most one x, one y and one z face of this cell lies on a recorded patch
        // face (patches of a refined level are at least 2 cells wide); register
        // elements [v][k][j] (x faces), [v][k][i] (y faces), [v][j][i] (z faces)
        // (constant indices into P: a runtime index would move P to scratch memory)
        int64_t rx = -1, ry = -1, rz = -1;
        if (REC && rec && act) {
          rx = i == 0 ? P.reg[0] : (i == P.n[0] - 1 ? P.reg[1] : -1);
          if (hasy) ry = j == 0 ? P.reg[2] : (j == P.n[1] - 1 ? P.reg[3] : -1);
          if (hasz) rz = k == 0 ? P.reg[4] : (k == P.n[2] - 1 ? P.reg[5] : -1);
        }
        // (a no-return atomic add: one lane writes each register element per launch, so
        // the sum is taken in the same order as a load, add and store, but no load waits -
        // a load here would make the wave wait for every prefetch in flight.  The registers
        // are device memory of the table's own allocation; the hardware FP64 add rounds to
        // nearest like the ALU's, and the hierarchy tests compare the results bit for bit)
        auto record = [&](int64_t e, double F) { (void)unsafeAtomicAdd(a.reg + e, hdt * F); };
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const double fl = (double)sFL[fb][v][sx], fh = (double)sFL[fb][v][sx + 1];
          const double d = fh - fl;
          if constexpr (FAST) L[v] = -d * P.rdx[0];
          else L[v] = 0.0 - d / P.dx[0];
          if (REC && rx >= 0) record(rx + ((int64_t)v * P.n[2] + k) * P.n[1] + j, i == 0 ? fl : fh);
        }
        if (hasy) {
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const double fl = (double)sFL[fb][v][sy], fh = (double)sFL[fb][v][sy + nxT];
            const double d = fh - fl;
            if constexpr (FAST) L[v] = fma(-d, P.rdx[1], L[v]);
            else L[v] = L[v] - d / P.dx[1];
            if (REC && ry >= 0) record(ry + ((int64_t)v * P.n[2] + k) * P.n[0] + i, j == 0 ? fl : fh);
          }
        }
        if (hasz) {
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            if (REC && rz >= 0) record(rz + ((int64_t)v * P.n[1] + j) * P.n[0] + i, (double)(k == 0 ? Fzm[v] : Fzp[v]));
            const double d = (double)Fzp[v] - (double)Fzm[v];
            if constexpr (FAST) L[v] = fma(-d, P.rdx[2], L[v]);
            else L[v] = L[v] - d / P.dx[2];
            if constexpr (RING) sV[k & 1][v][threadIdx.x] = Vn2[v];  // plane k+2 takes plane k's slot
            if constexpr (RREG) {
              VcA[v] = VcB[v];
              VcB[v] = Vn2[v];
            }
            qz[v] = qz1[v];
            qz1[v] = qn2[v];
            sgz[v] = sg1[v];
            Fzm[v] = Fzp[v];
          }
        }
        // TVD-RK2 (Sec. 4): stage 1 U1 = U + dt L(U); stage 2 U^{n+1} = U^n/2 + (U1 + dt L(U1))/2
        const int64_t e = ecellO;
        double un[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          double u1;
          if constexpr (FAST) u1 = fma(dt, L[v], Vc[v]);
          else u1 = Vc[v] + dt * L[v];
          un[v] = (STAGE == 1) ? u1 : 0.5 * U0c[v] + 0.5 * u1;
        }
        if (act) {
#pragma unroll
          for (int v = 0; v < NV; ++v) a.out[e + v * SO] = un[v];
          if (STAGE == 2 && a.smax != nullptr) smax = fmax(smax, cell_speed<FAST, NV>(un, C, P, bad));
        }
        if constexpr (STAGE == 2) {
          // (U^n used on every path: consumed only where a lane is active, its loads stay
          // pending on a path of idle lanes, and the next plane's first reuse of their
          // registers waited for them and for every memory operation issued after them,
          // this plane's stores included.  This use moves that wait here, after the
          // stores, which measured faster on the patch-fit tiles)
#pragma unroll
          for (int v = 0; v < NV; ++v) asm volatile("" ::"v"(U0c[v]));
        }
      }
    }
    if (STAGE == 2 && a.smax != nullptr) {  // fused next-dt reduction, per level
      if constexpr (WPB == 1) block_max_to(a.smax + P.level, smax);
      else wave_max_to(a.smax + P.level, smax);
      smax = 0.0;
    }
  }
  if (bad) atomicOr(a.flag, 1);
#undef NBO_V
}

// ------------------------------------------------------------------ launchers
// One (precision, variables, tile) instantiation: the recording variant where the
// table has refluxing registers, the theta = 1 / e-reconstruction variant where the
// scheme allows it.
template <typename RT, int NV, int TX, int TY, int NTH, int STAGE>
inline hipError_t launch_stage_t(dim3 grid, hipStream_t s, const StageArgs& a) {
  const bool th1 = a.c.theta == 1.0 && a.c.recon == RECON_E;
  if (a.reg) {
    if (th1) hipLaunchKernelGGL((stage_kernel<RT, NV, TX, TY, NTH, STAGE, true, true>), grid, dim3(NTH), 0, s, a);
    else hipLaunchKernelGGL((stage_kernel<RT, NV, TX, TY, NTH, STAGE, true, false>), grid, dim3(NTH), 0, s, a);
  } else {
    if (th1) hipLaunchKernelGGL((stage_kernel<RT, NV, TX, TY, NTH, STAGE, false, true>), grid, dim3(NTH), 0, s, a);
    else hipLaunchKernelGGL((stage_kernel<RT, NV, TX, TY, NTH, STAGE, false, false>), grid, dim3(NTH), 0, s, a);
  }
  return hipGetLastError();
}

template <typename RT, int NV, int TX, int TY, int NTH = NT>
inline hipError_t launch_stage_s(int stage, dim3 grid, hipStream_t s, const StageArgs& a) {
  return stage == 1 ? launch_stage_t<RT, NV, TX, TY, NTH, 1>(grid, s, a)
                    : launch_stage_t<RT, NV, TX, TY, NTH, 2>(grid, s, a);
}

// The theta = 1 instantiation with or without register recording (the theta
// instantiations share a resource class), for occupancy queries.
template <typename RT, int NV, int TX, int TY, int NTH = NT>
inline const void* stage_kernel_ptr_s(int stage, bool rec) {
  if (stage == 1)
    return rec ? reinterpret_cast<const void*>(&stage_kernel<RT, NV, TX, TY, NTH, 1, true, true>)
               : reinterpret_cast<const void*>(&stage_kernel<RT, NV, TX, TY, NTH, 1, false, true>);
  return rec ? reinterpret_cast<const void*>(&stage_kernel<RT, NV, TX, TY, NTH, 2, true, true>)
             : reinterpret_cast<const void*>(&stage_kernel<RT, NV, TX, TY, NTH, 2, false, true>);
}

// MHD and GLM (NV = 8, 9): the shapes whose LDS fits (mhd_shape_ok); another
// combination returns hipErrorInvalidValue / nullptr.
template <typename RT, int NV>
inline hipError_t launch_stage_mhd_rt(int shape, int stage, dim3 grid, hipStream_t s, const StageArgs& a) {
  switch (shape) {
    case 0: return launch_stage_s<RT, NV, 256, 1>(stage, grid, s, a);
    case 1: return launch_stage_s<RT, NV, 32, 8>(stage, grid, s, a);
    case 4: return launch_stage_s<RT, NV, 8, 8>(stage, grid, s, a);
    case SHAPE_FIT: return launch_stage_s<RT, NV, 0, 0>(stage, grid, s, a);
    case 5:
      if constexpr (Fast<RT>::value) return launch_stage_s<RT, NV, 32, 16, 512>(stage, grid, s, a);
      else return hipErrorInvalidValue;
    case 6:
      if constexpr (Fast<RT>::value) return launch_stage_s<RT, NV, 32, 12, 384>(stage, grid, s, a);
      else return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

template <int NV>
inline hipError_t launch_stage_mhd_t(int mixed, int shape, int stage, int grid, hipStream_t s, const StageArgs& a) {
  if (!mhd_shape_ok(mixed, shape)) return hipErrorInvalidValue;
  if (mixed) return launch_stage_mhd_rt<float, NV>(shape, stage, dim3(grid), s, a);
  return launch_stage_mhd_rt<double, NV>(shape, stage, dim3(grid), s, a);
}

template <int NV>
inline const void* stage_kernel_ptr_mhd_t(int mixed, int shape, int stage, bool rec) {
  if (!mhd_shape_ok(mixed, shape)) return nullptr;
  if (mixed) {
    switch (shape) {
      case 0: return stage_kernel_ptr_s<float, NV, 256, 1>(stage, rec);
      case 1: return stage_kernel_ptr_s<float, NV, 32, 8>(stage, rec);
      case 4: return stage_kernel_ptr_s<float, NV, 8, 8>(stage, rec);
      case SHAPE_FIT: return stage_kernel_ptr_s<float, NV, 0, 0>(stage, rec);
      case 5: return stage_kernel_ptr_s<float, NV, 32, 16, 512>(stage, rec);
      case 6: return stage_kernel_ptr_s<float, NV, 32, 12, 384>(stage, rec);
    }
  } else {
    switch (shape) {
      case 0: return stage_kernel_ptr_s<double, NV, 256, 1>(stage, rec);
      case 1: return stage_kernel_ptr_s<double, NV, 32, 8>(stage, rec);
      case 4: return stage_kernel_ptr_s<double, NV, 8, 8>(stage, rec);
      case SHAPE_FIT: return stage_kernel_ptr_s<double, NV, 0, 0>(stage, rec);
    }
  }
  return nullptr;
}

// Hydro (NV = 5): every shape.
template <typename RT>
inline hipError_t launch_stage_hydro_t(int shape, int stage, int grid, hipStream_t s, const StageArgs& a) {
  switch (shape) {
    case 0: return launch_stage_s<RT, NVAR, 256, 1>(stage, dim3(grid), s, a);
    case 1: return launch_stage_s<RT, NVAR, 32, 8>(stage, dim3(grid), s, a);
    case 2: return launch_stage_s<RT, NVAR, 64, 4>(stage, dim3(grid), s, a);
    case 3: return launch_stage_s<RT, NVAR, 16, 16>(stage, dim3(grid), s, a);
    case 4: return launch_stage_s<RT, NVAR, 8, 8>(stage, dim3(grid), s, a);
    case 5: return launch_stage_s<RT, NVAR, 32, 16, 512>(stage, dim3(grid), s, a);
    case 6: return launch_stage_s<RT, NVAR, 32, 12, 384>(stage, dim3(grid), s, a);
    case SHAPE_FIT: return launch_stage_s<RT, NVAR, 0, 0>(stage, dim3(grid), s, a);
    default: return hipErrorInvalidValue;
  }
}

template <typename RT>
inline const void* stage_kernel_ptr_hydro_t(int shape, int stage, bool rec) {
  switch (shape) {
    case 0: return stage_kernel_ptr_s<RT, NVAR, 256, 1>(stage, rec);
    case 1: return stage_kernel_ptr_s<RT, NVAR, 32, 8>(stage, rec);
    case 2: return stage_kernel_ptr_s<RT, NVAR, 64, 4>(stage, rec);
    case 3: return stage_kernel_ptr_s<RT, NVAR, 16, 16>(stage, rec);
    case 4: return stage_kernel_ptr_s<RT, NVAR, 8, 8>(stage, rec);
    case 5: return stage_kernel_ptr_s<RT, NVAR, 32, 16, 512>(stage, rec);
    case 6: return stage_kernel_ptr_s<RT, NVAR, 32, 12, 384>(stage, rec);
    case SHAPE_FIT: return stage_kernel_ptr_s<RT, NVAR, 0, 0>(stage, rec);
    default: return nullptr;
  }
}

}  // namespace amr
