// amr_device.h - device-side data structures and per-cell / per-face arithmetic
// of the MOL hydro update (Wang, Abel & Kaehler, Sec. 4), for gfx950, and of its
// ideal-MHD variant (the paper's MHD section with the cleaning field psi held at
// zero): NV = 5 conserved variables (rho, rho v, rho E) or NV = 8
// (rho, rho v, rho E + B^2/2, B), and of the GLM system with psi (NV = 9).
//
// RT is the reconstruction type: double for the FP64 path, float for the mixed
// path (FP32 reconstruction and face flux).  The conserved->primitive
// conversion, the flux divergence and the RK combine are always double.
//
// FP64 path: every expression performs the same IEEE operations in the same
// order as the plain definition of the scheme (the translation unit is built
// with -ffp-contract=off), so it reproduces a serial FP64 evaluation of the
// scheme bit for bit.
// Mixed path (Fast<float>): the same formulas evaluated for throughput -
// fused multiply-adds, one FP64 reciprocal of rho per conversion instead of
// five divisions, c_s = sqrt(gamma (gamma-1) e) (equal to sqrt(gamma p / rho)
// for the ideal gas) with the hardware square root, flux divergence as a
// multiply by 1/dx.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace amr {

constexpr int NVAR = 5;      // hydro
constexpr int NVAR_MHD = 8;  // ideal MHD
constexpr int NVAR_GLM = 9;  // GLM-MHD: the ideal-MHD set and the cleaning field psi
constexpr int NT = 256;  // threads per workgroup of the stage kernel (4 wave64s)
constexpr int MAX_LEVELS = 32;

enum { BC_OUTFLOW = 0, BC_PERIODIC = 1, BC_REFLECT = 2, BC_EXTERNAL = 3 };
enum { FLUX_PAPER = 0, FLUX_HLL2 = 1 };
enum { RECON_E = 0, RECON_P = 1 };

// One patch as the kernels see it (built on the host from amr_patch_desc).
struct PatchDev {
  int64_t off;   // element offset of variable 0
  int64_t S;     // element stride between variables (stored cells)
  int n[3];      // active cells
  int g[3];      // ghost layers (0 in absent dimensions)
  int s[3];      // stored cells = n + 2g
  int bc[6];     // faces -x,+x,-y,+y,-z,+z
  int level;
  int dmask;     // bit f: EXTERNAL face f reads its sibling's cells directly (nbo[f])
  double dx[3];  // cell widths at this level
  double rdx[3]; // 1/dx (mixed path)
  int64_t reg[6];  // fine-face flux register of each face (element offset), -1 = none
  // Direct sibling faces (single-level tables): the sibling has this patch's stored
  // shape, so the element of a ghost cell of face f in the sibling's storage is the
  // element of the same cell in this patch's ghost storage plus nbo[f].
  int64_t nbo[6];
  // Layout of the patch in the table's stage scratch U^(1): the caller's layout above,
  // or (tables whose patches need no stored ghosts) the active cells alone, s1 = n,
  // g1 = 0, at off1; nbo1 as nbo for that layout.
  int64_t off1, S1;
  int s1[3], g1[3];
  int64_t nbo1[6];
};

// One unit of stage-kernel work: a TX x TY column block of one patch, marched
// over planes z0 <= z < z1.
struct Tile {
  int patch, x0, y0, z0, z1, tx, pad1, pad2;  // tx: the tile's width (TX of its shape)
};

// Same-level ghost copy: dst ghost cells in box [lo, lo+sz) (dst active-relative
// coordinates) take the values of src cells at the same coordinates + sh.
struct CopyOp {
  int dst, src;
  int lo[3], sz[3], sh[3];
  int pad;
};

// Coarse -> fine ghost fill: dst ghost cells in box [lo, lo+sz) (dst-local) are
// prolonged from coarse patch src.  A dst-local cell x has fine level coordinate
// x + foff (foff = dst lo + periodic wrap, so it lies in the root domain), coarse
// level coordinate (x + foff) >> 1 and src-local coarse coordinate that minus clo.
struct ProlongOp {
  int dst, src;
  int lo[3], sz[3], foff[3], clo[3];
};

// Physical boundary ghosts written into storage: box [lo, lo+sz) of patch `patch`.
struct PhysOp {
  int patch, pad;
  int lo[3], sz[3];
};

// Refluxing of coarse cells [lo, lo+sz) (coarse-local) of patch `coarse` across
// the face (d, side) of fine patch `fine` (side 0: the fine patch's low face,
// which is the high face of these coarse cells).  The fine face cells under
// coarse cell x (coarse-local, other dimensions) start at fine-local 2 x + fo.
struct FixOp {
  int fine, coarse, d, side;
  int lo[3], sz[3], fo[3];
  int pad;
};

// Restriction of coarse cells [lo, lo+sz) (coarse-local) of `coarse` from `fine`:
// the children of coarse-local x start at fine-local 2 x + fo.
struct RestrictOp {
  int fine, coarse;
  int lo[3], sz[3], fo[3];
  int pad;
};

// Cell-granular distribution of a list of box ops over 256-lane workgroups: the
// cells of the ops, in list order, are numbered consecutively and workgroup b
// takes cells [256 b, 256 b + 256), one per lane, so small boxes share a
// workgroup instead of idling most of its lanes.  A segment is the part of one op
// that falls in one workgroup.
struct Seg {
  int op;     // index in the op list
  int cell0;  // the op's cell (x fastest in its box) held by lane `lane0`
  int lane0;
  int count;  // cells of the op in this workgroup
};
struct Work {
  const Seg* segs;  // segments of every work list of the table
  const int* blk;   // segments of workgroup b of this list: [blk[b], blk[b + 1])
  int nblk;
  int pad;
};

// Workgroup b of a launch runs on XCD b % 8; each XCD takes a contiguous run of the
// list instead (XCD x its q + (x < r) workgroups, q = n / 8, r = n % 8, from x q + min(x, r)
// on), so that neighbouring boxes' shared lines meet in one XCD's L2.  A bijection of [0, n).
__device__ __forceinline__ int xcd_run(int b, int n) {
  const int q = n >> 3, r = n & 7, x = b & 7;
  return x * q + min(x, r) + (b >> 3);
}

// The op index (or -1: no cell) and the cell within it of this lane.
__device__ __forceinline__ int work_item(const Work& w, int& cell) {
  int op = -1;
  cell = 0;
  const int lane = (int)threadIdx.x;
  const int b = xcd_run((int)blockIdx.x, w.nblk);
  for (int s = w.blk[b]; s < w.blk[b + 1]; ++s) {
    const Seg g = w.segs[s];
    const int c = lane - g.lane0;
    if (c >= 0 && c < g.count) {
      op = g.op;
      cell = g.cell0 + c;
    }
  }
  return op;
}

// Cell c (x fastest) of a box of sz cells -> its offsets b inside the box.
__device__ __forceinline__ void box_cell(const int sz[3], int c, int b[3]) {
  const int plane = sz[0] * sz[1];
  const int kk = c / plane, r = c - kk * plane;
  const int jj = r / sz[0];
  b[0] = r - jj * sz[0];
  b[1] = jj;
  b[2] = kk;
}

struct Consts {
  double gamma, gm1, gg1, theta, rho_floor, e_floor;  // gg1 = gamma (gamma - 1)
  double ch, ch2;  // GLM cleaning speed c_h and c_h^2 (NV = 9)
  int ndim, flux;
  int recon, pad;  // recon: RECON_E (slot 1 of the primitives holds e) or RECON_P (it holds p)
};

// Reconstruction-type traits: the mixed path is evaluated for speed.
template <typename RT>
struct Fast {
  static constexpr bool value = false;
};
template <>
struct Fast<float> {
  static constexpr bool value = true;
};

// a*b + c: two roundings in source order on the FP64 path, one fused op on the mixed path.
template <typename RT>
__device__ __forceinline__ RT madd(RT a, RT b, RT c) {
  if constexpr (Fast<RT>::value) return fmaf(a, b, c);
  else return a * b + c;
}

// ------------------------------------------------------------------ indexing
__device__ __forceinline__ int64_t cell_elem(const PatchDev& P, int i, int j, int k) {
  return P.off + ((int64_t)(k + P.g[2]) * P.s[1] + (j + P.g[1])) * P.s[0] + (i + P.g[0]);
}

// Boundary condition as an index map (Sec. 3 ghost zones): a coordinate outside
// [0, n) along one dimension is sent to the active cell whose value the ghost
// holds; EXTERNAL keeps it (stored ghost, filled beforehand).
__host__ __device__ __forceinline__ int map_index(int i, int n, int bclo, int bchi, bool& flip) {
  if (i < 0) {
    if (bclo == BC_OUTFLOW) return 0;
    if (bclo == BC_PERIODIC) return i + n;
    if (bclo == BC_REFLECT) { flip = true; return -1 - i; }
    return i;
  }
  if (i >= n) {
    if (bchi == BC_OUTFLOW) return n - 1;
    if (bchi == BC_PERIODIC) return i - n;
    if (bchi == BC_REFLECT) { flip = true; return 2 * n - 1 - i; }
    return i;
  }
  return i;
}

// A reflecting face negates the normal momentum (and, for MHD, the normal field).
template <int NV>
__device__ __forceinline__ void reflect_flip(double* u, int d) {
  u[1 + d] = -u[1 + d];
  if constexpr (NV >= NVAR_MHD) u[5 + d] = -u[5 + d];
}

// Conserved state of cell (i,j,k) (active-relative; at most one coordinate may be
// outside the active range - the MOL stencil is a cross, Sec. 4).
template <int NV = NVAR>
__device__ __forceinline__ void load_cons(const double* __restrict__ A, const PatchDev& P, int i, int j, int k,
                                          double u[NV]) {
  bool fx = false, fy = false, fz = false;
  const int ii = map_index(i, P.n[0], P.bc[0], P.bc[1], fx);
  const int jj = map_index(j, P.n[1], P.bc[2], P.bc[3], fy);
  const int kk = map_index(k, P.n[2], P.bc[4], P.bc[5], fz);
  const int64_t e = cell_elem(P, ii, jj, kk);
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = A[e + v * P.S];
  if (fx) reflect_flip<NV>(u, 0);
  if (fy) reflect_flip<NV>(u, 1);
  if (fz) reflect_flip<NV>(u, 2);
}

// ------------------------------------------------------------------ physics
// Conserved -> primitive (rho, e, vx, vy, vz[, Bx, By, Bz]), in FP64 (Sec. 4:
// E = v^2/2 + e, p = (gamma-1) rho e; for MHD the energy variable also holds
// B^2/2, subtracted as well; these subtractions cancel at high Mach or low beta,
// so they are never done in FP32).  Returns true for an unphysical state.
template <typename RT, int NV = NVAR>
__device__ __forceinline__ bool cons2prim(const double u[NV], const Consts& c, RT q[NV]) {
  constexpr bool MHD = NV >= NVAR_MHD;
  const double rho = u[0];
  double vx, vy, vz, e;
  if constexpr (Fast<RT>::value) {
    // 1/rho: hardware reciprocal estimate and two Newton steps (each squares the
    // relative error), in place of the correctly rounded division sequence
    double ri = __builtin_amdgcn_rcp(rho);
    ri = fma(ri, fma(-rho, ri, 1.0), ri);
    ri = fma(ri, fma(-rho, ri, 1.0), ri);
    vx = u[1] * ri;
    vy = u[2] * ri;
    vz = u[3] * ri;
    const double kin = 0.5 * fma(u[1], vx, fma(u[2], vy, u[3] * vz));
    if constexpr (MHD) {
      const double mag = 0.5 * fma(u[5], u[5], fma(u[6], u[6], u[7] * u[7]));
      e = ((u[4] - kin) - mag) * ri;
    } else {
      e = (u[4] - kin) * ri;
    }
  } else {
    vx = u[1] / rho;
    vy = u[2] / rho;
    vz = u[3] / rho;
    const double kin = 0.5 * ((u[1] * u[1] + u[2] * u[2]) + u[3] * u[3]) / rho;
    if constexpr (MHD) {
      const double mag = 0.5 * ((u[5] * u[5] + u[6] * u[6]) + u[7] * u[7]);
      e = ((u[4] - kin) - mag) / rho;
    } else {
      e = (u[4] - kin) / rho;
    }
  }
  bool bad = false;
#pragma unroll
  for (int v = 0; v < NV; ++v) bad |= !isfinite(u[v]);
  double r = rho;
  if (!(r > 0) && !(c.rho_floor > 0)) bad = true;
  if (!(e > 0) && !(c.e_floor > 0)) bad = true;
  if (c.rho_floor > 0 && r < c.rho_floor) r = c.rho_floor;
  if (c.e_floor > 0 && e < c.e_floor) e = c.e_floor;
  q[0] = (RT)r;
  q[1] = c.recon == RECON_P ? (RT)(c.gm1 * r * e) : (RT)e;
  q[2] = (RT)vx;
  q[3] = (RT)vy;
  q[4] = (RT)vz;
  if constexpr (MHD) {
    q[5] = (RT)u[5];
    q[6] = (RT)u[6];
    q[7] = (RT)u[7];
  }
  if constexpr (NV == NVAR_GLM) q[8] = (RT)u[8];
  return bad;
}

// Fast magnetosonic speed along D of a primitive MHD state, given a^2 = gamma p / rho:
//   c_f^2 = (a^2 + b^2 + sqrt((a^2 - b^2)^2 + 4 a^2 b_t^2)) / 2,
// b^2 = |B|^2 / rho, b_t^2 = (B_t1^2 + B_t2^2) / rho (t1, t2 = D+1, D+2 mod 3): the
// larger root of the fast/slow dispersion relation, its radicand written as a sum of
// non-negative terms (no cancellation where a = |B_D| / sqrt(rho)).
template <typename RT, int D>
__device__ __forceinline__ RT fast_speed(const RT* q, RT a2) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  if constexpr (Fast<RT>::value) {
    const RT ri = __builtin_amdgcn_rcpf(q[0]);
    const RT b2 = fmaf(q[5], q[5], fmaf(q[6], q[6], q[7] * q[7])) * ri;
    const RT bt2 = fmaf(q[5 + T1], q[5 + T1], q[5 + T2] * q[5 + T2]) * ri;
    const RT dab = a2 - b2;
    const RT r = fmaf(dab, dab, 4.0f * a2 * bt2);
    return __builtin_amdgcn_sqrtf(0.5f * ((a2 + b2) + __builtin_amdgcn_sqrtf(r)));
  } else {
    const RT b2 = ((q[5] * q[5] + q[6] * q[6]) + q[7] * q[7]) / q[0];
    const RT bt2 = (q[5 + T1] * q[5 + T1] + q[5 + T2] * q[5 + T2]) / q[0];
    const RT dab = a2 - b2;
    const RT r = dab * dab + RT(4) * a2 * bt2;
    return sqrt(RT(0.5) * ((a2 + b2) + sqrt(r)));
  }
}

// Largest signal speed of one cell, sum_d (|v_d| + c_d)/dx_d (the CFL rule), c_d the
// sound speed (hydro) or the fast magnetosonic speed along d (MHD).  FAST selects the
// mixed path's evaluation (used for tables of that precision, both by the CFL kernel
// and by the fused reduction in stage 2).
template <bool FAST, int NV = NVAR>
__device__ __forceinline__ double cell_speed(const double u[NV], const Consts& c, const PatchDev& P, int& bad) {
  constexpr bool MHD = NV >= NVAR_MHD;
  if constexpr (FAST) {
    float q[NV];
    bad |= cons2prim<float, NV>(u, c, q) ? 1 : 0;
    const float a2 = c.recon == RECON_P ? (float)c.gamma * q[1] * __builtin_amdgcn_rcpf(q[0]) : (float)c.gg1 * q[1];
    double cx, cy, cz;
    if constexpr (MHD) {
      cx = (double)fast_speed<float, 0>(q, a2);
      cy = c.ndim > 1 ? (double)fast_speed<float, 1>(q, a2) : 0.0;
      cz = c.ndim > 2 ? (double)fast_speed<float, 2>(q, a2) : 0.0;
    } else {
      cx = cy = cz = (double)__builtin_amdgcn_sqrtf(a2);
    }
    double sx = fabs((double)q[2]) + cx, sy = fabs((double)q[3]) + cy, sz = fabs((double)q[4]) + cz;
    if constexpr (NV == NVAR_GLM) {  // the cleaning waves travel at c_h
      sx = fmax(sx, c.ch);
      sy = fmax(sy, c.ch);
      sz = fmax(sz, c.ch);
    }
    double s = sx * P.rdx[0];
    if (c.ndim > 1) s = fma(sy, P.rdx[1], s);
    if (c.ndim > 2) s = fma(sz, P.rdx[2], s);
    return s;
  } else {
    double q[NV];
    bad |= cons2prim<double, NV>(u, c, q) ? 1 : 0;
    const double p = c.recon == RECON_P ? q[1] : c.gm1 * q[0] * q[1];
    const double a2 = c.gamma * p / q[0];
    double cx, cy, cz;
    if constexpr (MHD) {
      cx = fast_speed<double, 0>(q, a2);
      cy = c.ndim > 1 ? fast_speed<double, 1>(q, a2) : 0.0;
      cz = c.ndim > 2 ? fast_speed<double, 2>(q, a2) : 0.0;
    } else {
      cx = cy = cz = sqrt(a2);
    }
    double sx = fabs(q[2]) + cx, sy = fabs(q[3]) + cy, sz = fabs(q[4]) + cz;
    if constexpr (NV == NVAR_GLM) {
      sx = fmax(sx, c.ch);
      sy = fmax(sy, c.ch);
      sz = fmax(sz, c.ch);
    }
    double s = 0.0;
    s = s + sx / P.dx[0];
    if (c.ndim > 1) s = s + sy / P.dx[1];
    if (c.ndim > 2) s = s + sz / P.dx[2];
    return s;
  }
}

// Three-argument minmod of Sec. 4:
//   0.25 (sgn a + sgn b) |sgn a + sgn c| min(|a|,|b|,|c|)
// = sgn(a) max(0, min(|a|, sgn(a) b, sgn(a) c)): equal to the printed form for
// every input (up to the sign of a zero result).  FP32: the two-argument minmod is
// the median of (a, b, 0) - the smaller magnitude when a and b share a sign, else
// 0 - one v_med3_f32, and minmod(a, b, c) = minmod(minmod(a, b), c).  FP64 (no
// median instruction): sign-bit arithmetic, one min3 and one max.
__device__ __forceinline__ float minmod3(float a, float b, float c) {
  return __builtin_amdgcn_fmed3f(__builtin_amdgcn_fmed3f(a, b, 0.0f), c, 0.0f);
}
__device__ __forceinline__ double minmod3(double a, double b, double c) {
  const unsigned long long sa = (unsigned long long)__double_as_longlong(a) & 0x8000000000000000ull;
  const double bb = __longlong_as_double((long long)((unsigned long long)__double_as_longlong(b) ^ sa));
  const double cc = __longlong_as_double((long long)((unsigned long long)__double_as_longlong(c) ^ sa));
  const double m = fmax(fmin(fabs(a), fmin(bb, cc)), 0.0);
  return __longlong_as_double((long long)((unsigned long long)__double_as_longlong(m) | sa));
}

// Two-argument minmod, the limiter of the coarse -> fine prolongation slopes.
__device__ __forceinline__ double minmod2(double a, double b) {
  if (a > 0 && b > 0) return a < b ? a : b;
  if (a < 0 && b < 0) return a > b ? a : b;
  return 0.0;
}

// PLM limited slope of the middle of three cells (Sec. 4 with theta):
//   sigma_i = minmod(theta (q_i - q_{i-1}), theta (q_{i+1} - q_i), (q_{i+1} - q_{i-1})/2);
// face states are q_{i-1} + sigma_{i-1}/2 (left) and q_i - sigma_i/2 (right).
template <typename RT>
__device__ __forceinline__ RT plm_slope(RT qm, RT q0, RT qp, RT theta) {
  return minmod3(theta * (q0 - qm), theta * (qp - q0), (qp - qm) * RT(0.5));
}

// Two-argument minmod: FP32 the median of (a, b, 0); FP64 in the sign-bit form
// sgn(a) max(0, min(|a|, sgn(a) b)).
__device__ __forceinline__ float minmod_ab(float a, float b) { return __builtin_amdgcn_fmed3f(a, b, 0.0f); }
__device__ __forceinline__ double minmod_ab(double a, double b) {
  const unsigned long long sa = (unsigned long long)__double_as_longlong(a) & 0x8000000000000000ull;
  const double bb = __longlong_as_double((long long)((unsigned long long)__double_as_longlong(b) ^ sa));
  const double m = fmax(fmin(fabs(a), bb), 0.0);
  return __longlong_as_double((long long)((unsigned long long)__double_as_longlong(m) | sa));
}

// plm_slope with theta = 1 known at compile time (TH1).  The multiplications by
// theta are then exact, and when the one-sided differences a, b agree in sign the
// centred argument fl(fl(a + b)/2) is never below min(|a|, |b|) (rounding is
// monotone, halving exact), so the three-argument minmod returns the same value
// as the two-argument one, which skips the centred difference and a minmod per variable.
template <typename RT, bool TH1>
__device__ __forceinline__ RT plm_slope_t(RT qm, RT q0, RT qp, RT theta) {
  if constexpr (TH1) return minmod_ab(q0 - qm, qp - q0);
  else return plm_slope<RT>(qm, q0, qp, theta);
}

template <typename RT>
struct FaceConsts {
  RT gamma, gm1, gg1;
  int recon;
  RT ch, ch2;  // GLM cleaning speed and its square
};

// Specific internal energy e and pressure p of a face state whose slot 1 holds e
// (p = (gamma-1) rho e) or, with the pressure reconstruction, p (e = p / ((gamma-1) rho)).
template <typename RT>
__device__ __forceinline__ void face_eos(const RT* q, const FaceConsts<RT>& k, RT& e, RT& p) {
  if (k.recon == RECON_P) {
    p = q[1];
    if constexpr (Fast<RT>::value) e = q[1] * __builtin_amdgcn_rcpf(k.gm1 * q[0]);
    else e = q[1] / (k.gm1 * q[0]);
  } else {
    e = q[1];
    p = k.gm1 * q[0] * q[1];
  }
}

// Conserved state U(q), pressure and sound speed of one face state.
template <typename RT>
__device__ __forceinline__ void face_state(const RT q[NVAR], const FaceConsts<RT>& k, RT U[NVAR], RT& p, RT& c) {
  const RT rho = q[0], vx = q[2], vy = q[3], vz = q[4];
  RT e;
  face_eos<RT>(q, k, e, p);
  U[0] = rho;
  U[1] = rho * vx;
  U[2] = rho * vy;
  U[3] = rho * vz;
  if constexpr (Fast<RT>::value) {
    c = __builtin_amdgcn_sqrtf(k.gg1 * e);  // gamma p / rho = gamma (gamma-1) e
    U[4] = rho * fmaf(0.5f, fmaf(vx, vx, fmaf(vy, vy, vz * vz)), e);
  } else {
    c = sqrt(k.gamma * p / rho);
    U[4] = rho * (e + RT(0.5) * ((vx * vx + vy * vy) + vz * vz));
  }
}

// Physical flux F^D of one MHD face state (the paper's MHD flux vectors with psi = 0;
// the induction entries as in its x flux, v_D B_j - v_j B_D, which the y and z flux
// vectors equal up to the permutation of axes), its conserved state U and its fast
// magnetosonic speed c along D.  The FP64 path evaluates each entry in the order
//   momentum  (rho v_D v_j + [j = D] (p + B^2/2)) - B_j B_D
//   energy    ((rho E_h + p) v_D + B^2 v_D) - B_D (B . v)
// with rho E_h = rho (e + v^2/2) the gas part of the energy variable.  GLM (NV = 9):
// the B_D entry is psi and the psi entry c_h^2 B_D.
template <typename RT, int D, int NV>
__device__ __forceinline__ void mhd_face(const RT q[NV], const FaceConsts<RT>& k, RT U[NV], RT F[NV], RT& c) {
  const RT rho = q[0], vx = q[2], vy = q[3], vz = q[4], Bx = q[5], By = q[6], Bz = q[7];
  RT e, p;
  face_eos<RT>(q, k, e, p);
  const RT vd = q[2 + D], Bd = q[5 + D];
  U[0] = rho;
  U[1] = rho * vx;
  U[2] = rho * vy;
  U[3] = rho * vz;
  U[5] = Bx;
  U[6] = By;
  U[7] = Bz;
  F[0] = U[1 + D];
  F[5 + D] = RT(0);
  if constexpr (NV == NVAR_GLM) {
    U[8] = q[8];
    F[5 + D] = q[8];
    F[8] = k.ch2 * Bd;
  }
  if constexpr (Fast<RT>::value) {
    const RT a2 = k.gg1 * e;  // gamma p / rho
    c = fast_speed<RT, D>(q, a2);
    const RT B2 = fmaf(Bx, Bx, fmaf(By, By, Bz * Bz));
    const RT Bv = fmaf(Bx, vx, fmaf(By, vy, Bz * vz));
    const RT rEh = rho * fmaf(0.5f, fmaf(vx, vx, fmaf(vy, vy, vz * vz)), e);
    U[4] = fmaf(0.5f, B2, rEh);
#pragma unroll
    for (int j = 0; j < 3; ++j)
      F[1 + j] = fmaf(-q[5 + j], Bd, fmaf(U[1 + D], q[2 + j], j == D ? fmaf(0.5f, B2, p) : 0.0f));
    F[4] = fmaf(-Bd, Bv, ((rEh + p) + B2) * vd);
#pragma unroll
    for (int j = 0; j < 3; ++j)
      if (j != D) F[5 + j] = fmaf(vd, q[5 + j], -q[2 + j] * Bd);
  } else {
    const RT a2 = k.gamma * p / rho;
    c = fast_speed<RT, D>(q, a2);
    const RT B2 = (Bx * Bx + By * By) + Bz * Bz;
    const RT Bv = (Bx * vx + By * vy) + Bz * vz;
    const RT rEh = rho * (e + RT(0.5) * ((vx * vx + vy * vy) + vz * vz));
    U[4] = rEh + RT(0.5) * B2;
#pragma unroll
    for (int j = 0; j < 3; ++j)
      F[1 + j] = (U[1 + D] * q[2 + j] + (j == D ? p + RT(0.5) * B2 : RT(0))) - q[5 + j] * Bd;
    F[4] = ((rEh + p) * vd + B2 * vd) - Bd * Bv;
#pragma unroll
    for (int j = 0; j < 3; ++j)
      if (j != D) F[5 + j] = vd * q[5 + j] - q[2 + j] * Bd;
  }
}

// Riemann flux in direction D at a face with primitive states qL, qR (Sec. 4
// flux equation): lambda^+- = v_D +- c on each side (c the sound speed, or the
// fast magnetosonic speed along D for MHD), a+ = max(0, l+_L, l+_R),
// a- = max(0, -l-_L, -l-_R); the printed flux uses lambda0 = max(a+, a-).
// Hydro physical flux F^D(U) = (rho v_D, rho v_D v + p e_D, (rho E + p) v_D).
template <typename RT, int D, int NV = NVAR>
__device__ __forceinline__ void riemann_flux(const RT qL[NV], const RT qR[NV], const FaceConsts<RT>& k, int kind,
                                             RT F[NV]) {
  RT UL[NV], UR[NV], FL[NV], FR[NV], cL, cR;
  if constexpr (NV >= NVAR_MHD) {
    mhd_face<RT, D, NV>(qL, k, UL, FL, cL);
    mhd_face<RT, D, NV>(qR, k, UR, FR, cR);
  } else {
    RT pL, pR;
    face_state<RT>(qL, k, UL, pL, cL);
    face_state<RT>(qR, k, UR, pR, cR);
    FL[0] = UL[1 + D];
    FR[0] = UR[1 + D];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      FL[1 + j] = (j == D) ? UL[1 + D] * qL[2 + j] + pL : UL[1 + D] * qL[2 + j];
      FR[1 + j] = (j == D) ? UR[1 + D] * qR[2 + j] + pR : UR[1 + D] * qR[2 + j];
    }
    FL[4] = (UL[4] + pL) * qL[2 + D];
    FR[4] = (UR[4] + pR) * qR[2 + D];
  }
  const RT vL = qL[2 + D], vR = qR[2 + D];
  RT ap = fmax(RT(0), fmax(vL + cL, vR + cR));
  RT am = fmax(RT(0), fmax(-(vL - cL), -(vR - cR)));
  if constexpr (NV == NVAR_GLM) {  // the (B_D, psi) pair travels at -c_h and +c_h
    ap = fmax(ap, k.ch);
    am = fmax(am, k.ch);
  }
  if (kind == FLUX_HLL2) {
    const RT apm = ap * am, den = ap + am;
    if constexpr (Fast<RT>::value) {
      const RT rden = 1.0f / den;
#pragma unroll
      for (int v = 0; v < NV; ++v) F[v] = fmaf(-apm, UR[v] - UL[v], fmaf(ap, FL[v], am * FR[v])) * rden;
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) F[v] = ((ap * FL[v] + am * FR[v]) - apm * (UR[v] - UL[v])) / den;
    }
  } else {
    const RT lam = fmax(ap, am);
#pragma unroll
    for (int v = 0; v < NV; ++v) F[v] = RT(0.5) * madd(-lam, UR[v] - UL[v], FL[v] + FR[v]);
  }
}

// Riemann flux of a face whose normal is x (dir = 0) or y (dir = 1), the
// direction being a per-lane value: y faces are evaluated in the x frame with
// the x and y velocity (and field) components exchanged, then the two momentum
// (and induction) fluxes are exchanged back.  The arithmetic is that of
// riemann_flux<RT, dir>: every sum it reorders has two commuted operands.
template <typename RT, int NV = NVAR>
__device__ __forceinline__ void riemann_flux_xy(RT qL[NV], RT qR[NV], bool ydir, const FaceConsts<RT>& k,
                                                int kind, RT F[NV]) {
  auto swap = [](RT& a, RT& b) {
    const RT t = a;
    a = b;
    b = t;
  };
  if (ydir) {
    swap(qL[2], qL[3]);
    swap(qR[2], qR[3]);
    if constexpr (NV >= NVAR_MHD) {
      swap(qL[5], qL[6]);
      swap(qR[5], qR[6]);
    }
  }
  riemann_flux<RT, 0, NV>(qL, qR, k, kind, F);
  if (ydir) {
    swap(F[1], F[2]);
    if constexpr (NV >= NVAR_MHD) swap(F[5], F[6]);
  }
}

}  // namespace amr
