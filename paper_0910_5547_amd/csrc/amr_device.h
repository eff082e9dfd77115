// amr_device.h - device-side data structures and per-cell / per-face arithmetic
// of the MOL hydro update (Wang, Abel & Kaehler, Sec. 4), for gfx950.
//
// RT is the reconstruction type: double for the FP64 path, float for the mixed
// path (FP32 reconstruction and face flux).  The conserved->primitive
// conversion, the flux divergence and the RK combine are always double.  In
// the double instantiation every expression below performs the same IEEE
// operations in the same order as the plain definition of the scheme (the
// translation unit is built with -ffp-contract=off), so the FP64 path is
// reproducible operation by operation.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace amr {

constexpr int NVAR = 5;
constexpr int NT = 256;  // threads per workgroup of the stage kernel (4 wave64s)
constexpr int MAX_LEVELS = 32;

enum { BC_OUTFLOW = 0, BC_PERIODIC = 1, BC_REFLECT = 2, BC_EXTERNAL = 3 };
enum { FLUX_PAPER = 0, FLUX_HLL2 = 1 };

// One patch as the kernels see it (built on the host from amr_patch_desc).
struct PatchDev {
  int64_t off;   // element offset of variable 0
  int64_t S;     // element stride between variables (stored cells)
  int n[3];      // active cells
  int g[3];      // ghost layers (0 in absent dimensions)
  int s[3];      // stored cells = n + 2g
  int bc[6];     // faces -x,+x,-y,+y,-z,+z
  int level;
  int pad;
  double dx[3];  // cell widths at this level
};

// One unit of stage-kernel work: a TX x TY column block of one patch, marched
// over planes z0 <= z < z1.
struct Tile {
  int patch, x0, y0, z0, z1, pad0, pad1, pad2;
};

// Same-level ghost copy: dst ghost cells in box [lo, lo+sz) (dst active-relative
// coordinates) take the values of src cells at the same coordinates + sh.
struct CopyOp {
  int dst, src;
  int lo[3], sz[3], sh[3];
  int pad;
};

struct Consts {
  double gamma, gm1, theta, rho_floor, e_floor;
  int ndim, flux;
};

// ------------------------------------------------------------------ indexing
__device__ __forceinline__ int64_t cell_elem(const PatchDev& P, int i, int j, int k) {
  return P.off + ((int64_t)(k + P.g[2]) * P.s[1] + (j + P.g[1])) * P.s[0] + (i + P.g[0]);
}

// Boundary condition as an index map (Sec. 3 ghost zones): a coordinate outside
// [0, n) along one dimension is sent to the active cell whose value the ghost
// holds; EXTERNAL keeps it (stored ghost, filled beforehand).
__device__ __forceinline__ int map_index(int i, int n, int bclo, int bchi, bool& flip) {
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

// Conserved state of cell (i,j,k) (active-relative; at most one coordinate may be
// outside the active range - the MOL stencil is a cross, Sec. 4).
__device__ __forceinline__ void load_cons(const double* __restrict__ A, const PatchDev& P, int i, int j, int k,
                                          double u[NVAR]) {
  bool fx = false, fy = false, fz = false;
  const int ii = map_index(i, P.n[0], P.bc[0], P.bc[1], fx);
  const int jj = map_index(j, P.n[1], P.bc[2], P.bc[3], fy);
  const int kk = map_index(k, P.n[2], P.bc[4], P.bc[5], fz);
  const int64_t e = cell_elem(P, ii, jj, kk);
#pragma unroll
  for (int v = 0; v < NVAR; ++v) u[v] = A[e + v * P.S];
  if (fx) u[1] = -u[1];
  if (fy) u[2] = -u[2];
  if (fz) u[3] = -u[3];
}

// ------------------------------------------------------------------ physics
// Conserved -> primitive (rho, e, vx, vy, vz), in FP64 (Sec. 4: E = v^2/2 + e,
// p = (gamma-1) rho e; the kinetic-energy subtraction cancels at high Mach, so it
// is never done in FP32).  Returns true for an unphysical state.
template <typename RT>
__device__ __forceinline__ bool cons2prim(const double u[NVAR], const Consts& c, RT q[NVAR]) {
  const double rho = u[0];
  const double vx = u[1] / rho, vy = u[2] / rho, vz = u[3] / rho;
  const double kin = 0.5 * ((u[1] * u[1] + u[2] * u[2]) + u[3] * u[3]) / rho;
  double e = (u[4] - kin) / rho;
  bool bad = !(isfinite(u[0]) && isfinite(u[1]) && isfinite(u[2]) && isfinite(u[3]) && isfinite(u[4]));
  double r = rho;
  if (!(r > 0) && !(c.rho_floor > 0)) bad = true;
  if (!(e > 0) && !(c.e_floor > 0)) bad = true;
  if (c.rho_floor > 0 && r < c.rho_floor) r = c.rho_floor;
  if (c.e_floor > 0 && e < c.e_floor) e = c.e_floor;
  q[0] = (RT)r;
  q[1] = (RT)e;
  q[2] = (RT)vx;
  q[3] = (RT)vy;
  q[4] = (RT)vz;
  return bad;
}

// Largest signal speed of one cell, sum_d (|v_d| + c_s)/dx_d (the CFL rule).
__device__ __forceinline__ double cell_speed(const double u[NVAR], const Consts& c, const double dx[3], int& bad) {
  double q[NVAR];
  bad |= cons2prim<double>(u, c, q) ? 1 : 0;
  const double p = c.gm1 * q[0] * q[1];
  const double cs = sqrt(c.gamma * p / q[0]);
  double s = 0.0;
  s = s + (fabs(q[2]) + cs) / dx[0];
  if (c.ndim > 1) s = s + (fabs(q[3]) + cs) / dx[1];
  if (c.ndim > 2) s = s + (fabs(q[4]) + cs) / dx[2];
  return s;
}

// Three-argument minmod of Sec. 4:
//   0.25 (sgn a + sgn b) |sgn a + sgn c| min(|a|,|b|,|c|)
// = sgn(a) min(|a|,|b|,|c|) when a, b, c share a strict sign, else 0.
template <typename RT>
__device__ __forceinline__ RT minmod3(RT a, RT b, RT c) {
  const RT m = fmin(fabs(a), fmin(fabs(b), fabs(c)));
  const bool pos = (a > RT(0)) & (b > RT(0)) & (c > RT(0));
  const bool neg = (a < RT(0)) & (b < RT(0)) & (c < RT(0));
  return (pos | neg) ? copysign(m, a) : RT(0);
}

// PLM limited slope of the middle of three cells (Sec. 4 with theta):
//   sigma_i = minmod(theta (q_i - q_{i-1}), theta (q_{i+1} - q_i), (q_{i+1} - q_{i-1})/2);
// face states are q_{i-1} + sigma_{i-1}/2 (left) and q_i - sigma_i/2 (right).
template <typename RT>
__device__ __forceinline__ RT plm_slope(RT qm, RT q0, RT qp, RT theta) {
  return minmod3<RT>(theta * (q0 - qm), theta * (qp - q0), (qp - qm) / RT(2));
}

template <typename RT>
struct FaceConsts {
  RT gamma, gm1;
};

// Conserved state U(q), pressure and sound speed of one face state.
template <typename RT>
__device__ __forceinline__ void face_state(const RT q[NVAR], const FaceConsts<RT>& k, RT U[NVAR], RT& p, RT& c) {
  const RT rho = q[0], e = q[1], vx = q[2], vy = q[3], vz = q[4];
  p = k.gm1 * rho * e;
  c = sqrt(k.gamma * p / rho);
  U[0] = rho;
  U[1] = rho * vx;
  U[2] = rho * vy;
  U[3] = rho * vz;
  U[4] = rho * (e + RT(0.5) * ((vx * vx + vy * vy) + vz * vz));
}

// Riemann flux in direction D at a face with primitive states qL, qR (Sec. 4
// flux equation): lambda^+- = v_D +- c_s on each side, a+ = max(0, l+_L, l+_R),
// a- = max(0, -l-_L, -l-_R); the printed flux uses lambda0 = max(a+, a-).
// Physical flux F^D(U) = (rho v_D, rho v_D v + p e_D, (rho E + p) v_D).
template <typename RT, int D>
__device__ __forceinline__ void riemann_flux(const RT qL[NVAR], const RT qR[NVAR], const FaceConsts<RT>& k, int kind,
                                             RT F[NVAR]) {
  RT UL[NVAR], UR[NVAR], pL, pR, cL, cR;
  face_state<RT>(qL, k, UL, pL, cL);
  face_state<RT>(qR, k, UR, pR, cR);
  RT FL[NVAR], FR[NVAR];
  FL[0] = UL[1 + D];
  FR[0] = UR[1 + D];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    FL[1 + j] = (j == D) ? UL[1 + D] * qL[2 + j] + pL : UL[1 + D] * qL[2 + j];
    FR[1 + j] = (j == D) ? UR[1 + D] * qR[2 + j] + pR : UR[1 + D] * qR[2 + j];
  }
  const RT vL = qL[2 + D], vR = qR[2 + D];
  FL[4] = (UL[4] + pL) * vL;
  FR[4] = (UR[4] + pR) * vR;
  const RT ap = fmax(RT(0), fmax(vL + cL, vR + cR));
  const RT am = fmax(RT(0), fmax(-(vL - cL), -(vR - cR)));
  if (kind == FLUX_HLL2) {
    const RT apm = ap * am, den = ap + am;
#pragma unroll
    for (int v = 0; v < NVAR; ++v) F[v] = ((ap * FL[v] + am * FR[v]) - apm * (UR[v] - UL[v])) / den;
  } else {
    const RT lam = fmax(ap, am);
#pragma unroll
    for (int v = 0; v < NVAR; ++v) F[v] = RT(0.5) * ((FL[v] + FR[v]) - lam * (UR[v] - UL[v]));
  }
}

// Flux at the face between the 2nd and 3rd of four consecutive cells q0..q3
// along D: reconstruct both face states, then the Riemann flux.
template <typename RT, int D>
__device__ __forceinline__ void face_flux4(const RT q0[NVAR], const RT q1[NVAR], const RT q2[NVAR],
                                           const RT q3[NVAR], RT theta, const FaceConsts<RT>& k, int kind,
                                           RT F[NVAR]) {
  RT qL[NVAR], qR[NVAR];
#pragma unroll
  for (int v = 0; v < NVAR; ++v) {
    const RT s1 = plm_slope<RT>(q0[v], q1[v], q2[v], theta);
    const RT s2 = plm_slope<RT>(q1[v], q2[v], q3[v], theta);
    qL[v] = q1[v] + RT(0.5) * s1;
    qR[v] = q2[v] - RT(0.5) * s2;
  }
  riemann_flux<RT, D>(qL, qR, k, kind, F);
}

}  // namespace amr
