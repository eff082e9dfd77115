/* oracle.c - serial FP64 CPU oracle for the per-patch MOL hydro update of
 * Wang, Abel & Kaehler, "Adaptive Mesh Fluid Simulations on GPU" (Secs. 4-5).
 *
 * TEST INFRASTRUCTURE ONLY: the reference the GPU library is checked against.
 * Nothing on the product path links or calls it.  It is written as plain loops
 * that follow the paper's equations in the paper's order, one cell and one face
 * at a time, with no blocking, fusion or reuse beyond what the definitions say.
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math (no FMA contraction, so every
 * operation below is one IEEE-rounded operation in the order written).
 *
 * Readings of the paper taken here (the paper is silent or garbled):
 *  - PLM face states use half the limited slope (the printed formula omits the
 *    factor 1/2; without it a linear profile reconstructs the neighbour value).
 *  - The reconstructed primitives are (rho, e, vx, vy, vz), the set the paper's
 *    1D flux kernel stages; the face pressure is p = (gamma-1) rho e.  A flag
 *    reconstructs p instead of e (then e = p / ((gamma-1) rho) at the face).
 *  - The Riemann flux is the formula the paper prints in Sec. 4 (the symmetric
 *    one-speed form: F = (F_L + F_R - lambda0 (U_R - U_L))/2 with conserved
 *    U_R - U_L); the two-speed HLL of Harten, Lax & van Leer is a flag.
 *  - c_s = sqrt(gamma p / rho) at each face state; in a y or z sweep the normal
 *    velocity of that sweep replaces v_x in lambda^+-.  For MHD (nvar 8, psi held
 *    at 0) the fast magnetosonic speed along the sweep replaces c_s, B joins the
 *    reconstructed primitives, and reflect also negates the normal field.
 *  - Ghost layers are refilled before each RK stage; "outflow" is a zero-gradient
 *    copy of the edge cell's conserved variables; reflect mirrors and negates the
 *    normal momentum.
 *  - CFL rule (absent from the paper): dt = C / max_cells sum_d (|v_d|+c_d)/dx_d,
 *    c_d the signal speed above.
 */
#include "oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Threads the parallel regions below use: 1 in the serial build (the checker); the
 * OpenMP build of the same source, used only to time the oracle on all host cores,
 * reports its team size. */
#ifdef _OPENMP
#include <omp.h>
int or_threads(void) { return omp_get_max_threads(); }
#else
int or_threads(void) { return 1; }
#endif

/* ---------------------------------------------------------------- geometry */
typedef struct {
  int level, n[3], g[3], s[3], bc[6];
  int64_t off, S;
} geom;

static geom get_geom(const int32_t* m, int64_t off, int ndim) {
  geom G;
  G.level = m[0];
  for (int d = 0; d < 3; ++d) {
    G.n[d] = m[4 + d];
    G.g[d] = (d < ndim) ? m[7] : 0;
    G.s[d] = G.n[d] + 2 * G.g[d];
  }
  for (int f = 0; f < 6; ++f) G.bc[f] = m[8 + f];
  G.off = off;
  G.S = (int64_t)G.s[0] * G.s[1] * G.s[2];
  return G;
}

/* Element index of variable k of the cell with active-relative coordinates c[3]
 * (c[d] in [-g, n+g)). */
static int64_t at(const geom* G, int k, const int c[3]) {
  int64_t cell = ((int64_t)(c[2] + G->g[2]) * G->s[1] + (c[1] + G->g[1])) * G->s[0] + (c[0] + G->g[0]);
  return G->off + (int64_t)k * G->S + cell;
}

static int is_level(const int32_t* m, int level) { return level < 0 || m[0] == level; }

/* ---------------------------------------------------------------- physics */
double or_minmod3(double a, double b, double c) {
  /* Sec. 4: minmod(a,b,c) = 0.25 (sgn a + sgn b) |sgn a + sgn c| min(|a|,|b|,|c|). */
  double sa = (a > 0) - (a < 0), sb = (b > 0) - (b < 0), sc = (c > 0) - (c < 0);
  double m = fmin(fabs(a), fmin(fabs(b), fabs(c)));
  return 0.25 * (sa + sb) * fabs(sa + sc) * m;
}

int or_prim(const or_phys* ph, const double* U, double* q) {
  /* Sec. 4: U = (rho, rho v, rho E), E = v^2/2 + e, ideal gas p = (gamma-1) rho e.
   * MHD section: the energy variable is rho E + B^2/2 and B follows; the reconstructed
   * primitives are the hydro set plus B. */
  const int nv = ph->nvar;
  int bad = 0;
  for (int k = 0; k < nv; ++k)
    if (!isfinite(U[k])) bad = 1;
  double rho = U[0];
  double vx = U[1] / rho, vy = U[2] / rho, vz = U[3] / rho;
  double kin = 0.5 * ((U[1] * U[1] + U[2] * U[2]) + U[3] * U[3]) / rho; /* rho v^2 / 2 */
  double e;
  if (nv >= 8) {
    double mag = 0.5 * ((U[5] * U[5] + U[6] * U[6]) + U[7] * U[7]); /* B^2 / 2 */
    e = ((U[4] - kin) - mag) / rho;
  } else {
    e = (U[4] - kin) / rho;
  }
  if (!(rho > 0) && !(ph->rho_floor > 0)) bad = 1;
  if (!(e > 0) && !(ph->e_floor > 0)) bad = 1;
  if (ph->rho_floor > 0 && rho < ph->rho_floor) rho = ph->rho_floor;
  if (ph->e_floor > 0 && e < ph->e_floor) e = ph->e_floor;
  q[0] = rho;
  q[1] = ph->recon == OR_RECON_P ? (ph->gamma - 1.0) * rho * e : e;
  q[2] = vx;
  q[3] = vy;
  q[4] = vz;
  if (nv >= 8) {
    q[5] = U[5];
    q[6] = U[6];
    q[7] = U[7];
  }
  if (nv == 9) q[8] = U[8]; /* psi */
  q[nv] = (ph->gamma - 1.0) * rho * e;
  return bad;
}

/* Specific internal energy and pressure of a primitive state, whose slot 1 holds e
 * (p = (gamma-1) rho e) or, with the pressure reconstruction, p (e = p / ((gamma-1) rho)). */
static void eos(const or_phys* ph, const double* q, double* e, double* p) {
  if (ph->recon == OR_RECON_P) {
    *p = q[1];
    *e = q[1] / ((ph->gamma - 1.0) * q[0]);
  } else {
    *e = q[1];
    *p = (ph->gamma - 1.0) * q[0] * q[1];
  }
}

/* Signal speed along d of a primitive state: the sound speed sqrt(gamma p / rho) for
 * hydro; for MHD the fast magnetosonic speed
 *   c_f^2 = (a^2 + b^2 + sqrt((a^2 + b^2)^2 - 4 a^2 b_d^2)) / 2,
 * a^2 = gamma p / rho, b^2 = |B|^2 / rho, b_d^2 = B_d^2 / rho.  The radicand is evaluated
 * as (a^2 - b^2)^2 + 4 a^2 b_t^2 with b_t^2 = b^2 - b_d^2 formed from the two transverse
 * components: the same quantity, a sum of non-negative terms, with no cancellation where
 * a = b_d. */
double or_signal_speed(const or_phys* ph, int d, const double* q) {
  double e, p;
  eos(ph, q, &e, &p);
  double a2 = ph->gamma * p / q[0];
  if (ph->nvar < 8) return sqrt(a2);
  double b2 = ((q[5] * q[5] + q[6] * q[6]) + q[7] * q[7]) / q[0];
  int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  double bt2 = (q[5 + t1] * q[5 + t1] + q[5 + t2] * q[5 + t2]) / q[0];
  double dab = a2 - b2;
  double r = dab * dab + 4.0 * a2 * bt2;
  return sqrt(0.5 * ((a2 + b2) + sqrt(r)));
}

/* Conserved state, pressure and signal speed along d of one primitive face state. */
static void face_state(const or_phys* ph, int d, const double* q, double* U, double* p, double* c) {
  double rho = q[0], vx = q[2], vy = q[3], vz = q[4], e;
  eos(ph, q, &e, p);
  *c = or_signal_speed(ph, d, q);
  U[0] = rho;
  U[1] = rho * vx;
  U[2] = rho * vy;
  U[3] = rho * vz;
  U[4] = rho * (e + 0.5 * ((vx * vx + vy * vy) + vz * vz));
  if (ph->nvar >= 8) {
    U[4] = U[4] + 0.5 * ((q[5] * q[5] + q[6] * q[6]) + q[7] * q[7]); /* + B^2/2 */
    U[5] = q[5];
    U[6] = q[6];
    U[7] = q[7];
  }
  if (ph->nvar == 9) U[8] = q[8];
}

void or_phys_flux(const or_phys* ph, int d, const double* q, double* F) {
  /* Sec. 4 flux vectors: F^d = (rho v_d, rho v_d v + p e_d, rho (v^2/2 + h) v_d),
   * with rho (v^2/2 + h) = rho E_h + p, E_h = v^2/2 + e, since h = e + p/rho.
   * MHD fluxes: momentum rho v_d v_j + (p + B^2/2) delta_jd - B_j B_d; energy
   * rho (v^2/2 + h) v_d + B^2 v_d - B_d (B . v); induction v_d B_j - v_j B_d for j != d
   * (the x flux as printed; the printed y and z induction entries are permuted, and the
   * axis-permutation invariance of the system fixes them) and psi for j = d (0 with 8
   * variables); with 9 variables the psi flux is c_h^2 B_d (GLM). */
  double U[OR_NVMAX], p, c;
  face_state(ph, d, q, U, &p, &c);
  double vd = q[2 + d], e, pe;
  eos(ph, q, &e, &pe);
  double rEh = q[0] * (e + 0.5 * ((q[2] * q[2] + q[3] * q[3]) + q[4] * q[4]));
  F[0] = U[1 + d];
  if (ph->nvar < 8) {
    for (int j = 0; j < 3; ++j) F[1 + j] = U[1 + d] * q[2 + j] + (j == d ? p : 0.0);
    F[4] = (rEh + p) * vd;
    return;
  }
  double B2 = (q[5] * q[5] + q[6] * q[6]) + q[7] * q[7];
  double Bd = q[5 + d];
  double Bv = (q[5] * q[2] + q[6] * q[3]) + q[7] * q[4];
  for (int j = 0; j < 3; ++j)
    F[1 + j] = (U[1 + d] * q[2 + j] + (j == d ? p + 0.5 * B2 : 0.0)) - q[5 + j] * Bd;
  F[4] = ((rEh + p) * vd + B2 * vd) - Bd * Bv;
  for (int j = 0; j < 3; ++j) F[5 + j] = j == d ? 0.0 : vd * q[5 + j] - q[2 + j] * Bd;
  if (ph->nvar == 9) { /* GLM: the normal field is carried by psi, psi by c_h^2 B_d */
    F[5 + d] = q[8];
    F[8] = ph->ch * ph->ch * Bd;
  }
}

void or_face_flux(const or_phys* ph, int d, const double* qL, const double* qR, double* F) {
  /* Sec. 4 Riemann flux.  lambda^+- = v_d +- c for each face state (c the sound speed,
   * or for MHD the fast magnetosonic speed along d), a+ = max(0, lambda+_L, lambda+_R),
   * a- = max(0, -lambda-_L, -lambda-_R), lambda0 = max(a+, a-);
   * F = 0.5 (F_L + F_R - lambda0 (U_R - U_L)). */
  const int nv = ph->nvar;
  double UL[OR_NVMAX], UR[OR_NVMAX], FL[OR_NVMAX], FR[OR_NVMAX], pL, pR, cL, cR;
  face_state(ph, d, qL, UL, &pL, &cL);
  face_state(ph, d, qR, UR, &pR, &cR);
  or_phys_flux(ph, d, qL, FL);
  or_phys_flux(ph, d, qR, FR);
  double vL = qL[2 + d], vR = qR[2 + d];
  double ap = fmax(0.0, fmax(vL + cL, vR + cR));
  double am = fmax(0.0, fmax(-(vL - cL), -(vR - cR)));
  if (nv == 9) { /* the (B_d, psi) pair travels at -c_h and +c_h */
    ap = fmax(ap, ph->ch);
    am = fmax(am, ph->ch);
  }
  if (ph->flux == OR_FLUX_HLL2) {
    /* Two-speed HLL (Harten, Lax & van Leer 1983) with S_R = a+, S_L = -a-. */
    for (int k = 0; k < nv; ++k)
      F[k] = ((ap * FL[k] + am * FR[k]) - (ap * am) * (UR[k] - UL[k])) / (ap + am);
  } else {
    double lam = fmax(ap, am);
    for (int k = 0; k < nv; ++k) F[k] = 0.5 * ((FL[k] + FR[k]) - lam * (UR[k] - UL[k]));
  }
}

/* ---------------------------------------------------------------- O1 ghosts */
/* EXTERNAL face of patch p: each ghost cell takes the value of the same cell
 * (in level index space) of the same-level patch that holds it as an active
 * cell (Sec. 3: grids of one level exchange boundary values). */
/* Coarse data at time fraction alpha between the coarse level's old and new states
 * (linear in time), for one storage element. */
static double coarse_at(const double* Cold, const double* Cnew, double alpha, int64_t e) {
  double a = (1.0 - alpha) * Cold[e];
  double b = alpha * Cnew[e];
  return a + b;
}

/* Two-argument minmod (the classic limiter of the prolongation slopes). */
static double minmod2(double a, double b) {
  if (a > 0 && b > 0) return a < b ? a : b;
  if (a < 0 && b < 0) return a > b ? a : b;
  return 0.0;
}

/* Coarse -> fine conservative prolongation of one fine ghost cell at level index L
 * (Berger & Colella refinement by 2): the coarse cell C = L/2 holding it, a limited
 * linear profile per dimension with slopes minmod(u(C+1)-u(C), u(C)-u(C-1)) of the
 * time-interpolated coarse state, evaluated at the fine cell's centre (offset +-1/4
 * of a coarse cell).  The 2^d children of C average to u(C).  Returns 0 if no coarse
 * patch holds C. */
static int prolong_cell(int32_t np, const int32_t* meta, const int64_t* off, const or_phys* ph, const double* Cold,
                        const double* Cnew, double alpha, int level, const int L[3], double* out) {
  int Cc[3] = {0, 0, 0};
  for (int e = 0; e < ph->ndim; ++e) Cc[e] = L[e] >> 1; /* L >= 0 after the periodic wrap */
  /* the patches of a level are disjoint, so at most one holds C; the search starts at the
   * patch that held the previous cell (neighbouring ghost cells share it) */
  static _Thread_local int last = 0;
  for (int i = 0; i < np; ++i) {
    const int q = (last + i) % np;
    const int32_t* mq = meta + (size_t)q * OR_META;
    if (mq[0] != level - 1) continue;
    int inside = 1;
    for (int e = 0; e < ph->ndim; ++e)
      if (Cc[e] < mq[1 + e] || Cc[e] >= mq[1 + e] + mq[4 + e]) inside = 0;
    if (!inside) continue;
    geom Q = get_geom(mq, off[q], ph->ndim);
    int c0[3] = {0, 0, 0};
    for (int e = 0; e < ph->ndim; ++e) c0[e] = Cc[e] - mq[1 + e];
    for (int k = 0; k < ph->nvar; ++k) {
      double u0 = coarse_at(Cold, Cnew, alpha, at(&Q, k, c0));
      double v = u0;
      for (int e = 0; e < ph->ndim; ++e) {
        int cp[3] = {c0[0], c0[1], c0[2]}, cm[3] = {c0[0], c0[1], c0[2]};
        cp[e] += 1;
        cm[e] -= 1;
        double up = coarse_at(Cold, Cnew, alpha, at(&Q, k, cp));
        double um = coarse_at(Cold, Cnew, alpha, at(&Q, k, cm));
        double sg = minmod2(up - u0, u0 - um);
        double sgn = (L[e] & 1) ? 0.25 : -0.25;
        v = v + sgn * sg;
      }
      out[k] = v;
    }
    last = q;
    return 1;
  }
  return 0;
}

/* Does the cell interval [a, b) of an axis meet [c, e)?  On a periodic axis of length D
 * (D > 0) the interval is taken modulo D. */
static int axis_meets(int a, int b, int c, int e, int D) {
  if (D <= 0) return a < e && c < b;
  if (b - a >= D) return 1;
  int a0 = ((a % D) + D) % D, b0 = a0 + (b - a);
  if (b0 <= D) return a0 < e && c < b0;
  return (a0 < e && c < D) || (0 < e && c < b0 - D);
}

static void fill_external(int32_t np, const int32_t* meta, const int64_t* off, const or_phys* ph, double* V, int p,
                          const geom* G, int d, int side, const double* Cold, const double* Cnew, double alpha) {
  const int32_t* m = meta + (size_t)p * OR_META;
  int a = (d + 1) % 3, b = (d + 2) % 3;
  /* The same-level patches whose box meets this face's ghost slab: only these can hold a
   * ghost cell (a pure lookup; the patches of a level are disjoint, so the holder of a
   * cell is unique and the search order does not matter). */
  int* cand = malloc(sizeof(int) * (size_t)np);
  int nc = 0;
  {
    int slo[3], shi[3];
    for (int e = 0; e < 3; ++e) {
      slo[e] = m[1 + e];
      shi[e] = m[1 + e] + G->n[e];
    }
    slo[d] = side == 0 ? m[1 + d] - G->g[d] : m[1 + d] + G->n[d];
    shi[d] = slo[d] + G->g[d];
    for (int q = 0; q < np; ++q) {
      const int32_t* mq = meta + (size_t)q * OR_META;
      if (mq[0] != m[0]) continue; /* p itself can hold them across a periodic wrap */
      int meets = 1;
      for (int e = 0; e < ph->ndim && meets; ++e) {
        int D = ((ph->periodic >> e) & 1) ? (ph->domain[e] << m[0]) : 0;
        meets = axis_meets(slo[e], shi[e], mq[1 + e], mq[1 + e] + mq[4 + e], D);
      }
      if (meets) cand[nc++] = q;
    }
  }
  int last = 0;
  for (int layer = 1; layer <= G->g[d]; ++layer) {
    int gi = side == 0 ? -layer : G->n[d] - 1 + layer;
    for (int ib = 0; ib < G->n[b]; ++ib)
      for (int ia = 0; ia < G->n[a]; ++ia) {
        int cg[3], L[3];
        cg[d] = gi; cg[a] = ia; cg[b] = ib;
        for (int e = 0; e < 3; ++e) {
          L[e] = m[1 + e] + cg[e]; /* level index space */
          if (e < ph->ndim && ((ph->periodic >> e) & 1)) {
            int dom = ph->domain[e] << m[0];
            L[e] = ((L[e] % dom) + dom) % dom;
          }
        }
        int found = 0;
        for (int i = 0; i < nc; ++i) { /* start at the last hit: neighbouring cells share it */
          const int q = cand[(last + i) % nc];
          const int32_t* mq = meta + (size_t)q * OR_META;
          int inside = 1;
          for (int e = 0; e < ph->ndim; ++e)
            if (L[e] < mq[1 + e] || L[e] >= mq[1 + e] + mq[4 + e]) inside = 0;
          if (!inside) continue;
          geom Q = get_geom(mq, off[q], ph->ndim);
          int cs[3] = {0, 0, 0};
          for (int e = 0; e < ph->ndim; ++e) cs[e] = L[e] - mq[1 + e];
          for (int k = 0; k < ph->nvar; ++k) V[at(G, k, cg)] = V[at(&Q, k, cs)];
          found = 1;
          last = (last + i) % nc;
          break;
        }
        if (!found && m[0] > 0 && Cold && Cnew) {
          double u[OR_NVMAX];
          if (prolong_cell(np, meta, off, ph, Cold, Cnew, alpha, m[0], L, u))
            for (int k = 0; k < ph->nvar; ++k) V[at(G, k, cg)] = u[k];
        }
      }
  }
  free(cand);
}


int or_fill_ghosts(int32_t np, const int32_t* meta, const int64_t* off, const or_phys* ph,
                   double* V, int32_t level) {
  return or_fill_ghosts_amr(np, meta, off, ph, V, level, NULL, NULL, 0.0);
}

int or_fill_ghosts_amr(int32_t np, const int32_t* meta, const int64_t* off, const or_phys* ph, double* V,
                       int32_t level, const double* Cold, const double* Cnew, double alpha) {
  /* each patch writes only its own ghost cells and reads active cells */
#pragma omp parallel for schedule(dynamic)
  for (int p = 0; p < np; ++p) {
    const int32_t* m = meta + (size_t)p * OR_META;
    if (!is_level(m, level)) continue;
    geom G = get_geom(m, off[p], ph->ndim);
    for (int d = 0; d < ph->ndim; ++d) {
      int a = (d + 1) % 3, b = (d + 2) % 3; /* the two other dimensions */
      for (int side = 0; side < 2; ++side) {
        int bc = G.bc[2 * d + side];
        if (bc == OR_BC_EXTERNAL) {
          fill_external(np, meta, off, ph, V, p, &G, d, side, Cold, Cnew, alpha);
          continue;
        }
        for (int layer = 1; layer <= G.g[d]; ++layer) {
          int gi = side == 0 ? -layer : G.n[d] - 1 + layer; /* ghost index along d */
          int si;                                            /* source index along d */
          double sgn = 1.0;
          if (bc == OR_BC_OUTFLOW) {
            si = side == 0 ? 0 : G.n[d] - 1;
          } else if (bc == OR_BC_PERIODIC) {
            si = ((gi % G.n[d]) + G.n[d]) % G.n[d];
          } else { /* reflect about the boundary face */
            si = side == 0 ? layer - 1 : G.n[d] - layer;
            sgn = -1.0;
          }
          for (int ib = 0; ib < G.n[b]; ++ib)
            for (int ia = 0; ia < G.n[a]; ++ia) {
              int cg[3], cs[3];
              cg[d] = gi; cg[a] = ia; cg[b] = ib;
              cs[d] = si; cs[a] = ia; cs[b] = ib;
              for (int k = 0; k < ph->nvar; ++k) {
                double v = V[at(&G, k, cs)];
                if (k == 1 + d || (ph->nvar >= 8 && k == 5 + d)) v = sgn * v; /* normal v and B */
                V[at(&G, k, cg)] = v;
              }
            }
        }
      }
    }
  }
  return 0;
}

/* ---------------------------------------------------------------- regrid */
/* Fill the active cells of a new hierarchy (np patches, arena U) from an old one (npo
 * patches, arena Uo) when the hierarchy is rebuilt (Sec. 3: the host rebuilds the grid
 * hierarchy, and new fine grids take their data from the grids they replace, else from the
 * coarser level).  Level by level from the root: a cell that an old patch of the same level
 * holds is copied from it; any other cell is prolonged (the conservative minmod-linear
 * interpolation of the ghost cells) from the new level below, whose ghost layers are filled
 * first (siblings, physical boundaries, and coarser data for its own coarse/fine faces).
 * Returns the number of cells that had no source (0 for a properly nested new root level
 * covered by the old root). */
int64_t or_regrid_fill(int32_t npo, const int32_t* meta_o, const int64_t* off_o, const double* Uo, int32_t np,
                       const int32_t* meta, const int64_t* off, const or_phys* ph, double* U) {
  int nlev = 0;
  for (int p = 0; p < np; ++p)
    if (meta[(size_t)p * OR_META] + 1 > nlev) nlev = meta[(size_t)p * OR_META] + 1;
  int64_t missing = 0;
  for (int l = 0; l < nlev; ++l) {
    for (int p = 0; p < np; ++p) {
      const int32_t* m = meta + (size_t)p * OR_META;
      if (m[0] != l) continue;
      geom G = get_geom(m, off[p], ph->ndim);
      for (int k3 = 0; k3 < G.n[2]; ++k3)
        for (int j = 0; j < G.n[1]; ++j)
          for (int i = 0; i < G.n[0]; ++i) {
            int c[3] = {i, j, k3}, L[3] = {0, 0, 0};
            for (int e = 0; e < ph->ndim; ++e) L[e] = m[1 + e] + c[e];
            int done = 0;
            for (int q = 0; q < npo && !done; ++q) { /* an old patch of this level holding L */
              const int32_t* mq = meta_o + (size_t)q * OR_META;
              if (mq[0] != l) continue;
              int inside = 1;
              for (int e = 0; e < ph->ndim; ++e)
                if (L[e] < mq[1 + e] || L[e] >= mq[1 + e] + mq[4 + e]) inside = 0;
              if (!inside) continue;
              geom Q = get_geom(mq, off_o[q], ph->ndim);
              int cs[3] = {0, 0, 0};
              for (int e = 0; e < ph->ndim; ++e) cs[e] = L[e] - mq[1 + e];
              for (int k = 0; k < ph->nvar; ++k) U[at(&G, k, c)] = Uo[at(&Q, k, cs)];
              done = 1;
            }
            if (!done && l > 0) {
              double u[OR_NVMAX];
              if (prolong_cell(np, meta, off, ph, U, U, 0.0, l, L, u)) {
                for (int k = 0; k < ph->nvar; ++k) U[at(&G, k, c)] = u[k];
                done = 1;
              }
            }
            if (!done) ++missing;
          }
    }
    /* this level's ghost layers, read by the next level's prolongation stencils */
    or_fill_ghosts_amr(np, meta, off, ph, U, l, U, U, 0.0);
  }
  return missing;
}

/* ---------------------------------------------------------------- O2-O6 L(U) */
int or_patch_L(const int32_t* m, int64_t off, const or_phys* ph, const double* V, double* L) {
  return or_patch_L_rec(m, off, ph, V, L, NULL);
}

int64_t or_face_record_size(const int32_t* m, const or_phys* ph) {
  int64_t tot = 0;
  for (int d = 0; d < ph->ndim; ++d) {
    int64_t c = (int64_t)ph->nvar * (m[4 + d] + 1);
    for (int e = 0; e < 3; ++e)
      if (e != d) c *= m[4 + e];
    tot += c;
  }
  return tot;
}

int or_patch_L_rec(const int32_t* m, int64_t off, const or_phys* ph, const double* V, double* L, double* Frec) {
  geom G = get_geom(m, off, ph->ndim);
  const int nv = ph->nvar;
  int bad = 0;
  int64_t nact = (int64_t)G.n[0] * G.n[1] * G.n[2];
  for (int64_t i = 0; i < nv * nact; ++i) L[i] = 0.0;
  int maxn = G.n[0] > G.n[1] ? G.n[0] : G.n[1];
  if (G.n[2] > maxn) maxn = G.n[2];
  /* line buffers, indexed by position along the line + 2 (cells -2 .. n+1) */
  double(*q)[OR_NVMAX] = malloc(sizeof(double[OR_NVMAX]) * (size_t)(maxn + 4));
  double(*sig)[OR_NVMAX] = malloc(sizeof(double[OR_NVMAX]) * (size_t)(maxn + 4));
  double(*F)[OR_NVMAX] = malloc(sizeof(double[OR_NVMAX]) * (size_t)(maxn + 1));
  for (int d = 0; d < ph->ndim; ++d) {
    /* Sec. 4 MOL equation: the d-flux needs only cells along d; level l has dx0/2^l. */
    double dxd = ldexp(ph->dx0[d], -G.level);
    int a = (d + 1) % 3, b = (d + 2) % 3, n = G.n[d];
    for (int ib = 0; ib < G.n[b]; ++ib)
      for (int ia = 0; ia < G.n[a]; ++ia) {
        /* O2: primitives of cells -2 .. n+1 along the line */
        for (int i = -2; i <= n + 1; ++i) {
          int c[3];
          c[d] = i; c[a] = ia; c[b] = ib;
          double Uc[OR_NVMAX], w[OR_NVMAX + 1];
          for (int k = 0; k < nv; ++k) Uc[k] = V[at(&G, k, c)];
          bad |= or_prim(ph, Uc, w);
          for (int k = 0; k < nv; ++k) q[i + 2][k] = w[k];
        }
        /* O3: limited slope of cells -1 .. n (Sec. 4 PLM with theta-minmod) */
        for (int i = -1; i <= n; ++i)
          for (int k = 0; k < nv; ++k) {
            double qm = q[i + 1][k], q0 = q[i + 2][k], qp = q[i + 3][k];
            sig[i + 2][k] = or_minmod3(ph->theta * (q0 - qm), ph->theta * (qp - q0), (qp - qm) / 2.0);
          }
        /* O4-O5: flux at face f (between cells f-1 and f), f = 0 .. n */
        for (int f = 0; f <= n; ++f) {
          double qL[OR_NVMAX], qR[OR_NVMAX];
          for (int k = 0; k < nv; ++k) {
            qL[k] = q[f + 1][k] + 0.5 * sig[f + 1][k]; /* u_{f-1/2,l} = u_{f-1} + sigma_{f-1}/2 */
            qR[k] = q[f + 2][k] - 0.5 * sig[f + 2][k]; /* u_{f-1/2,r} = u_f - sigma_f/2 */
          }
          or_face_flux(ph, d, qL, qR, F[f]);
        }
        if (Frec) { /* every face flux of the line: [v][ib][ia][f] within this dimension's block */
          int64_t base = 0;
          for (int e = 0; e < d; ++e) {
            int64_t c = (int64_t)nv * (G.n[e] + 1);
            for (int e2 = 0; e2 < 3; ++e2)
              if (e2 != e) c *= G.n[e2];
            base += c;
          }
          for (int k = 0; k < nv; ++k)
            for (int f = 0; f <= n; ++f)
              Frec[base + (((int64_t)k * G.n[b] + ib) * G.n[a] + ia) * (n + 1) + f] = F[f][k];
        }
        /* O6: L_i -= (F_{i+1/2} - F_{i-1/2}) / dx_d, dimensions in the order x, y, z */
        for (int i = 0; i < n; ++i) {
          int c[3];
          c[d] = i; c[a] = ia; c[b] = ib;
          int64_t cell = ((int64_t)c[2] * G.n[1] + c[1]) * G.n[0] + c[0];
          for (int k = 0; k < nv; ++k) L[k * nact + cell] = L[k * nact + cell] - (F[i + 1][k] - F[i][k]) / dxd;
        }
      }
  }
  free(q);
  free(sig);
  free(F);
  return bad;
}

/* ---------------------------------------------------------------- O7 stages */
int or_stage(int32_t np, const int32_t* meta, const int64_t* off, const or_phys* ph,
             const double* V, const double* U0, double* out, double dt, int32_t stage, int32_t level) {
  return or_stage_rec(np, meta, off, ph, V, U0, out, dt, stage, level, NULL, NULL);
}

int or_stage_rec(int32_t np, const int32_t* meta, const int64_t* off, const or_phys* ph, const double* V,
                 const double* U0, double* out, double dt, int32_t stage, int32_t level, const int64_t* rec_off,
                 double* Frec) {
  int bad = 0;
  /* patches are independent within a stage: the OpenMP build (timing only) runs them on
   * several cores; the serial build ignores the pragma */
#pragma omp parallel for schedule(dynamic) reduction(| : bad)
  for (int p = 0; p < np; ++p) {
    const int32_t* m = meta + (size_t)p * OR_META;
    if (!is_level(m, level)) continue;
    geom G = get_geom(m, off[p], ph->ndim);
    int64_t nact = (int64_t)G.n[0] * G.n[1] * G.n[2];
    double* L = malloc(sizeof(double) * ph->nvar * (size_t)nact);
    bad |= or_patch_L_rec(m, off[p], ph, V, L, (Frec && rec_off && rec_off[p] >= 0) ? Frec + rec_off[p] : NULL);
    for (int k3 = 0; k3 < G.n[2]; ++k3)
      for (int j = 0; j < G.n[1]; ++j)
        for (int i = 0; i < G.n[0]; ++i) {
          int c[3] = {i, j, k3};
          int64_t cell = ((int64_t)k3 * G.n[1] + j) * G.n[0] + i;
          for (int k = 0; k < ph->nvar; ++k) {
            int64_t e = at(&G, k, c);
            double u1 = V[e] + dt * L[k * nact + cell]; /* Sec. 4 TVD-RK2: U + dt L(U) */
            out[e] = stage == 1 ? u1 : 0.5 * U0[e] + 0.5 * u1;
          }
        }
    free(L);
  }
  return bad;
}

int or_rk2_step(int32_t np, const int32_t* meta, const int64_t* off, const or_phys* ph,
                double* U, double* W, double dt, int32_t level) {
  /* Sec. 4 (Shu-Osher TVD-RK2): U1 = Un + dt L(Un); Un+1 = Un/2 + U1/2 + dt L(U1)/2. */
  int bad = 0;
  or_fill_ghosts(np, meta, off, ph, U, level);
  bad |= or_stage(np, meta, off, ph, U, NULL, W, dt, 1, level);
  or_fill_ghosts(np, meta, off, ph, W, level);
  bad |= or_stage(np, meta, off, ph, W, U, U, dt, 2, level);
  return bad;
}

/* ---------------------------------------------------------------- O9 CFL */
double or_max_speed(int32_t np, const int32_t* meta, const int64_t* off, const or_phys* ph,
                    const double* U, int32_t level, int* flag) {
  double smax = 0.0;
  int bad = 0;
#pragma omp parallel for schedule(dynamic) reduction(max : smax) reduction(| : bad)
  for (int p = 0; p < np; ++p) {
    const int32_t* m = meta + (size_t)p * OR_META;
    if (!is_level(m, level)) continue;
    geom G = get_geom(m, off[p], ph->ndim);
    for (int k3 = 0; k3 < G.n[2]; ++k3)
      for (int j = 0; j < G.n[1]; ++j)
        for (int i = 0; i < G.n[0]; ++i) {
          int c[3] = {i, j, k3};
          double Uc[OR_NVMAX], w[OR_NVMAX + 1];
          for (int k = 0; k < ph->nvar; ++k) Uc[k] = U[at(&G, k, c)];
          bad |= or_prim(ph, Uc, w);
          double s = 0.0;
          for (int d = 0; d < ph->ndim; ++d) {
            double sd = fabs(w[2 + d]) + or_signal_speed(ph, d, w);
            if (ph->nvar == 9) sd = fmax(sd, ph->ch); /* the GLM waves */
            s = s + sd / ldexp(ph->dx0[d], -G.level);
          }
          if (s > smax) smax = s;
        }
  }
  if (flag) *flag = bad;
  return smax;
}

double or_cfl_dt(int32_t np, const int32_t* meta, const int64_t* off, const or_phys* ph,
                 const double* U, double cfl, int32_t level) {
  int bad = 0;
  double s = or_max_speed(np, meta, off, ph, U, level, &bad);
  return cfl / s;
}

/* ---------------------------------------------------------------- flagging */
int64_t or_flag_cells(int32_t np, const int32_t* meta, const int64_t* off, const or_phys* ph, const double* V,
                      int32_t level, double eps, uint8_t* flags) {
  /* A cell is flagged for refinement where its density jumps by more than eps, relative to
   * the smaller of the two, to any face neighbour: |rho_n - rho_c| / min(rho_n, rho_c) > eps.
   * Neighbours across a patch face are read from ghost storage (filled beforehand). */
  int64_t w = 0;
  for (int p = 0; p < np; ++p) {
    const int32_t* m = meta + (size_t)p * OR_META;
    if (!is_level(m, level)) continue;
    geom G = get_geom(m, off[p], ph->ndim);
    for (int k3 = 0; k3 < G.n[2]; ++k3)
      for (int j = 0; j < G.n[1]; ++j)
        for (int i = 0; i < G.n[0]; ++i) {
          int c[3] = {i, j, k3};
          double rc = V[at(&G, 0, c)];
          int f = 0;
          for (int d = 0; d < ph->ndim; ++d)
            for (int s = -1; s <= 1; s += 2) {
              int nb[3] = {i, j, k3};
              nb[d] += s;
              double rn = V[at(&G, 0, nb)];
              if (fabs(rn - rc) / fmin(rn, rc) > eps) f = 1;
            }
          flags[w++] = (uint8_t)f;
        }
  }
  return w;
}
