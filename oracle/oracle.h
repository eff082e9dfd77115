/* oracle.h - serial FP64 CPU oracle for the per-patch MOL hydro update of
 * Wang, Abel & Kaehler, "Adaptive Mesh Fluid Simulations on GPU".
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously correct
 * reference that the GPU path is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark load it; the product
 * path never links, imports or calls it.  It shares no code, header or table
 * with the GPU library.
 *
 * Storage convention (the same *format* the GPU library accepts, written here
 * independently): a patch has n[d] active cells and g[d] ghost layers per side
 * in each active dimension d < ndim (g[d] = 0, n[d] = 1 in absent dimensions);
 * s[d] = n[d] + 2 g[d].  Variable k of cell (i,j,k) (storage indices, x fastest)
 * lives at  U[off + k*S + (kz*s[1] + jy)*s[0] + ix]  with S = s[0]*s[1]*s[2].
 * Variables (nvar = 5) are the conserved U = (rho, rho vx, rho vy, rho vz, rho E)
 * of the paper's Sec. 4, with rho E the total energy density; for ideal MHD
 * (nvar = 8) they are (rho, rho v, rho E + B^2/2, Bx, By, Bz), the paper's MHD
 * variables with the divergence-cleaning field psi held at zero; for GLM-MHD (nvar = 9)
 * psi follows B, with the cleaning speed ch of the physics block.
 *
 * Patch metadata is an int32 array of OR_META entries per patch:
 *   [0] level, [1..3] lo (lower active index in level space), [4..6] n,
 *   [7] ng, [8..13] bc for faces -x,+x,-y,+y,-z,+z, [14..15] unused.
 */
#ifndef PAPER_ORACLE_H
#define PAPER_ORACLE_H
#include <stdint.h>

#define OR_META 16
#define OR_NVMAX 9 /* hydro: 5 variables; ideal MHD: 8; GLM-MHD (with the cleaning field psi): 9 */
enum { OR_BC_OUTFLOW = 0, OR_BC_PERIODIC = 1, OR_BC_REFLECT = 2, OR_BC_EXTERNAL = 3 };
enum { OR_FLUX_PAPER = 0, OR_FLUX_HLL2 = 1 };
/* Second reconstructed thermodynamic variable: specific internal energy e (the set the
 * paper's flux kernel stages), or pressure p. */
enum { OR_RECON_E = 0, OR_RECON_P = 1 };

typedef struct {
  int32_t nvar, ndim;
  double gamma, theta;
  double dx0[3];
  int32_t flux, periodic;  /* periodic: bit d = root domain periodic in d (EXTERNAL ghosts wrap) */
  int32_t domain[3];       /* root-level domain extent in cells */
  int32_t recon;           /* OR_RECON_E or OR_RECON_P */
  double rho_floor, e_floor;
  double ch;               /* GLM cleaning speed c_h (nvar = 9) */
} or_phys;

#ifdef __cplusplus
extern "C" {
#endif

/* Three-argument minmod of Sec. 4 (0.25(sgn a+sgn b)|sgn a+sgn c| min|.|). */
double or_minmod3(double a, double b, double c);
/* Conserved -> primitives for one cell; returns 1 if unphysical.
 * nvar 5: q = (rho, e, vx, vy, vz), q[5] = p.  nvar 8: q = (rho, e, vx, vy, vz, Bx, By, Bz),
 * q[8] = p.  (nvar + 1 entries are written.)  With recon = OR_RECON_P, q[1] holds p. */
int or_prim(const or_phys* ph, const double* U, double* q);
/* Face flux in direction d (nvar entries) from primitive face states qL, qR (nvar entries). */
void or_face_flux(const or_phys* ph, int d, const double* qL, const double* qR, double* F);
/* Physical flux F^d(U(q)) for one primitive state (Sec. 4; MHD section for nvar 8). */
void or_phys_flux(const or_phys* ph, int d, const double* q, double* F);
/* Signal speed along d: sound speed (nvar 5) or fast magnetosonic speed (nvar 8). */
double or_signal_speed(const or_phys* ph, int d, const double* q);

/* O1: fill the face ghosts (all ng layers, over the active range of the other
 * dimensions) of every patch on `level` (-1 = all) from the boundary condition
 * of each face.  EXTERNAL ghosts are copied from the same-level patch whose
 * active cells contain them (after periodic wrap of the root domain); ghosts
 * with no such patch are left untouched. */
int or_fill_ghosts(int32_t np, const int32_t* meta, const int64_t* off, const or_phys* ph,
                   double* V, int32_t level);
/* As or_fill_ghosts, and EXTERNAL ghost cells that no same-level patch holds are
 * prolonged (conservative minmod-linear, refinement 2) from level-1 data taken at
 * time fraction alpha between Cold and Cnew (arenas with the coarse ghosts filled). */
int or_fill_ghosts_amr(int32_t np, const int32_t* meta, const int64_t* off, const or_phys* ph, double* V,
                       int32_t level, const double* Cold, const double* Cnew, double alpha);
/* Size of the face-flux record of one patch: for each active dimension d, nvar x
 * (n_d + 1) x prod(other n), laid out [v][b][a][face] with (a, b) the other two
 * dimensions in cyclic order after d. */
int64_t or_face_record_size(const int32_t* meta, const or_phys* ph);
/* L(V) as or_patch_L, also writing every face flux to Frec (if not NULL). */
int or_patch_L_rec(const int32_t* meta, int64_t off, const or_phys* ph, const double* V, double* L, double* Frec);
/* or_stage that also records each patch's face fluxes at Frec + rec_off[p] (rec_off[p] < 0: none). */
int or_stage_rec(int32_t np, const int32_t* meta, const int64_t* off, const or_phys* ph, const double* V,
                 const double* U0, double* out, double dt, int32_t stage, int32_t level, const int64_t* rec_off,
                 double* Frec);
/* L(V) of the MOL equation for one patch, written to L (nvar x active cells, x fastest).
 * V must have its ghosts filled.  Returns 1 if an unphysical state was met. */
int or_patch_L(const int32_t* meta, int64_t off, const or_phys* ph, const double* V, double* L);
/* One RK2 stage over the patches of `level`: stage 1 out = V + dt L(V);
 * stage 2 out = 0.5 U0 + 0.5 (V + dt L(V)).  Active cells only. */
int or_stage(int32_t np, const int32_t* meta, const int64_t* off, const or_phys* ph,
             const double* V, const double* U0, double* out, double dt, int32_t stage, int32_t level);
/* One full TVD-RK2 step of `level` on U (in place), W = scratch arena of the same size. */
int or_rk2_step(int32_t np, const int32_t* meta, const int64_t* off, const or_phys* ph,
                double* U, double* W, double dt, int32_t level);
/* Largest signal speed sum_d (|v_d| + c_d)/dx_d over active cells of `level`, c_d the
 * sound speed (hydro) or the fast magnetosonic speed along d (MHD). */
double or_max_speed(int32_t np, const int32_t* meta, const int64_t* off, const or_phys* ph,
                    const double* U, int32_t level, int* flag);
/* Refinement flags of the active cells of `level` (-1 = all), patch order, x fastest: 1 where
 * |rho_n - rho_c| / min(rho_n, rho_c) > eps for a face neighbour n (ghosts of V filled
 * beforehand).  Returns the number of flags written. */
int64_t or_flag_cells(int32_t np, const int32_t* meta, const int64_t* off, const or_phys* ph, const double* V,
                      int32_t level, double eps, uint8_t* flags);
/* dt = cfl / max speed (one level or a single-level table). */
double or_cfl_dt(int32_t np, const int32_t* meta, const int64_t* off, const or_phys* ph,
                 const double* U, double cfl, int32_t level);

/* New hierarchy (np patches, arena U) filled from an old one (npo patches, arena Uo): per
 * level from the root, copy from an old same-level patch, else prolong from the new level
 * below (its ghosts filled first).  Returns the number of cells left without a source. */
int64_t or_regrid_fill(int32_t npo, const int32_t* meta_o, const int64_t* off_o, const double* Uo, int32_t np,
                       const int32_t* meta, const int64_t* off, const or_phys* ph, double* U);
/* Threads of the oracle's parallel patch loops: 1 in the serial build. */
int or_threads(void);

#ifdef __cplusplus
}
#endif
#endif
