/* amr_hydro.h - C ABI of the MI355X (gfx950) per-patch hydro update.
 *
 * The library advances the Euler equations of Wang, Abel & Kaehler,
 * "Adaptive Mesh Fluid Simulations on GPU", Sec. 4 (conservation law in
 * conserved variables U = (rho, rho vx, rho vy, rho vz, rho E), ideal-gas EOS
 * p = (gamma-1) rho e), discretised by the method of lines (Sec. 4, MOL
 * equation dU/dt = L(U)) with PLM theta-minmod reconstruction of primitives
 * (Sec. 4, PLM and minmod equations), the paper's Riemann flux on every face of
 * every active dimension (Sec. 4, flux equation) and the two-stage TVD
 * Runge-Kutta scheme (Sec. 4, RK2 equation; three-step form of Sec. 5.1), on
 * each grid patch of a block-structured AMR hierarchy (Sec. 3), one patch being
 * the unit of GPU work (Sec. 5.2, Sec. 8).
 *
 * With nvar = 8 the same update advances ideal MHD (the paper's MHD section,
 * its divergence-cleaning field psi held at zero, so c_h plays no part):
 * U = (rho, rho vx, rho vy, rho vz, rho E + B^2/2, Bx, By, Bz), B joins the
 * reconstructed primitives, the physical flux is the paper's MHD flux with the
 * induction entries v_d B_j - v_j B_d (its x flux; the printed y and z induction
 * entries have their components permuted), the signal speed in the Riemann
 * flux and in the CFL rule is the fast magnetosonic speed along the face
 * normal, and REFLECT also negates the normal field.  With nvar = 9 the
 * cleaning field psi follows B (the paper's GLM system): the B_d entry of the
 * d-flux is psi, the psi entry c_h^2 B_d, and the pair's wave speeds -c_h and
 * +c_h join the Riemann flux's a+ and a- and the CFL rule (no damping source:
 * the paper writes none).  On a hierarchy the coarse/fine coupling (ghost
 * prolongation, restriction, refluxing) treats every conserved variable alike,
 * B and psi included: the prolonged and restricted field keeps the totals but is
 * not divergence-free in general (the paper's GLM field is what transports such
 * divergence away).
 *
 * Conventions shared by every entry point
 *   - Every function returns an amr_status: AMR_OK (0) or a negative code.
 *   - Device pointers (U, dt_dev) are caller-owned device memory (hipMalloc or
 *     a framework allocator); the caller keeps them alive until the stream
 *     work that uses them completes.
 *   - Streams: all work is enqueued on the caller's stream `stream` (0 = the
 *     null stream) and returns without waiting, unless a host pointer for a
 *     result is given (then the call synchronises that stream).
 *   - Argument errors are detected on the host before anything is enqueued and
 *     return AMR_EINVAL with nothing changed.  HIP runtime failures return
 *     AMR_EHIP.  An unphysical state met on the device (rho <= 0, e <= 0 or a
 *     non-finite value in a cell the stencil reads) is latched in the table and
 *     returned as AMR_EUNPHYSICAL by the next synchronising call
 *     (amr_cfl_dt with dt_host, amr_table_status); the U it produced is not
 *     meaningful.  Recovery is the caller's: amr_table_status (which clears
 *     the latch), restore U^n, then retry with a smaller dt.
 *   - A table is not thread-safe; calls on one table must be serialised.
 *
 * The U arena (layout of conserved state, caller-owned, FP64)
 *   One contiguous array of doubles holds every patch.  Patch p with n[d]
 *   active cells and ng ghost layers per side in each active dimension d < ndim
 *   (no ghosts, n[d] = 1 in absent dimensions) stores s[d] = n[d] + 2 g[d]
 *   cells per dimension, x fastest; variable k (0..nvar-1 in the order of U above)
 *   of storage cell (ix, iy, iz) is at element
 *       offset + k * S + (iz * s[1] + iy) * s[0] + ix,   S = s[0] s[1] s[2].
 *   Active cells are ix in [g, g + n[0]) and likewise in y and z.  Patches
 *   must not overlap.  Ghost storage is only read on faces whose boundary
 *   condition is AMR_BC_EXTERNAL (filled by the library from other patches);
 *   the other conditions are applied by index mapping, so those ghost cells
 *   may hold anything, and a patch may store none (ng = 0, g = 0: s = n).
 *   The library writes the active cells of U, the ghost cells of EXTERNAL
 *   faces, and, on a level with children in a hierarchy, the two ghost layers of
 *   the other faces (the children's prolongation stencils read them).
 */
#ifndef AMR_HYDRO_H
#define AMR_HYDRO_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t amr_status;
#define AMR_OK 0
#define AMR_EINVAL (-1)       /* bad argument; nothing was enqueued            */
#define AMR_ENOMEM (-2)       /* device or host allocation failed             */
#define AMR_EHIP (-3)         /* a HIP runtime call failed                     */
#define AMR_EUNPHYSICAL (-4)  /* rho <= 0, e <= 0 or non-finite state met       */
#define AMR_ESTATE (-5)       /* call not valid in the table's current state    */

/* Boundary condition of one patch face (Sec. 3 ghost zones; on-the-fly maps):
 *   OUTFLOW  ghost = copy of the nearest active cell (zero gradient),
 *   PERIODIC ghost = active cell one patch-length away (wrap within the patch),
 *   REFLECT  ghost = mirror image across the face, normal momentum (and, for MHD,
 *            normal field) negated,
 *   EXTERNAL ghost = filled by the library from the same-level patch that
 *            covers it (sibling copy); ghost storage is read by the stencil.
 *            In a single-level table, a face whose ghost cells all lie in one
 *            sibling with the same n and ng is read from that sibling's cells
 *            directly and its ghost storage is left untouched. */
enum { AMR_BC_OUTFLOW = 0, AMR_BC_PERIODIC = 1, AMR_BC_REFLECT = 2, AMR_BC_EXTERNAL = 3 };
/* Face flux: AMR_FLUX_PAPER = the formula printed in Sec. 4,
 *   F = (F_L + F_R - lambda0 (U_R - U_L)) / 2, lambda0 = max(a+, a-);
 * AMR_FLUX_HLL2 = the two-speed HLL flux with the same a+, a-:
 *   F = (a+ F_L + a- F_R - a+ a- (U_R - U_L)) / (a+ + a-). */
enum { AMR_FLUX_PAPER = 0, AMR_FLUX_HLL2 = 1 };
/* Arithmetic: FP64 throughout, or FP32 reconstruction and face flux with the
 * conserved->primitive conversion (pressure recovery), the flux divergence and
 * the RK combine in FP64. */
enum { AMR_PREC_FP64 = 0, AMR_PREC_MIXED = 1 };
/* Execution form: PLAIN = one launch per patch per stage; BATCHED = one
 * persistent launch per stage over a tile list of all selected patches, the
 * whole RK2 step replayed from a captured HIP graph. */
enum { AMR_EXEC_PLAIN = 0, AMR_EXEC_BATCHED = 1 };
/* Second reconstructed thermodynamic variable: AMR_RECON_E = the specific internal
 * energy e, the set (rho, e, v) the paper's flux kernel stages (Sec. 5), with the face
 * pressure p = (gamma-1) rho e; AMR_RECON_P = the pressure p, with e = p / ((gamma-1) rho)
 * at the face (keeps p and v exactly uniform across a contact). */
enum { AMR_RECON_E = 0, AMR_RECON_P = 1 };

/* flags of amr_hydro_rk2_step */
#define AMR_STEP_FUSE_DT 0x1u /* stage 2 also reduces the max signal speed of U^{n+1}; the
                                 next amr_cfl_dt on the same U and level then reads it
                                 instead of scanning U again */
#define AMR_STEP_TIMED 0x2u   /* enqueue this step eagerly (same kernels, same launch
                                 shapes as the batched graph) with HIP events around each
                                 stage kernel; read them with amr_table_last_stage_ms */
#define AMR_STEP_SUBSTEP1 0x4u /* hierarchies: this level step is the second of the two
                                 its parent level's step contains (its prolonged ghosts
                                 take the parent's state at times 1/2 and 1 of that step,
                                 instead of 0 and 1/2).  It must follow the same level's
                                 first substep of that parent step, with only the
                                 recursion below this level in between: the ghosts of
                                 its first stage (time 1/2) are the ones that first
                                 substep's second stage prolonged, reused, not
                                 interpolated again (without that first substep the
                                 step returns AMR_ESTATE) */

typedef struct {
  int32_t level;    /* refinement level, 0 = root; cell width dx0[d] / 2^level          */
  int32_t lo[3];    /* index of the first active cell in level index space             */
  int32_t n[3];     /* active cells per dimension, >= max(2, ng); 1 in dims >= ndim    */
  int32_t ng;       /* ghost layers stored per side in active dimensions, 2 <= ng <= 8, ng <= n;
                       or 0: no ghost storage (s = n), for a patch of a single-level table
                       whose faces are OUTFLOW, PERIODIC, REFLECT or EXTERNAL faces read
                       directly from one sibling of the same shape (see AMR_BC_EXTERNAL);
                       the stencil's two ghost layers per side are then never stored */
  int64_t offset;   /* element offset of variable 0 of this patch in the U arena       */
  int32_t bc[6];    /* AMR_BC_* of faces -x, +x, -y, +y, -z, +z                         */
  int32_t reserved[2]; /* must be 0                                                    */
} amr_patch_desc;

typedef struct {
  int32_t nvar;      /* conserved variables: 5 (hydro, Sec. 4), 8 (ideal MHD, psi = 0) or
                        9 (GLM-MHD: psi follows B)                                        */
  int32_t ndim;      /* 1, 2 or 3 active dimensions                                      */
  double gamma;      /* adiabatic index of p = (gamma-1) rho e, > 1                      */
  double theta;      /* PLM limiter parameter, 0 <= theta <= 2 (Sec. 4)                  */
  double dx0[3];     /* root-level cell widths, > 0                                      */
  int32_t flux;      /* AMR_FLUX_*                                                       */
  int32_t precision; /* AMR_PREC_*                                                       */
  int32_t exec;      /* AMR_EXEC_*                                                       */
  int32_t periodic;  /* bit d set: the root domain is periodic in d, so EXTERNAL ghost
                        cells beyond the domain wrap (needs domain[d])                   */
  int32_t domain[3]; /* root-level domain extent in cells per dimension (0 = not given)  */
  int32_t recon;     /* AMR_RECON_E (the paper's primitives) or AMR_RECON_P               */
  double rho_floor;  /* > 0: floor applied to recovered density (primitives only); 0 = off */
  double e_floor;    /* > 0: floor applied to recovered specific internal energy; 0 = off */
  double ch;         /* nvar 9: GLM cleaning speed c_h >= 0 (ignored otherwise)           */
} amr_physics;

typedef struct amr_table amr_table; /* opaque, library-owned */

/* Create a table for `npatch` patches (Sec. 3 hierarchy as a flat list).
 * Copies the descriptors, validates them (AMR_EINVAL on: npatch < 1, n < 1,
 * n < max(2, ng) or ng out of range in an active dimension, ng = 0 on a patch of a table with
 * several levels or with an EXTERNAL face that is not read from one same-shaped
 * sibling, n > 1 in an absent dimension,
 * overlapping storage, unknown bc/flux/precision/exec/recon, nvar not 5, 8 or 9,
 * ch negative or not finite,
 * gamma <= 1, theta outside [0,2], dx0 <= 0, a PERIODIC face whose opposite
 * face is not PERIODIC), allocates the device-side copy, the stage scratch
 * arena U^(1) (same size as the U arena) and the reduction/flag words, builds
 * the tile lists and selects the default tile shape.  Uses the current HIP
 * device; `stream` orders the uploads.  On success *out owns all of that until
 * amr_patch_table_destroy. */
amr_status amr_patch_table_create(const amr_patch_desc* patches, int32_t npatch, const amr_physics* phys,
                                  hipStream_t stream, amr_table** out);

/* Free everything the table owns (waits for the device to finish using it). */
amr_status amr_patch_table_destroy(amr_table* table);

/* Number of doubles the U arena must hold (max over patches of offset + nvar S). */
int64_t amr_table_arena_elems(const amr_table* table);

/* Global CFL time step (a rule the paper leaves unstated; the unsplit sum form
 * keeps 3D runs stable at cfl = 0.8): dt = cfl / max over active cells of
 * sum_d (|v_d| + c_s) / dx_d, with
 * c_s = sqrt(gamma p / rho), over the patches of `level` (-1 = all levels).
 * With several levels and level = -1 the root step of a factor-2 subcycled
 * hierarchy is returned: dt0 = cfl * min_l 2^l / smax_l.  The result is written
 * to dt_dev[0] (device, caller-owned).  If dt_host is not NULL the call waits
 * for the stream, copies the value there, and returns AMR_EUNPHYSICAL if the
 * device flag is set (the latch stays set: every later call with dt_host returns
 * AMR_EUNPHYSICAL until amr_table_status clears it).  The max is
 * order-independent, so the value is deterministic.  After a step with
 * AMR_STEP_FUSE_DT the first call on the same U and level reads the maxima that
 * step reduced instead of scanning U, unless amr_table_status was called in
 * between; any later call scans U again.
 * Recovery (from AMR_EUNPHYSICAL, or any rejected step): amr_table_status (clears
 * the latch and the fused maxima), restore U^n, amr_cfl_dt (a fresh scan of U^n),
 * then retry with a smaller dt. */
amr_status amr_cfl_dt(amr_table* table, const double* U, double cfl, int32_t level, double* dt_dev,
                      double* dt_host, hipStream_t stream);

/* One TVD-RK2 step (Sec. 4, RK2 equation) of the patches of `level` (-1 = all),
 * in place:  U^(1) = U^n + dt L(U^n) (into the table's scratch arena), then
 * U^{n+1} = U^n/2 + (U^(1) + dt L(U^(1)))/2 written over U^n.  dt is read from
 * dt_dev[0] on the device when the step runs (so a captured step replays with
 * new values).  EXTERNAL ghosts of the stage input are filled before each
 * stage.  flags: AMR_STEP_*.  Asynchronous.
 * Tables with several levels: `level` must name one level (-1 and
 * AMR_STEP_FUSE_DT give AMR_EINVAL).  Such a step is one node of the subcycled
 * recursion amr_hydro_advance runs: the patches of a level > 0 record their
 * coarse/fine face fluxes into the flux registers, a level with children keeps
 * U^n as the snapshot its children's ghosts interpolate from and clears their
 * registers, and AMR_STEP_SUBSTEP1 marks the second of a parent step's two
 * substeps.  A driver of its own calls, for level l: this step, then (if l has
 * children) the same recursion for l+1 twice (the second with
 * AMR_STEP_SUBSTEP1), then amr_flux_correct(l); dt_dev[0] = dt0 / 2^l. */
amr_status amr_hydro_rk2_step(amr_table* table, double* U, const double* dt_dev, int32_t level, uint32_t flags,
                              hipStream_t stream);

/* Coarse/fine flux correction and restriction for `coarse_level` (Berger &
 * Colella refluxing; the paper's hierarchy, Sec. 3, is Berger & Colella AMR):
 * every coarse cell next to a level coarse_level+1 patch and not covered by one
 * replaces its own interface flux by the average of the fine fluxes recorded over
 * the fine level's two steps, U_c += s (R_c - <R_f>) / dx_c (R = dt/2 per RK2
 * stage, s = +1 where the interface is the cell's high face); then every covered
 * coarse cell becomes the mean of its 2^ndim children.  Call after the coarse
 * level's step and its children's two steps.  AMR_ESTATE if the level has no
 * children or has not stepped. */
amr_status amr_flux_correct(amr_table* table, double* U, int32_t coarse_level, hipStream_t stream);

/* One root step of the whole hierarchy (factor-2 refinement in space and time,
 * Sec. 3): level l advances with dt0 / 2^l; after a level's step its children take
 * two steps, whose EXTERNAL ghosts not held by a sibling are prolonged
 * (conservative, minmod-limited linear) from the parent interpolated linearly in
 * time, then the level is flux-corrected and restricted.  dt0 is read from
 * dt0_dev[0] (e.g. amr_cfl_dt with level -1).  flags must be 0.  For a
 * single-level table this is amr_hydro_rk2_step of all patches.  Batched tables
 * replay the whole root step from one captured HIP graph.  Asynchronous. */
amr_status amr_hydro_advance(amr_table* table, double* U, const double* dt0_dev, uint32_t flags,
                             hipStream_t stream);

/* Wait for `stream`, then return AMR_EUNPHYSICAL if any kernel latched an
 * unphysical state since the table was created or last cleared, else AMR_OK.
 * Clears the latch, and drops the maxima fused into the last step (the next
 * amr_cfl_dt scans U, which the caller may have rewritten since). */
amr_status amr_table_status(amr_table* table, hipStream_t stream);

/* Tile shape control (batched and plain forms share the kernels).
 * amr_table_num_tilings: number of compiled tile shapes.
 * amr_table_set_tiling: select shape `id` (0 <= id < num) and z-slab length
 *   zslab (>= 1; 0 = automatic: the slab length that fills whole rounds of the
 *   persistent launch); invalidates a captured graph.  AMR_EINVAL for a shape
 *   the table cannot run: shape 0 is the 1D shape and the only one for ndim 1;
 *   MHD tables (nvar 8 and 9) have shapes 0, 1 and 4, and 5 and 6 in mixed precision
 *   (in FP64 the larger tiles' LDS does not hold eight variables).
 * amr_table_get_tiling: current id and (resolved) zslab.
 * amr_table_tiling_shape: the (TX, TY) cells per tile of shape `id`. */
int32_t amr_table_num_tilings(const amr_table* table);
amr_status amr_table_set_tiling(amr_table* table, int32_t id, int32_t zslab);
amr_status amr_table_get_tiling(amr_table* table, int32_t* id, int32_t* zslab);
amr_status amr_table_tiling_shape(const amr_table* table, int32_t id, int32_t* tx, int32_t* ty);

/* Autotuner: time every (shape, zslab) candidate on the caller's data with
 * HIP events (each candidate runs `reps` full RK2 steps of `level` on a copy of
 * U in a temporary device buffer of amr_table_arena_elems doubles that the call
 * allocates and frees, so U is not modified), keep the fastest (it stays the
 * table's tiling until amr_table_set_tiling), and return its time per step in
 * *ms_best (nullable).  Synchronises the stream.  The unphysical latch is left as
 * it was before the call.  Tables with several levels: `level` must name one
 * level (AMR_EINVAL otherwise), and AMR_ESTATE is returned while a caller-driven
 * recursion is open (a level with children has stepped and its amr_flux_correct
 * is still due), because the candidates reuse the snapshot, U^(1) and the flux
 * registers that recursion needs.  AMR_ENOMEM if the copy cannot be allocated. */
amr_status amr_autotune(amr_table* table, const double* U, const double* dt_dev, int32_t level, int32_t reps,
                        hipStream_t stream, float* ms_best);

/* Durations of the two stage kernels of the last AMR_STEP_TIMED step (in ms,
 * from HIP events on the step's stream around each stage's launches, so the
 * ghost fill of the stage 2 input is in neither; summed over launches in the
 * plain form).  Waits for that step.  AMR_ESTATE if no timed step was run. */
amr_status amr_table_last_stage_ms(amr_table* table, float ms[2]);

/* Refinement flags (the steps beside the update that build a dynamic hierarchy; the
 * paper does this on the host, Sec. 3).
 * amr_table_cells: active cells of `level` (-1 = all levels), -1 for a bad argument.
 * amr_flag_cells: one byte per active cell of `level` (-1 = all) into flags_dev (device
 *   memory of amr_table_cells(level) bytes), patches in table order, cells x fastest:
 *   1 where the density jumps by more than eps relative to the smaller value,
 *   |rho_n - rho_c| / min(rho_n, rho_c) > eps, to a face neighbour n, else 0 (the
 *   criterion that places the deep-AMR configuration's levels).  Neighbours across
 *   patch faces follow the boundary conditions; EXTERNAL ghosts of the flagged level
 *   and of every coarser level are refilled first from U's current state (this
 *   writes U's EXTERNAL ghost storage, as a step does).  AMR_EINVAL for null
 *   pointers, a level out of range or a negative eps.  Asynchronous. */
int64_t amr_table_cells(const amr_table* table, int32_t level);
amr_status amr_flag_cells(amr_table* table, double* U, int32_t level, double eps, uint8_t* flags_dev,
                          hipStream_t stream);

/* Fill the active cells of U (arena of `table`, a new hierarchy) from U_old (arena of
 * old_table, the hierarchy it replaces): level by level from the root, a cell that an
 * old patch of the same level holds is copied, any other is prolonged (conservative,
 * minmod-limited linear, as for ghost cells) from the new level below, whose ghosts are
 * filled first.  The root level must be covered by the old root patches, and every new
 * box to be prolonged must lie in one patch of the level below (proper nesting).  Same
 * nvar and ndim in both tables.  Synchronises
 * `stream` (the op lists are temporary device memory).  AMR_EINVAL otherwise. */
amr_status amr_regrid_fill(const amr_table* old_table, const double* U_old, amr_table* table, double* U,
                           hipStream_t stream);

/* Host-side clustering of the flags of level `level` (host bytes, the layout of
 * amr_flag_cells for the patches of that level in the given descriptor order) into the
 * boxes of level `level`+1 (refinement 2), written to boxes[6 i .. 6 i + 5] = lo[3], n[3]
 * in level+1 index space, sorted by lo then extent; *nboxes receives their count.  Each
 * flagged cell, dilated by one cell along each axis, marks the fine bricks (brick^3
 * fine cells, aligned) holding its children; a marked brick is kept when its level-l
 * footprint dilated by one coarse cell (clipped to the root domain `domain` << level)
 * lies on level l (proper nesting); kept bricks are grouped per aligned block^3 fine
 * block into the group's bounding box if that box is nested, else into half-block
 * bounding boxes, else single bricks.  Requires brick-aligned level-l patches, block a
 * multiple of 2 brick.  AMR_EINVAL for bad arguments or more boxes than max_boxes (then
 * *nboxes is the number needed).  No device work. */
amr_status amr_cluster_flags(const amr_patch_desc* patches, int32_t npatch, int32_t ndim, const int32_t domain[3],
                             int32_t level, const uint8_t* flags, int32_t brick, int32_t block, int32_t* boxes,
                             int32_t max_boxes, int32_t* nboxes);

/* Allocation-free RK2 step of one patch, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same update and same bits as amr_hydro_rk2_step on a single-level table
 * made of this one patch (any precision; the persistent launch of the batched form,
 * enqueued eagerly), with no table: the patch descriptor, its tile list and the
 * stage output U^(1) live in a device array of AMR_NOALLOC_SCRATCH_BYTES that the
 * library holds on each GPU it runs on until the process ends.  The call allocates
 * nothing and copies nothing from the host; it enqueues three kernels on `stream`.
 *   patch   host descriptor: level 0, bc OUTFLOW, PERIODIC or REFLECT on every face
 *           (no EXTERNAL face: a lone patch has no source for it), other rules as in
 *           amr_patch_table_create; phys as there (exec is ignored).
 *   U       caller-owned device arena holding the patch at patch->offset; U^n in,
 *           U^{n+1} out.
 *   dt_dev  caller-owned device double, read when the step runs.
 *   flag_dev caller-owned device int32, set nonzero (never cleared) if the step meets
 *           an unphysical state (the table's latch).
 * AMR_EINVAL (nothing enqueued) for a bad argument, an EXTERNAL face, a level other
 * than 0, or a patch whose U^(1) (nvar doubles per active cell) plus its tile list
 * exceed the scratch (e.g. 5 variables of 144^3 active cells fit, 8 variables of
 * 128^3 do not);
 * the last case also prints the bytes needed to stderr.  Every call on one GPU shares
 * that GPU's scratch: calls that overlap on one GPU (other streams, other host
 * threads) race and must be serialised by the caller. */
#define AMR_NOALLOC_SCRATCH_BYTES (134217728ull) /* 128 MiB per GPU */
amr_status amr_patch_rk2_step_noalloc(const amr_patch_desc* patch, const amr_physics* phys, double* U,
                                      const double* dt_dev, int32_t* flag_dev, hipStream_t stream);

/* Streaming ceiling, a measurement aid beside the update (not a step of it): out[i] =
 * (a[i] + b[i]) / 2 for i < n, the HBM access pattern of the second RK stage (Sec. 4,
 * RK2 combine: two arrays read, one written, each element once) with no other work, in
 * one launch on `stream` (plus one for an odd last element).  Its bandwidth, 24 n bytes
 * over its duration, is the practical ceiling the stage kernels' bandwidth is compared
 * with.  a, b, out: caller-owned device arrays of n doubles, 16-byte aligned, out not
 * overlapping a or b.  wg_per_cu: 0 = one workgroup per 2048 elements (a single pass),
 * else a persistent grid of that many 256-lane workgroups per CU (at most 64).
 * AMR_EINVAL for null or misaligned pointers, n < 1 or wg_per_cu out of range. */
amr_status amr_stream_ceiling(const double* a, const double* b, double* out, int64_t n, int32_t wg_per_cu,
                              hipStream_t stream);

const char* amr_status_string(amr_status status);

#ifdef __cplusplus
}
#endif
#endif /* AMR_HYDRO_H */
