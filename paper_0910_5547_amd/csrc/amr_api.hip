// amr_api.hip - host side of the C ABI declared in include/amr_hydro.h.
//
// The table owns: the validated descriptors and their device copy, the stage
// scratch arena U^(1), the unphysical-state latch and the per-level
// signal-speed maxima, the tile lists of every (level scope, tile shape,
// z-slab) in use, the EXTERNAL ghost copy plan, and the captured HIP graph of
// the batched RK2 step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <tuple>
#include <unordered_set>
#include <vector>

#include "../../include/amr_hydro.h"
#include "amr_internal.h"

using namespace amr;

namespace amr {

amr_status validate_patches(const amr_patch_desc* P, int32_t np, const amr_physics* ph) {
  if (!P || !ph || np < 1) return AMR_EINVAL;
  if ((ph->nvar != NVAR && ph->nvar != NVAR_MHD && ph->nvar != NVAR_GLM) || ph->ndim < 1 || ph->ndim > 3)
    return AMR_EINVAL;
  if (!(ph->ch >= 0.0 && ph->ch < 1e300)) return AMR_EINVAL;
  if (!(ph->gamma > 1.0) || !(ph->theta >= 0.0 && ph->theta <= 2.0)) return AMR_EINVAL;
  for (int d = 0; d < 3; ++d)
    if (!(ph->dx0[d] > 0)) return AMR_EINVAL;
  if (ph->flux != AMR_FLUX_PAPER && ph->flux != AMR_FLUX_HLL2) return AMR_EINVAL;
  if (ph->precision != AMR_PREC_FP64 && ph->precision != AMR_PREC_MIXED) return AMR_EINVAL;
  if (ph->exec != AMR_EXEC_PLAIN && ph->exec != AMR_EXEC_BATCHED) return AMR_EINVAL;
  if ((ph->recon != AMR_RECON_E && ph->recon != AMR_RECON_P) || ph->periodic < 0 || ph->periodic > 7)
    return AMR_EINVAL;
  for (int d = 0; d < 3; ++d)
    if (((ph->periodic >> d) & 1) && ph->domain[d] < 1) return AMR_EINVAL;
  if (ph->rho_floor < 0 || ph->e_floor < 0) return AMR_EINVAL;
  std::vector<std::pair<int64_t, int64_t>> spans;
  for (int p = 0; p < np; ++p) {
    const amr_patch_desc& D = P[p];
    if (D.level < 0 || D.level >= MAX_LEVELS || D.offset < 0 || D.reserved[0] || D.reserved[1]) return AMR_EINVAL;
    // ng 0: no ghost storage (faces applied by index maps or read from direct siblings;
    // the table checks that no face needs stored ghosts)
    if (D.ng != 0 && (D.ng < 2 || D.ng > 8)) return AMR_EINVAL;
    int64_t S = 1;
    for (int d = 0; d < 3; ++d) {
      if (D.n[d] < 1) return AMR_EINVAL;
      if (d >= ph->ndim && D.n[d] != 1) return AMR_EINVAL;
      // (two cells at least: the boundary maps of the two-cell stencil stay in the patch)
      if (d < ph->ndim && D.n[d] < std::max(2, D.ng)) return AMR_EINVAL;
      if (D.n[d] > (1 << 24)) return AMR_EINVAL;
      S *= D.n[d] + (d < ph->ndim ? 2 * D.ng : 0);
      for (int s = 0; s < 2; ++s) {
        const int b = D.bc[2 * d + s];
        if (b < AMR_BC_OUTFLOW || b > AMR_BC_EXTERNAL) return AMR_EINVAL;
      }
      if (d < ph->ndim && ((D.bc[2 * d] == AMR_BC_PERIODIC) != (D.bc[2 * d + 1] == AMR_BC_PERIODIC)))
        return AMR_EINVAL;
    }
    spans.emplace_back(D.offset, D.offset + ph->nvar * S);
  }
  std::sort(spans.begin(), spans.end());
  for (size_t i = 1; i < spans.size(); ++i)
    if (spans[i].first < spans[i - 1].second) return AMR_EINVAL;
  return AMR_OK;
}

Consts consts_of_phys(const amr_physics& ph) {
  Consts c{};
  c.gamma = ph.gamma;
  c.gm1 = ph.gamma - 1.0;
  c.gg1 = ph.gamma * (ph.gamma - 1.0);
  c.theta = ph.theta;
  c.rho_floor = ph.rho_floor;
  c.e_floor = ph.e_floor;
  c.ndim = ph.ndim;
  c.flux = ph.flux;
  c.recon = ph.recon;
  c.ch = ph.nvar == NVAR_GLM ? ph.ch : 0.0;
  c.ch2 = c.ch * c.ch;
  return c;
}

}  // namespace amr

namespace {

struct TileSet {
  Tile* d = nullptr;
  int n = 0;
  std::vector<int> first, count;  // per patch (plain form): range in the list
};

struct GraphCache {
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  const double* U = nullptr;
  const double* dt = nullptr;
  int level = -2, shape = -1, zslab = -1;
  uint32_t flags = 0;
};

// A work list: its workgroups' segment ranges start at blk_d + blk_base.
struct WorkList {
  int blk_base = 0, nblk = 0;
};

// The patches of a level scope and the prefix sums of their active cells (flagging).
struct CellList {
  int* plist = nullptr;
  int64_t* cofs = nullptr;
  int npl = 0;
  int64_t ncells = 0;
};

}  // namespace

struct amr_table {
  int device = 0;
  int ncu = 0;
  amr_physics ph{};
  std::vector<amr_patch_desc> desc;
  std::vector<PatchDev> pdev;
  PatchDev* pdev_d = nullptr;
  int64_t arena = 0;
  int64_t arena1 = 0;  // doubles of the stage scratch U^(1) (its own layout, PatchDev::off1)
  int max_level = 0;
  // direct sibling faces found by the ghost plan: source patch and shift per face
  std::vector<int> dsrc;
  std::vector<int> dsh;
  double* U1 = nullptr;
  int* flag_d = nullptr;
  unsigned long long* smax_d = nullptr;  // [MAX_LEVELS + 1] scan maxima
  unsigned long long* fused_d = nullptr; // [MAX_LEVELS + 1] maxima fused into stage 2
  // EXTERNAL ghost plan: ops sorted by destination level; level_first/count index it
  CopyOp* ops_d = nullptr;
  int nops = 0;
  std::vector<int> ops_level_first, ops_level_count;
  int shape = 1, zslab = 0;
  std::map<std::tuple<int, int, int>, TileSet> tiles;  // (level scope, shape, zslab)
  GraphCache gc;
  hipStream_t cap_stream = nullptr;
  // fused dt bookkeeping: the U and level whose maxima stage 2 reduced into fused_d,
  // valid until amr_cfl_dt reads them or the unphysical latch is found set
  const double* fused_U = nullptr;
  int fused_level = -2;
  // caller-driven recursion: bit l is set by a step of level l that has children and
  // cleared by amr_flux_correct(l) (the snapshot, U^(1) and registers are in use)
  uint32_t open_mask = 0;
  // bit l (l > 0): level l's first substep of its parent's current step has been
  // enqueued, so its U^(1) holds the half-step prolonged ghosts the second reuses
  uint32_t half_mask = 0;
  int occ[3][2][NSHAPES][2][2] = {};  // resident stage workgroups per CU: [5/8/9 variables][mixed][shape][stage][recording]
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};  // AMR_STEP_TIMED: around each stage kernel
  bool timed_valid = false;
  // ---- hierarchy (levels > 0 present): coarse/fine coupling plans, see build_hierarchy
  std::vector<char> has_kids;                   // per level: a finer level exists
  double* snap = nullptr;                       // U^n of levels with children (same layout as U)
  double* reg = nullptr;                        // fine-face flux registers
  double* dtl = nullptr;                        // per-level dt of the subcycled root step
  std::vector<int64_t> reg_first, reg_len;      // per level, for clearing
  ProlongOp* prol_d = nullptr;
  CopyOp* pcp_d = nullptr;                      // the prolongation boxes as same-cell copies (U^(1) -> U)
  std::vector<int> prol_first, prol_count;      // per destination level
  PhysOp* phys_d = nullptr;
  std::vector<int> phys_first, phys_count;      // per level with children
  FixOp* fix_d = nullptr;
  std::vector<std::vector<std::pair<int, int>>> fix_colors;  // per coarse level: (first, count) per color
  RestrictOp* rst_d = nullptr;
  std::vector<int> rst_first, rst_count;        // per coarse level
  CopyOp* snap_d = nullptr;                     // snapshot boxes (dst = src = the coarse patch)
  std::vector<int> snap_first, snap_count;      // per level
  std::vector<WorkList> w_snap;
  std::vector<const double*> last_dt;           // dt pointer of each level's last step
  GraphCache gadv;                              // captured root step (batched form)
  // cell-granular work lists of the box-op kernels (see Seg): per level, and for
  // the refluxing ops per coarse level and colour
  Seg* segs_d = nullptr;
  int* blk_d = nullptr;
  std::vector<WorkList> w_copy, w_prol, w_phys, w_rst;
  std::vector<std::vector<WorkList>> w_fix;
  std::map<int, CellList> cell_lists;           // per level scope (-1 = all), built on first use
};

#define HIPCHECK(x)                                     \
  do {                                                  \
    hipError_t _e = (x);                                \
    if (_e != hipSuccess) {                             \
      fprintf(stderr, "amr_hydro: %s failed: %s\n", #x, \
              hipGetErrorString(_e));                   \
      return AMR_EHIP;                                  \
    }                                                   \
  } while (0)

namespace {

bool shape_valid(int ndim, int shape) {
  if (shape < 0 || shape >= NSHAPES) return false;
  return ndim == 1 ? shape == 0 : shape != 0;
}

// A shape this table can run: right for its dimensionality and compiled for its
// variable count and precision.
bool shape_ok(const amr_table* t, int shape) {
  if (!shape_valid(t->ph.ndim, shape)) return false;
  return t->ph.nvar == NVAR || mhd_shape_ok(t->ph.precision == AMR_PREC_MIXED, shape);
}

int occupancy_grid(amr_table* t, int stage, int ntiles, bool rec);

// z-slab length that balances the persistent launch: per-tile time is taken as
// proportional to its planes + 4 (the z prologue reads 4 planes); with T_xy column
// blocks of the level scope and G resident workgroups, choose the slab count that
// minimises rounds x (slab + 4).  Levels with enough tiles keep whole patches.
int auto_zslab(amr_table* t, int level, int shape) {
  if (t->ph.ndim != 3) return 1;
  int64_t txy = 0;
  int nz = 1;
  for (const PatchDev& P : t->pdev) {
    if (level >= 0 && P.level != level) continue;
    int TX, TY;
    tile_dims(shape, P.n[0], TX, TY);
    txy += (int64_t)((P.n[0] + TX - 1) / TX) * ((P.n[1] + TY - 1) / TY);
    nz = std::max(nz, P.n[2]);
  }
  const int keep = t->shape;
  t->shape = shape;
  const bool rec = level > 0 && t->reg != nullptr;
  // tiles in flight, counted at no more than two workgroups per CU: beyond that the
  // co-resident tiles' halo rows (the neighbours' interiors) no longer stay in the
  // XCD's L2 between the two reads (on the 256^3 box two slabs of 128 planes beat
  // three of 86 although three fill every resident slot)
  const int64_t G = (int64_t)std::min(occupancy_grid(t, 2, 1 << 30, rec), 2 * t->ncu) * shape_tiles_per_wg(shape);
  t->shape = keep;
  return balanced_zslab(txy, nz, G);
}

int default_zslab(const amr_table* t) { return t->ph.ndim == 3 ? 0 : 1; }  // 0 = auto_zslab

// Default tile shape: 32 x 16 tiles (512 threads) where they are nearly full (the
// smallest halo share per cell), else 32 x 8, unless small patches would leave more
// than half of those lanes idle; then 8 x 8 wavefront tiles, which fill every lane
// of patches whose x-y extents are multiples of 8 (their larger halo share makes
// them slower where the workgroup tiles are at least half full).
int default_shape(const amr_table* t) {
  if (t->ph.ndim == 1) return 0;
  auto lane_use = [&](int shape) {
    double cols = 0, lanes = 0;
    for (const PatchDev& P : t->pdev) {
      int TX, TY;
      tile_dims(shape, P.n[0], TX, TY);
      cols += (double)P.n[0] * P.n[1] * P.n[2];
      lanes += (double)((P.n[0] + TX - 1) / TX) * ((P.n[1] + TY - 1) / TY) * TX * TY * P.n[2];
    }
    return cols / lanes;
  };
  const double u1 = lane_use(1), us = lane_use(SHAPE_SMALL);
  // 32 x 16 where those tiles are nearly full (one barrier per plane; for MHD only in
  // mixed precision, the FP64 eight-variable tile not fitting in LDS)
  if (t->ph.ndim == 3 && (t->ph.nvar == NVAR || t->ph.precision == AMR_PREC_MIXED) && lane_use(5) >= 0.9) return 5;
  return (u1 < 0.5 && us > u1) ? SHAPE_SMALL : 1;
}

// Tile list of the patches of `level` (-1 = all) for a shape and z-slab length.
amr_status get_tiles(amr_table* t, int level, int shape, int zslab, TileSet** out) {
  if (zslab == 0) zslab = auto_zslab(t, level, shape);
  auto key = std::make_tuple(level, shape, zslab);
  auto it = t->tiles.find(key);
  if (it != t->tiles.end()) {
    *out = &it->second;
    return AMR_OK;
  }
  std::vector<Tile> list;
  TileSet ts;
  ts.first.assign(t->pdev.size(), 0);
  ts.count.assign(t->pdev.size(), 0);
  for (size_t p = 0; p < t->pdev.size(); ++p) {
    const PatchDev& P = t->pdev[p];
    ts.first[p] = (int)list.size();
    if (level >= 0 && P.level != level) continue;
    int TX, TY;
    tile_dims(shape, P.n[0], TX, TY);
    const int zs = std::min(zslab, P.n[2]);
    for (int z0 = 0; z0 < P.n[2]; z0 += zs)
      for (int y0 = 0; y0 < P.n[1]; y0 += TY)
        for (int x0 = 0; x0 < P.n[0]; x0 += TX) {
          Tile T{};
          T.patch = (int)p;
          T.x0 = x0;
          T.y0 = y0;
          T.z0 = z0;
          T.z1 = std::min(z0 + zs, P.n[2]);
          T.tx = TX;
          list.push_back(T);
        }
    ts.count[p] = (int)list.size() - ts.first[p];
  }
  ts.n = (int)list.size();
  if (ts.n > 0) {
    // The batched form's persistent workgroup b runs on XCD b % 8 (the dispatcher
    // deals workgroups round-robin over the 8 XCDs) and walks groups b, b+G, ... of
    // W consecutive positions (W tiles per workgroup; G, the grid, is a multiple of
    // 8).  Split the list - in patch, z-slab, y, x order - into 8 contiguous chunks
    // of equal cost and interleave them group by group, so that every XCD works on
    // one compact region and a tile's halo is its neighbours' interior in the same
    // L2.  Within a chunk, longer tiles go first (LPT) so the workgroups finish
    // together; equal-cost tiles keep their spatial order.  The plain form uses the
    // per-patch ranges of the unsorted list, kept as a second copy at the end of
    // the same buffer.
    const int NX = 8;
    auto cost = [](const Tile& a) { return (int64_t)(a.z1 - a.z0) + 2; };
    int64_t total = 0;
    for (const Tile& a : list) total += cost(a);
    std::vector<std::vector<Tile>> chunk(NX);
    int64_t acc = 0;
    for (const Tile& a : list) {
      const int c = (int)std::min<int64_t>(NX - 1, acc * NX / std::max<int64_t>(total, 1));
      chunk[c].push_back(a);
      acc += cost(a);
    }
    size_t longest = 0;
    for (auto& c : chunk) {
      std::stable_sort(c.begin(), c.end(), [&](const Tile& a, const Tile& b) { return cost(a) > cost(b); });
      longest = std::max(longest, c.size());
    }
    const size_t W = (size_t)shape_tiles_per_wg(shape);
    std::vector<Tile> sorted;
    sorted.reserve(list.size());
    for (size_t m = 0; m < longest; m += W)
      for (int c = 0; c < NX; ++c)
        for (size_t q = m; q < std::min(m + W, chunk[c].size()); ++q) sorted.push_back(chunk[c][q]);
    std::vector<Tile> both = sorted;
    both.insert(both.end(), list.begin(), list.end());
    if (hipMalloc(&ts.d, sizeof(Tile) * both.size()) != hipSuccess) return AMR_ENOMEM;
    HIPCHECK(hipMemcpy(ts.d, both.data(), sizeof(Tile) * both.size(), hipMemcpyHostToDevice));
  }
  auto res = t->tiles.emplace(key, std::move(ts));
  *out = &res.first->second;
  return AMR_OK;
}

Consts consts_of(const amr_table* t) { return consts_of_phys(t->ph); }

// Resident workgroups per CU of the stage kernel in use (queried once per
// (precision, shape, stage, recording), outside any graph capture); the grid of a
// persistent launch, no larger than what is resident at once.
int occupancy_grid(amr_table* t, int stage, int ntiles, bool rec) {
  if (ntiles < 1) ntiles = 1;
  const int mixed = t->ph.precision == AMR_PREC_MIXED;
  const int vk = t->ph.nvar == NVAR_MHD ? 1 : t->ph.nvar == NVAR_GLM ? 2 : 0;
  int& per_cu = t->occ[vk][mixed][t->shape][stage - 1][rec ? 1 : 0];
  if (per_cu <= 0) {
    const void* k = stage_kernel_ptr(t->ph.nvar, mixed, t->shape, stage, rec);
    if (!k) {  // not compiled for this shape: never launched, nothing to size
      per_cu = 1;
    } else if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, SHAPE_NT[t->shape], 0) != hipSuccess ||
               per_cu < 1) {
      per_cu = 1;
    }
  }
  const int g = std::max(1, std::min(ntiles, per_cu * t->ncu));
  return g >= 8 ? g / 8 * 8 : g;  // a multiple of the XCD count (tile list interleave)
}

// Enqueue the EXTERNAL ghost fill of arena A for the patches of `level`: sibling
// copies, then (levels > 0) prolongation from the coarse level interpolated in time
// between its snapshot and its state in U at fraction alpha.
Work work_of(const amr_table* t, const WorkList& w) { return Work{t->segs_d, t->blk_d + w.blk_base, w.nblk, 0}; }

// The prolonged ghosts: computed (PROL_COMPUTE), copied from the same ghost cells of
// U^(1), which hold them at this alpha already (PROL_FROM_U1), or left as they are
// (PROL_KEEP: A holds them at this alpha).
enum { PROL_COMPUTE = 0, PROL_FROM_U1 = 1, PROL_KEEP = 2 };

amr_status enqueue_ghosts(amr_table* t, double* A, const double* U, int level, double alpha, hipStream_t s,
                          const double* Cold = nullptr, int prol = PROL_COMPUTE) {
  const int l0 = level < 0 ? 0 : level, l1 = level < 0 ? t->max_level : level;
  for (int l = l0; l <= l1; ++l)
    if (t->w_copy[l].nblk > 0)
      HIPCHECK(launch_copy_ghosts(s, t->ops_d + t->ops_level_first[l], work_of(t, t->w_copy[l]), t->pdev_d, A,
                                  t->ph.nvar));
  if (level > 0 && t->w_prol[level].nblk > 0) {
    if (prol == PROL_COMPUTE)
      HIPCHECK(launch_prolong(s, t->prol_d + t->prol_first[level], work_of(t, t->w_prol[level]), t->pdev_d, A,
                              Cold ? Cold : t->snap, U, alpha, t->ph.ndim, t->ph.nvar));
    else if (prol == PROL_FROM_U1)
      HIPCHECK(launch_copy_cells_x(s, t->pcp_d + t->prol_first[level], work_of(t, t->w_prol[level]), t->pdev_d,
                                   t->pdev_d, A, t->U1, t->ph.nvar));
  }
  return AMR_OK;
}

// One stage kernel launch (or one per patch in the plain form) over `level`.
amr_status enqueue_stage(amr_table* t, TileSet* ts, int stage, const double* V, const double* U0, double* out,
                         const double* dt, bool fuse, bool rec, hipStream_t s) {
  const int mixed = t->ph.precision == AMR_PREC_MIXED;
  StageArgs a{};
  a.V = V;
  a.U0 = U0;
  a.out = out;
  a.dt = dt;
  a.patches = t->pdev_d;
  a.flag = t->flag_d;
  a.smax = (stage == 2 && fuse) ? t->fused_d : nullptr;
  a.reg = rec ? t->reg : nullptr;
  a.c = consts_of(t);
  const int W = shape_tiles_per_wg(t->shape);
  if (t->ph.exec == AMR_EXEC_BATCHED) {
    a.tiles = ts->d;
    a.ntiles = ts->n;
    HIPCHECK(launch_stage(t->ph.nvar, mixed, t->shape, stage, occupancy_grid(t, stage, (ts->n + W - 1) / W, rec), s,
                          a));
  } else {
    for (size_t p = 0; p < t->pdev.size(); ++p) {
      if (ts->count[p] == 0) continue;
      a.tiles = ts->d + ts->n + ts->first[p];
      a.ntiles = ts->count[p];
      HIPCHECK(launch_stage(t->ph.nvar, mixed, t->shape, stage, (ts->count[p] + W - 1) / W, s, a));
    }
  }
  return AMR_OK;
}

// Enqueue one RK2 step (both stages) of `level` on stream s.  `substep` (0 or 1) is
// the step's position inside its parent level's step: the coarse data of its
// prolonged ghosts is taken at parent-time fractions substep/2 (stage 1 input) and
// (substep+1)/2 (stage 2 input).  A level with children also writes its physical
// ghosts into storage, keeps U^n (the snapshot its children interpolate from),
// refills U^{n+1}'s ghosts and clears its children's registers.  With `ev`, record
// ev[0] and ev[1] around the stage 1 kernel, ev[2] and ev[3] around the stage 2 kernel
// (the ghost fill of stage 2's input lies between ev[1] and ev[2]).
amr_status enqueue_step(amr_table* t, double* U, const double* dt, int level, uint32_t flags, hipStream_t s,
                        hipEvent_t* ev = nullptr, int substep = 0) {
  TileSet* ts = nullptr;
  amr_status st = get_tiles(t, level, t->shape, t->zslab, &ts);
  if (st != AMR_OK) return st;
  if (ts->n == 0) return AMR_OK;
  const bool fuse = (flags & AMR_STEP_FUSE_DT) != 0;
  const bool kids = level >= 0 && t->has_kids[level];
  const bool rec = level > 0 && t->reg != nullptr;
  const double a1 = 0.5 * substep, a2 = 0.5 * (substep + 1);
  if (fuse) HIPCHECK(launch_fill_u64(s, t->fused_d, MAX_LEVELS + 1, 0ull));
  // The second substep's first stage takes its prolonged ghosts at time 1/2 of the parent
  // step, as the first substep's second stage did into U^(1): a level with children
  // copied them into U at the end of that step already; a level without copies them now.
  const int prol1 = (level > 0 && substep == 1) ? (kids ? PROL_KEEP : PROL_FROM_U1) : PROL_COMPUTE;
  st = enqueue_ghosts(t, U, U, level, a1, s, nullptr, prol1);
  if (st != AMR_OK) return st;
  if (kids) {
    if (t->w_phys[level].nblk > 0)
      HIPCHECK(launch_phys(s, t->phys_d + t->phys_first[level], work_of(t, t->w_phys[level]), t->pdev_d, U,
                                 t->ph.nvar));
    if (t->w_snap[level].nblk > 0)
      HIPCHECK(launch_copy_cells_x(s, t->snap_d + t->snap_first[level], work_of(t, t->w_snap[level]), t->pdev_d,
                                   t->pdev_d, t->snap, U, t->ph.nvar));
  }
  if (ev) HIPCHECK(hipEventRecord(ev[0], s));
  st = enqueue_stage(t, ts, 1, U, nullptr, t->U1, dt, fuse, rec, s);
  if (st != AMR_OK) return st;
  if (ev) HIPCHECK(hipEventRecord(ev[1], s));
  st = enqueue_ghosts(t, t->U1, U, level, a2, s);
  if (st != AMR_OK) return st;
  if (ev) HIPCHECK(hipEventRecord(ev[2], s));
  st = enqueue_stage(t, ts, 2, t->U1, U, U, dt, fuse, rec, s);
  if (st != AMR_OK) return st;
  if (ev) HIPCHECK(hipEventRecord(ev[3], s));
  if (kids) {
    // U^{n+1}'s ghosts for the children's stencils: the prolonged ones equal those of U^(1)
    st = enqueue_ghosts(t, U, U, level, a2, s, nullptr, PROL_FROM_U1);
    if (st != AMR_OK) return st;
    if (t->w_phys[level].nblk > 0)
      HIPCHECK(launch_phys(s, t->phys_d + t->phys_first[level], work_of(t, t->w_phys[level]), t->pdev_d, U,
                                 t->ph.nvar));
    const int64_t len = t->reg_len[level + 1];
    if (len > 0) {
      for (int64_t o = 0; o < len; o += (int64_t)1 << 30)
        HIPCHECK(launch_fill_u64(s, reinterpret_cast<unsigned long long*>(t->reg + t->reg_first[level + 1] + o),
                                 (int)std::min<int64_t>(len - o, (int64_t)1 << 30), 0ull));
    }
  }
  if (level >= 0) t->last_dt[level] = dt;
  return AMR_OK;
}

// Refluxing of `l` against level l+1, then restriction of the covered cells.
amr_status enqueue_correct(amr_table* t, double* U, int l, hipStream_t s) {
  const int mixed = t->ph.precision == AMR_PREC_MIXED;
  for (size_t c = 0; c < t->fix_colors[l].size(); ++c)
    if (t->w_fix[l][c].nblk > 0)
      HIPCHECK(launch_flux_fix(mixed, t->ph.nvar, s, t->fix_d + t->fix_colors[l][c].first,
                               work_of(t, t->w_fix[l][c]), t->pdev_d, U, t->snap, t->U1, t->reg, t->last_dt[l],
                               consts_of(t), t->flag_d));
  if (t->w_rst[l].nblk > 0)
    HIPCHECK(launch_restrict(s, t->rst_d + t->rst_first[l], work_of(t, t->w_rst[l]), t->pdev_d, U, t->ph.ndim,
                             t->ph.nvar));
  return AMR_OK;
}

// The subcycled root step: level l steps once, then (if it has children) level
// l+1 steps twice with half the time step, then level l is corrected.
amr_status enqueue_advance(amr_table* t, double* U, int l, int substep, hipStream_t s) {
  amr_status st = enqueue_step(t, U, t->dtl + l, l, 0, s, nullptr, substep);
  if (st != AMR_OK) return st;
  if (l < t->max_level && t->has_kids[l]) {
    for (int k = 0; k < 2; ++k) {
      st = enqueue_advance(t, U, l + 1, k, s);
      if (st != AMR_OK) return st;
    }
    st = enqueue_correct(t, U, l, s);
    if (st != AMR_OK) return st;
  }
  return AMR_OK;
}

void drop_graph(amr_table* t) {
  if (t->gc.exec) (void)hipGraphExecDestroy(t->gc.exec);
  if (t->gc.graph) (void)hipGraphDestroy(t->gc.graph);
  t->gc = GraphCache{};
  if (t->gadv.exec) (void)hipGraphExecDestroy(t->gadv.exec);
  if (t->gadv.graph) (void)hipGraphDestroy(t->gadv.graph);
  t->gadv = GraphCache{};
}


// EXTERNAL ghost plan: each ghost cell (two layers, the cross region) is copied
// from the same-level patch that holds it as an active cell (periodic root domain
// wrap applied) or, on levels > 0, prolonged from the level-1 patch holding its
// coarse cell.  Fails with AMR_EINVAL if a ghost cell has no source.
// Disjoint boxes covering the marked cells of an n[0] x n[1] x n[2] mask (x
// fastest), greedily: from the first marked cell grow along x, then y, then z
// while every cell of the grown box is marked; emit(lo, sz) per box.
template <class Emit>
void cover_boxes(const int n[3], std::vector<char>& m, Emit emit) {
  auto at = [&](int x, int y, int z) -> char& { return m[((size_t)z * n[1] + y) * n[0] + x]; };
  for (int z = 0; z < n[2]; ++z)
    for (int y = 0; y < n[1]; ++y)
      for (int x = 0; x < n[0]; ++x) {
        if (!at(x, y, z)) continue;
        int x1 = x;
        while (x1 < n[0] && at(x1, y, z)) ++x1;
        int y1 = y + 1;
        for (; y1 < n[1]; ++y1) {
          bool ok = true;
          for (int i = x; i < x1 && ok; ++i) ok = at(i, y1, z) != 0;
          if (!ok) break;
        }
        int z1 = z + 1;
        for (; z1 < n[2]; ++z1) {
          bool ok = true;
          for (int j = y; j < y1 && ok; ++j)
            for (int i = x; i < x1 && ok; ++i) ok = at(i, j, z1) != 0;
          if (!ok) break;
        }
        for (int k = z; k < z1; ++k)
          for (int j = y; j < y1; ++j)
            for (int i = x; i < x1; ++i) at(i, j, k) = 0;
        const int lo[3] = {x, y, z}, sz[3] = {x1 - x, y1 - y, z1 - z};
        emit(lo, sz);
      }
}

// Cell-granular work list of ops[0..count) (boxes of sz cells), appended to the
// table-wide segment and workgroup arrays.
template <class Op>
WorkList add_work(std::vector<Seg>& segs, std::vector<int>& blk, const Op* ops, int count) {
  WorkList w;
  w.blk_base = (int)blk.size();
  int64_t cum = 0;
  for (int i = 0; i < count; ++i) {
    const int64_t n = (int64_t)ops[i].sz[0] * ops[i].sz[1] * ops[i].sz[2];
    for (int64_t c = 0; c < n;) {
      const int lane0 = (int)(cum % NT);
      if (lane0 == 0) blk.push_back((int)segs.size());  // first segment of a new workgroup
      const int take = (int)std::min<int64_t>(n - c, NT - lane0);
      segs.push_back(Seg{i, (int)c, lane0, take});
      c += take;
      cum += take;
    }
  }
  w.nblk = (int)((cum + NT - 1) / NT);
  blk.push_back((int)segs.size());  // end of the last workgroup's segments
  return w;
}

amr_status build_ghost_plan(amr_table* t, std::vector<CopyOp>& ops, std::vector<ProlongOp>& pops) {
  const int nd = t->ph.ndim;
  const int np = (int)t->desc.size();
  t->dsrc.assign(6 * (size_t)np, -1);
  t->dsh.assign(18 * (size_t)np, 0);
  const int layers = 2;  // the PLM stencil reads two ghost layers
  for (int p = 0; p < np; ++p) {
    const amr_patch_desc& D = t->desc[p];
    for (int d = 0; d < nd; ++d)
      for (int side = 0; side < 2; ++side) {
        if (D.bc[2 * d + side] != AMR_BC_EXTERNAL) continue;
        int blo[3], bsz[3];  // ghost box in p-local active-relative coordinates
        for (int e = 0; e < 3; ++e) {
          blo[e] = 0;
          bsz[e] = D.n[e];
        }
        blo[d] = side == 0 ? -layers : D.n[d];
        bsz[d] = layers;
        int wrap[3] = {0, 0, 0};
        for (int e = 0; e < nd; ++e) {
          const int glo = D.lo[e] + blo[e], ghi = glo + bsz[e];
          if ((t->ph.periodic >> e) & 1) {
            const int dom = t->ph.domain[e] << D.level;
            if (ghi <= 0) wrap[e] = dom;
            else if (glo >= dom) wrap[e] = -dom;
          }
        }
        // coverage map of the box, x fastest
        std::vector<char> cov((size_t)bsz[0] * bsz[1] * bsz[2], 0);
        auto mark = [&](const int lo[3], const int sz[3]) {  // box in p-local coordinates
          for (int k = 0; k < sz[2]; ++k)
            for (int j = 0; j < sz[1]; ++j)
              for (int i = 0; i < sz[0]; ++i) {
                const int x = lo[0] + i - blo[0], y = lo[1] + j - blo[1], z = lo[2] + k - blo[2];
                cov[((size_t)z * bsz[1] + y) * bsz[0] + x]++;
              }
        };
        const size_t first_op = ops.size();
        for (int q = 0; q < np; ++q) {
          const amr_patch_desc& Q = t->desc[q];
          if (Q.level != D.level) continue;
          if (q == p && wrap[0] == 0 && wrap[1] == 0 && wrap[2] == 0) continue;
          CopyOp op{};
          op.dst = p;
          op.src = q;
          bool empty = false;
          for (int e = 0; e < 3; ++e) {
            const int glo = D.lo[e] + blo[e] + wrap[e], ghi = glo + bsz[e];
            const int lo = std::max(glo, Q.lo[e]), hi = std::min(ghi, Q.lo[e] + Q.n[e]);
            if (e >= nd) {
              op.lo[e] = 0;
              op.sz[e] = 1;
              op.sh[e] = 0;
              continue;
            }
            if (hi <= lo) {
              empty = true;
              break;
            }
            op.lo[e] = lo - D.lo[e] - wrap[e];
            op.sz[e] = hi - lo;
            op.sh[e] = D.lo[e] + wrap[e] - Q.lo[e];
          }
          if (empty) continue;
          mark(op.lo, op.sz);
          ops.push_back(op);
        }
        // Single-level tables: a face whose whole ghost slab lies in one sibling of the
        // same stored shape is read by the stage kernel from that sibling's cells (an
        // element offset, PatchDev::nbo) and needs no copy.  (Hierarchies keep the
        // copies: refluxing and prolongation read ghost storage.)
        if (t->max_level == 0 && ops.size() == first_op + 1) {
          const CopyOp& op = ops.back();
          const amr_patch_desc& Q = t->desc[op.src];
          bool whole = Q.ng == D.ng;
          for (int e = 0; e < 3; ++e) whole = whole && op.sz[e] == bsz[e] && Q.n[e] == D.n[e];
          if (whole) {
            PatchDev& P = t->pdev[p];
            const int f = 2 * d + side;
            P.dmask |= 1 << f;
            P.nbo[f] = (t->pdev[op.src].off - P.off) + ((int64_t)op.sh[2] * P.s[1] + op.sh[1]) * P.s[0] + op.sh[0];
            t->dsrc[6 * p + f] = op.src;
            for (int e = 0; e < 3; ++e) t->dsh[3 * (6 * p + f) + e] = op.sh[e];
            ops.pop_back();
          }
        }
        // a patch without ghost storage takes every EXTERNAL face from a direct sibling
        if (D.ng == 0 && (ops.size() != first_op || D.level > 0)) return AMR_EINVAL;
        if (D.level > 0) {
          for (int q = 0; q < np; ++q) {
            const amr_patch_desc& Q = t->desc[q];
            if (Q.level != D.level - 1) continue;
            int ilo[3], isz[3];  // intersection with the refined coarse patch, p-local
            bool empty = false;
            for (int e = 0; e < 3; ++e) {
              if (e >= nd) {
                ilo[e] = 0;
                isz[e] = 1;
                continue;
              }
              const int glo = D.lo[e] + blo[e] + wrap[e], ghi = glo + bsz[e];
              const int lo = std::max(glo, 2 * Q.lo[e]), hi = std::min(ghi, 2 * (Q.lo[e] + Q.n[e]));
              if (hi <= lo) {
                empty = true;
                break;
              }
              ilo[e] = lo - D.lo[e] - wrap[e];
              isz[e] = hi - lo;
            }
            if (empty) continue;
            // boxes of the cells not held by a sibling
            std::vector<char> need((size_t)isz[0] * isz[1] * isz[2]);
            for (int k = 0; k < isz[2]; ++k)
              for (int j = 0; j < isz[1]; ++j)
                for (int i = 0; i < isz[0]; ++i) {
                  const int x = ilo[0] + i - blo[0], y = ilo[1] + j - blo[1], z = ilo[2] + k - blo[2];
                  need[((size_t)k * isz[1] + j) * isz[0] + i] = cov[((size_t)z * bsz[1] + y) * bsz[0] + x] == 0;
                }
            cover_boxes(isz, need, [&](const int lo[3], const int sz[3]) {
              ProlongOp op{};
              op.dst = p;
              op.src = q;
              for (int e = 0; e < 3; ++e) {
                op.lo[e] = ilo[e] + lo[e];
                op.sz[e] = sz[e];
                op.foff[e] = e < nd ? D.lo[e] + wrap[e] : 0;
                op.clo[e] = e < nd ? Q.lo[e] : 0;
              }
              pops.push_back(op);
              mark(op.lo, op.sz);
            });
          }
        }
        for (char c : cov)
          if (c != 1) return AMR_EINVAL;  // a ghost cell without (or with two) sources
      }
  }
  std::stable_sort(ops.begin(), ops.end(),
                   [&](const CopyOp& a, const CopyOp& b) { return t->desc[a.dst].level < t->desc[b.dst].level; });
  t->ops_level_first.assign(MAX_LEVELS, 0);
  t->ops_level_count.assign(MAX_LEVELS, 0);
  for (int i = (int)ops.size() - 1; i >= 0; --i) {
    const int l = t->desc[ops[i].dst].level;
    t->ops_level_first[l] = i;
    t->ops_level_count[l]++;
  }
  std::stable_sort(pops.begin(), pops.end(),
                   [&](const ProlongOp& a, const ProlongOp& b) { return t->desc[a.dst].level < t->desc[b.dst].level; });
  t->prol_first.assign(MAX_LEVELS, 0);
  t->prol_count.assign(MAX_LEVELS, 0);
  for (int i = (int)pops.size() - 1; i >= 0; --i) {
    const int l = t->desc[pops[i].dst].level;
    t->prol_first[l] = i;
    t->prol_count[l]++;
  }
  return AMR_OK;
}

// Coarse/fine coupling plans of the hierarchy: registers, physical-ghost fills and
// snapshots of levels with children, refluxing ops (coloured so that ops sharing a
// coarse cell run in plan order, one colour after another) and restriction ops.
struct HierPlan {
  std::vector<PhysOp> phys;
  std::vector<FixOp> fix;
  std::vector<int> fix_color;
  std::vector<RestrictOp> rst;
  std::vector<CopyOp> snap;  // storage boxes of levels with children copied into the snapshot
  int64_t nreg = 0;
};

amr_status build_hierarchy(amr_table* t, HierPlan& H, const std::vector<ProlongOp>& pops) {
  const int nd = t->ph.ndim;
  const int np = (int)t->desc.size();
  const int L = t->max_level + 1;
  t->has_kids.assign(MAX_LEVELS, 0);
  for (const auto& D : t->desc)
    if (D.level > 0) t->has_kids[D.level - 1] = 1;
  // level > 0 patches start and end on coarse cell boundaries
  for (const auto& D : t->desc)
    if (D.level > 0)
      for (int e = 0; e < nd; ++e)
        if ((D.lo[e] & 1) || (D.n[e] & 1)) return AMR_EINVAL;
  // registers, level by level
  t->reg_first.assign(MAX_LEVELS, 0);
  t->reg_len.assign(MAX_LEVELS, 0);
  for (int l = 1; l < L; ++l) {
    t->reg_first[l] = H.nreg;
    for (int p = 0; p < np; ++p) {
      const auto& D = t->desc[p];
      if (D.level != l) continue;
      for (int d = 0; d < nd; ++d)
        for (int side = 0; side < 2; ++side) {
          if (D.bc[2 * d + side] != AMR_BC_EXTERNAL) continue;
          int64_t area = 1;
          for (int e = 0; e < 3; ++e)
            if (e != d) area *= D.n[e];
          t->pdev[p].reg[2 * d + side] = H.nreg;
          H.nreg += t->ph.nvar * area;
        }
    }
    t->reg_len[l] = H.nreg - t->reg_first[l];
  }
  // physical ghosts of levels with children
  t->phys_first.assign(MAX_LEVELS, 0);
  t->phys_count.assign(MAX_LEVELS, 0);
  for (int l = 0; l < L; ++l) {
    if (!t->has_kids[l]) continue;
    t->phys_first[l] = (int)H.phys.size();
    for (int p = 0; p < np; ++p) {
      const auto& D = t->desc[p];
      if (D.level != l) continue;
      for (int d = 0; d < nd; ++d)
        for (int side = 0; side < 2; ++side) {
          if (D.bc[2 * d + side] == AMR_BC_EXTERNAL) continue;
          PhysOp op{};
          op.patch = p;
          for (int e = 0; e < 3; ++e) {
            op.lo[e] = 0;
            op.sz[e] = D.n[e];
          }
          op.lo[d] = side == 0 ? -2 : D.n[d];
          op.sz[d] = 2;
          H.phys.push_back(op);
        }
    }
    t->phys_count[l] = (int)H.phys.size() - t->phys_first[l];
  }
  // coarse cells (level l coordinates) under a level l+1 patch
  auto key3 = [](int x, int y, int z) { return ((int64_t)z << 42) ^ ((int64_t)y << 21) ^ (int64_t)x; };
  std::vector<std::unordered_set<int64_t>> cov(L);
  for (const auto& F : t->desc) {
    if (F.level == 0) continue;
    int lo[3], hi[3];
    for (int e = 0; e < 3; ++e) {
      lo[e] = e < nd ? F.lo[e] / 2 : 0;
      hi[e] = e < nd ? (F.lo[e] + F.n[e]) / 2 : 1;
    }
    for (int z = lo[2]; z < hi[2]; ++z)
      for (int y = lo[1]; y < hi[1]; ++y)
        for (int x = lo[0]; x < hi[0]; ++x) cov[F.level - 1].insert(key3(x, y, z));
  }
  auto covered = [&](int l, const int c[3]) { return cov[l].count(key3(c[0], c[1], c[2])) != 0; };
  // refluxing and restriction ops, coarse level by coarse level
  t->fix_colors.assign(MAX_LEVELS, {});
  t->rst_first.assign(MAX_LEVELS, 0);
  t->rst_count.assign(MAX_LEVELS, 0);
  std::vector<FixOp> fixall;
  std::vector<int> colall;
  for (int l = 0; l + 1 < L; ++l) {
    std::map<std::pair<int, int64_t>, int> last_color;  // (coarse patch, cell) -> colour of its last op
    std::vector<FixOp> fl;
    std::vector<int> cl;
    for (int p = 0; p < np; ++p) {
      const auto& F = t->desc[p];
      if (F.level != l + 1) continue;
      for (int d = 0; d < nd; ++d)
        for (int side = 0; side < 2; ++side) {
          if (F.bc[2 * d + side] != AMR_BC_EXTERNAL) continue;
          const int cf = (F.lo[d] + (side ? F.n[d] : 0)) / 2;
          int Cd = side == 0 ? cf - 1 : cf;
          if ((t->ph.periodic >> d) & 1) {
            const int dom = t->ph.domain[d] << l;
            Cd = ((Cd % dom) + dom) % dom;
          }
          int flo[3], fhi[3];  // coarse footprint (level l coordinates)
          for (int e = 0; e < 3; ++e) {
            flo[e] = e < nd ? F.lo[e] / 2 : 0;
            fhi[e] = e < nd ? (F.lo[e] + F.n[e]) / 2 : 1;
          }
          flo[d] = Cd;
          fhi[d] = Cd + 1;
          for (int q = 0; q < np; ++q) {
            const auto& Q = t->desc[q];
            if (Q.level != l) continue;
            int lo[3], hi[3];
            bool empty = false;
            for (int e = 0; e < 3; ++e) {
              lo[e] = e < nd ? std::max(flo[e], Q.lo[e]) : 0;
              hi[e] = e < nd ? std::min(fhi[e], Q.lo[e] + Q.n[e]) : 1;
              if (hi[e] <= lo[e]) empty = true;
            }
            if (empty) continue;
            // boxes of uncovered cells; an op's colour exceeds that of every earlier
            // op touching one of its cells
            const int bsz[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
            std::vector<char> need((size_t)bsz[0] * bsz[1] * bsz[2]);
            for (int z = lo[2]; z < hi[2]; ++z)
              for (int y = lo[1]; y < hi[1]; ++y)
                for (int x = lo[0]; x < hi[0]; ++x) {
                  const int c3[3] = {x, y, z};
                  need[((size_t)(z - lo[2]) * bsz[1] + (y - lo[1])) * bsz[0] + (x - lo[0])] = !covered(l, c3);
                }
            cover_boxes(bsz, need, [&](const int blo[3], const int sz[3]) {
              FixOp op{};
              op.fine = p;
              op.coarse = q;
              op.d = d;
              op.side = side;
              for (int e = 0; e < 3; ++e) {
                op.lo[e] = lo[e] + blo[e] - (e < nd ? Q.lo[e] : 0);
                op.sz[e] = sz[e];
                op.fo[e] = e < nd ? 2 * Q.lo[e] - F.lo[e] : 0;
              }
              auto key = [&](int x, int y, int z) { return ((int64_t)z * 65536 + y) * 65536 + x; };
              int color = 0;
              for (int z = 0; z < sz[2]; ++z)
                for (int y = 0; y < sz[1]; ++y)
                  for (int x = 0; x < sz[0]; ++x) {
                    auto it = last_color.find({q, key(lo[0] + blo[0] + x, lo[1] + blo[1] + y, lo[2] + blo[2] + z)});
                    if (it != last_color.end()) color = std::max(color, it->second + 1);
                  }
              for (int z = 0; z < sz[2]; ++z)
                for (int y = 0; y < sz[1]; ++y)
                  for (int x = 0; x < sz[0]; ++x)
                    last_color[{q, key(lo[0] + blo[0] + x, lo[1] + blo[1] + y, lo[2] + blo[2] + z)}] = color;
              fl.push_back(op);
              cl.push_back(color);
            });
          }
        }
    }
    // order by colour (stable: plan order within a colour)
    int ncol = 0;
    for (int c : cl) ncol = std::max(ncol, c + 1);
    for (int c = 0; c < ncol; ++c) {
      const int first = (int)fixall.size();
      for (size_t i = 0; i < fl.size(); ++i)
        if (cl[i] == c) fixall.push_back(fl[i]);
      t->fix_colors[l].push_back({first, (int)fixall.size() - first});
    }
    // restriction
    t->rst_first[l] = (int)H.rst.size();
    for (int p = 0; p < np; ++p) {
      const auto& F = t->desc[p];
      if (F.level != l + 1) continue;
      for (int q = 0; q < np; ++q) {
        const auto& Q = t->desc[q];
        if (Q.level != l) continue;
        RestrictOp op{};
        op.fine = p;
        op.coarse = q;
        bool empty = false;
        for (int e = 0; e < 3; ++e) {
          if (e >= nd) {
            op.lo[e] = 0;
            op.sz[e] = 1;
            op.fo[e] = 0;
            continue;
          }
          const int lo = std::max(F.lo[e] / 2, Q.lo[e]), hi = std::min((F.lo[e] + F.n[e]) / 2, Q.lo[e] + Q.n[e]);
          if (hi <= lo) empty = true;
          op.lo[e] = lo - Q.lo[e];
          op.sz[e] = hi - lo;
          op.fo[e] = 2 * Q.lo[e] - F.lo[e];
        }
        if (!empty) H.rst.push_back(op);
      }
    }
    t->rst_count[l] = (int)H.rst.size() - t->rst_first[l];
  }
  H.fix = fixall;
  // Snapshot boxes.  A level's U^n is read later by its children's prolongation (the
  // coarse cell of each fine ghost cell and its face neighbours, from storage) and by
  // refluxing (the coarse stage inputs two cells either side of each corrected face,
  // through the boundary conditions' index maps): only those storage cells are copied,
  // as boxes covering a per-patch mask of them.
  t->snap_first.assign(MAX_LEVELS, 0);
  t->snap_count.assign(MAX_LEVELS, 0);
  std::vector<std::vector<char>> smask(np);
  auto mark = [&](int q, int x, int y, int z) {
    const PatchDev& Q = t->pdev[q];
    const int c[3] = {x, y, z};
    for (int e = 0; e < 3; ++e)
      if (c[e] < -Q.g[e] || c[e] >= Q.n[e] + Q.g[e]) return;  // outside storage: nothing to read there
    std::vector<char>& m = smask[q];
    if (m.empty()) m.assign((size_t)Q.S, 0);
    m[((size_t)(z + Q.g[2]) * Q.s[1] + (y + Q.g[1])) * Q.s[0] + (x + Q.g[0])] = 1;
  };
  for (const ProlongOp& op : pops) {
    const int q = op.src;
    int lo[3], hi[3];
    for (int e = 0; e < 3; ++e) {
      if (e >= nd) {
        lo[e] = 0;
        hi[e] = 1;
        continue;
      }
      lo[e] = ((op.lo[e] + op.foff[e]) >> 1) - op.clo[e] - 1;
      hi[e] = ((op.lo[e] + op.sz[e] - 1 + op.foff[e]) >> 1) - op.clo[e] + 2;
    }
    for (int z = lo[2]; z < hi[2]; ++z)
      for (int y = lo[1]; y < hi[1]; ++y)
        for (int x = lo[0]; x < hi[0]; ++x) mark(q, x, y, z);
  }
  for (const FixOp& op : fixall) {
    const PatchDev& Q = t->pdev[op.coarse];
    int lo[3], hi[3];
    for (int e = 0; e < 3; ++e) {
      lo[e] = op.lo[e];
      hi[e] = op.lo[e] + op.sz[e];
    }
    lo[op.d] -= 2;
    hi[op.d] += 2;
    for (int z = lo[2]; z < hi[2]; ++z)
      for (int y = lo[1]; y < hi[1]; ++y)
        for (int x = lo[0]; x < hi[0]; ++x) {
          int c[3] = {x, y, z};
          bool flip = false;
          const int dd = op.d;
          c[dd] = map_index(c[dd], Q.n[dd], Q.bc[2 * dd], Q.bc[2 * dd + 1], flip);
          mark(op.coarse, c[0], c[1], c[2]);
        }
  }
  for (int l = 0; l < L; ++l) {
    t->snap_first[l] = (int)H.snap.size();
    if (!t->has_kids[l]) continue;
    for (int q = 0; q < np; ++q) {
      if (t->desc[q].level != l || smask[q].empty()) continue;
      const PatchDev& Q = t->pdev[q];
      cover_boxes(Q.s, smask[q], [&](const int blo[3], const int sz[3]) {
        CopyOp op{};
        op.dst = q;
        op.src = q;
        for (int e = 0; e < 3; ++e) {
          op.lo[e] = blo[e] - Q.g[e];
          op.sz[e] = sz[e];
          op.sh[e] = 0;
        }
        H.snap.push_back(op);
      });
    }
    t->snap_count[l] = (int)H.snap.size() - t->snap_first[l];
  }
  return AMR_OK;
}

}  // namespace

namespace {
// Layout of the stage scratch U^(1).  Where no patch needs stored ghosts (a single
// level, every EXTERNAL face read directly from a same-shaped sibling), U^(1) holds the
// active cells alone, patch after patch (the stage kernels write and read whole 128-byte
// lines instead of rows framed by ghost cells); otherwise it mirrors U's layout, whose
// ghost storage the ghost fill and refluxing use.
void set_scratch_layout(amr_table* t, bool dense) {
  dense = dense && t->max_level == 0;
  const int np = (int)t->pdev.size();
  int64_t cur = 0;
  for (int p = 0; p < np; ++p) {
    PatchDev& P = t->pdev[p];
    if (!dense) {
      P.off1 = P.off;
      P.S1 = P.S;
      for (int d = 0; d < 3; ++d) {
        P.s1[d] = P.s[d];
        P.g1[d] = P.g[d];
      }
      for (int f = 0; f < 6; ++f) P.nbo1[f] = P.nbo[f];
      continue;
    }
    cur = (cur + 63) / 64 * 64;  // 512-byte aligned patches
    P.off1 = cur;
    P.S1 = (int64_t)P.n[0] * P.n[1] * P.n[2];
    for (int d = 0; d < 3; ++d) {
      P.s1[d] = P.n[d];
      P.g1[d] = 0;
    }
    cur += t->ph.nvar * P.S1;
  }
  if (dense) {
    for (int p = 0; p < np; ++p) {
      PatchDev& P = t->pdev[p];
      for (int f = 0; f < 6; ++f) {
        const int q = t->dsrc[6 * p + f];
        if (q < 0) {
          P.nbo1[f] = 0;
          continue;
        }
        const int* sh = &t->dsh[3 * (6 * p + f)];
        P.nbo1[f] = (t->pdev[q].off1 - P.off1) + ((int64_t)sh[2] * P.s1[1] + sh[1]) * P.s1[0] + sh[0];
      }
    }
  }
  t->arena1 = dense ? std::max<int64_t>(cur, 1) : t->arena;
}

}  // namespace

extern "C" {

const char* amr_status_string(amr_status s) {
  switch (s) {
    case AMR_OK: return "AMR_OK";
    case AMR_EINVAL: return "AMR_EINVAL: invalid argument";
    case AMR_ENOMEM: return "AMR_ENOMEM: allocation failed";
    case AMR_EHIP: return "AMR_EHIP: HIP runtime error";
    case AMR_EUNPHYSICAL: return "AMR_EUNPHYSICAL: rho <= 0, e <= 0 or non-finite state met";
    case AMR_ESTATE: return "AMR_ESTATE: call not valid in the table's current state";
    default: return "unknown amr_status";
  }
}

amr_status amr_patch_table_create(const amr_patch_desc* patches, int32_t npatch, const amr_physics* phys,
                                  hipStream_t stream, amr_table** out) {
  if (!out) return AMR_EINVAL;
  *out = nullptr;
  amr_status st = validate_patches(patches, npatch, phys);
  if (st != AMR_OK) return st;
  amr_table* t = new (std::nothrow) amr_table();
  if (!t) return AMR_ENOMEM;
  t->ph = *phys;
  t->desc.assign(patches, patches + npatch);
  for (int p = 0; p < npatch; ++p) {
    const amr_patch_desc& D = patches[p];
    PatchDev P{};
    P.off = D.offset;
    P.level = D.level;
    int64_t S = 1;
    for (int d = 0; d < 3; ++d) {
      P.n[d] = D.n[d];
      P.g[d] = d < phys->ndim ? D.ng : 0;
      P.s[d] = P.n[d] + 2 * P.g[d];
      P.dx[d] = ldexp(phys->dx0[d], -D.level);
      P.rdx[d] = 1.0 / P.dx[d];
      S *= P.s[d];
    }
    P.S = S;
    for (int f = 0; f < 6; ++f) {
      P.bc[f] = D.bc[f];
      P.reg[f] = -1;
    }
    t->pdev.push_back(P);
    t->arena = std::max(t->arena, D.offset + phys->nvar * S);
    t->max_level = std::max(t->max_level, D.level);
  }
  // hierarchies store ghosts (prolongation, physical ghosts for the children's stencils)
  for (int p = 0; p < npatch && t->max_level > 0; ++p)
    if (patches[p].ng == 0) {
      delete t;
      return AMR_EINVAL;
    }
  std::vector<CopyOp> ops;
  std::vector<ProlongOp> pops;
  HierPlan H;
  st = build_ghost_plan(t, ops, pops);
  if (st == AMR_OK) st = build_hierarchy(t, H, pops);
  if (st != AMR_OK) {
    delete t;
    return st;
  }
  set_scratch_layout(t, ops.empty() && pops.empty());
  t->last_dt.assign(MAX_LEVELS, nullptr);
  auto fail = [&](amr_status s) {
    amr_patch_table_destroy(t);
    return s;
  };
  if (hipGetDevice(&t->device) != hipSuccess) return fail(AMR_EHIP);
  if (hipDeviceGetAttribute(&t->ncu, hipDeviceAttributeMultiprocessorCount, t->device) != hipSuccess)
    return fail(AMR_EHIP);
  if (hipMalloc(&t->pdev_d, sizeof(PatchDev) * t->pdev.size()) != hipSuccess) return fail(AMR_ENOMEM);
  if (hipMalloc(&t->U1, sizeof(double) * (size_t)t->arena1) != hipSuccess) return fail(AMR_ENOMEM);
  if (hipMalloc(&t->flag_d, sizeof(int)) != hipSuccess) return fail(AMR_ENOMEM);
  if (hipMalloc(&t->smax_d, sizeof(unsigned long long) * (MAX_LEVELS + 1)) != hipSuccess) return fail(AMR_ENOMEM);
  if (hipMalloc(&t->fused_d, sizeof(unsigned long long) * (MAX_LEVELS + 1)) != hipSuccess) return fail(AMR_ENOMEM);
  t->nops = (int)ops.size();
  if (t->nops > 0 && hipMalloc(&t->ops_d, sizeof(CopyOp) * ops.size()) != hipSuccess) return fail(AMR_ENOMEM);
  if (hipMemcpyAsync(t->pdev_d, t->pdev.data(), sizeof(PatchDev) * t->pdev.size(), hipMemcpyHostToDevice,
                     stream) != hipSuccess)
    return fail(AMR_EHIP);
  if (t->nops > 0 && hipMemcpyAsync(t->ops_d, ops.data(), sizeof(CopyOp) * ops.size(), hipMemcpyHostToDevice,
                                    stream) != hipSuccess)
    return fail(AMR_EHIP);
  // hierarchy plans
  auto upload = [&](auto** dst, const auto& v) -> bool {
    if (v.empty()) return true;
    using T = typename std::remove_reference<decltype(v)>::type::value_type;
    if (hipMalloc(dst, sizeof(T) * v.size()) != hipSuccess) return false;
    return hipMemcpyAsync(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, stream) == hipSuccess;
  };
  std::vector<CopyOp> pcp(pops.size());
  for (size_t i = 0; i < pops.size(); ++i) {
    pcp[i].dst = pcp[i].src = pops[i].dst;
    for (int e = 0; e < 3; ++e) {
      pcp[i].lo[e] = pops[i].lo[e];
      pcp[i].sz[e] = pops[i].sz[e];
      pcp[i].sh[e] = 0;
    }
  }
  if (!upload(&t->prol_d, pops) || !upload(&t->pcp_d, pcp) || !upload(&t->phys_d, H.phys) || !upload(&t->fix_d, H.fix) ||
      !upload(&t->rst_d, H.rst) || !upload(&t->snap_d, H.snap))
    return fail(AMR_ENOMEM);
  // cell-granular work lists of every box-op launch
  {
    std::vector<Seg> segs;
    std::vector<int> blk;
    t->w_copy.assign(MAX_LEVELS, {});
    t->w_prol.assign(MAX_LEVELS, {});
    t->w_phys.assign(MAX_LEVELS, {});
    t->w_rst.assign(MAX_LEVELS, {});
    t->w_snap.assign(MAX_LEVELS, {});
    t->w_fix.assign(MAX_LEVELS, {});
    for (int l = 0; l <= t->max_level; ++l) {
      t->w_copy[l] = add_work(segs, blk, ops.data() + t->ops_level_first[l], t->ops_level_count[l]);
      t->w_prol[l] = add_work(segs, blk, pops.data() + t->prol_first[l], t->prol_count[l]);
      t->w_phys[l] = add_work(segs, blk, H.phys.data() + t->phys_first[l], t->phys_count[l]);
      t->w_rst[l] = add_work(segs, blk, H.rst.data() + t->rst_first[l], t->rst_count[l]);
      t->w_snap[l] = add_work(segs, blk, H.snap.data() + t->snap_first[l], t->snap_count[l]);
      for (const auto& fc : t->fix_colors[l]) t->w_fix[l].push_back(add_work(segs, blk, H.fix.data() + fc.first, fc.second));
    }
    if (!upload(&t->segs_d, segs) || !upload(&t->blk_d, blk)) return fail(AMR_ENOMEM);
  }
  if (t->max_level > 0) {
    if (hipMalloc(&t->snap, sizeof(double) * (size_t)t->arena) != hipSuccess) return fail(AMR_ENOMEM);
    if (hipMalloc(&t->dtl, sizeof(double) * MAX_LEVELS) != hipSuccess) return fail(AMR_ENOMEM);
    if (H.nreg > 0) {
      if (hipMalloc(&t->reg, sizeof(double) * (size_t)H.nreg) != hipSuccess) return fail(AMR_ENOMEM);
      for (int64_t o = 0; o < H.nreg; o += (int64_t)1 << 30)
        if (launch_fill_u64(stream, reinterpret_cast<unsigned long long*>(t->reg + o),
                            (int)std::min<int64_t>(H.nreg - o, (int64_t)1 << 30), 0ull) != hipSuccess)
          return fail(AMR_EHIP);
    }
  }
  // the patch copy carries the register offsets
  if (hipMemcpyAsync(t->pdev_d, t->pdev.data(), sizeof(PatchDev) * t->pdev.size(), hipMemcpyHostToDevice,
                     stream) != hipSuccess)
    return fail(AMR_EHIP);
  if (launch_fill_i32(stream, t->flag_d, 1, 0) != hipSuccess) return fail(AMR_EHIP);
  if (launch_fill_u64(stream, t->fused_d, MAX_LEVELS + 1, 0ull) != hipSuccess) return fail(AMR_EHIP);
  if (hipStreamSynchronize(stream) != hipSuccess) return fail(AMR_EHIP);
  if (hipStreamCreateWithFlags(&t->cap_stream, hipStreamNonBlocking) != hipSuccess) return fail(AMR_EHIP);
  t->shape = default_shape(t);
  t->zslab = default_zslab(t);
  *out = t;
  return AMR_OK;
}

amr_status amr_patch_table_destroy(amr_table* t) {
  if (!t) return AMR_EINVAL;
  (void)hipDeviceSynchronize();
  drop_graph(t);
  for (auto& kv : t->tiles)
    if (kv.second.d) (void)hipFree(kv.second.d);
  for (auto& kv : t->cell_lists) {
    if (kv.second.plist) (void)hipFree(kv.second.plist);
    if (kv.second.cofs) (void)hipFree(kv.second.cofs);
  }
  if (t->pdev_d) (void)hipFree(t->pdev_d);
  if (t->U1) (void)hipFree(t->U1);
  if (t->flag_d) (void)hipFree(t->flag_d);
  if (t->smax_d) (void)hipFree(t->smax_d);
  if (t->fused_d) (void)hipFree(t->fused_d);
  if (t->ops_d) (void)hipFree(t->ops_d);
  for (void* q : {(void*)t->snap, (void*)t->reg, (void*)t->dtl, (void*)t->prol_d, (void*)t->pcp_d, (void*)t->phys_d, (void*)t->fix_d,
                  (void*)t->rst_d, (void*)t->snap_d, (void*)t->segs_d, (void*)t->blk_d})
    if (q) (void)hipFree(q);
  if (t->cap_stream) (void)hipStreamDestroy(t->cap_stream);
  for (auto& e : t->ev)
    if (e) (void)hipEventDestroy(e);
  delete t;
  return AMR_OK;
}

int64_t amr_table_arena_elems(const amr_table* t) { return t ? t->arena : -1; }

amr_status amr_hydro_rk2_step(amr_table* t, double* U, const double* dt_dev, int32_t level, uint32_t flags,
                              hipStream_t stream) {
  if (!t || !U || !dt_dev || level < -1 || level > t->max_level ||
      (flags & ~(AMR_STEP_FUSE_DT | AMR_STEP_TIMED | AMR_STEP_SUBSTEP1)))
    return AMR_EINVAL;
  if (t->max_level > 0 && (level < 0 || (flags & AMR_STEP_FUSE_DT))) return AMR_EINVAL;
  const bool fuse = (flags & AMR_STEP_FUSE_DT) != 0;
  const int substep = (flags & AMR_STEP_SUBSTEP1) ? 1 : 0;
  // the second substep reuses the first's half-step ghosts: it needs that first substep
  if (substep && level > 0 && !(t->half_mask & (1u << level))) return AMR_ESTATE;
  if (flags & AMR_STEP_TIMED) {
    for (auto& e : t->ev)
      if (!e) HIPCHECK(hipEventCreate(&e));
    t->timed_valid = false;
    amr_status st = enqueue_step(t, U, dt_dev, level, flags & AMR_STEP_FUSE_DT, stream, t->ev, substep);
    if (st != AMR_OK) return st;
    t->timed_valid = true;
  } else if (t->ph.exec == AMR_EXEC_BATCHED) {
    GraphCache& g = t->gc;
    if (!(g.exec && g.U == U && g.dt == dt_dev && g.level == level && g.flags == flags && g.shape == t->shape &&
          g.zslab == t->zslab)) {
      drop_graph(t);
      // tile list upload and occupancy queries happen before capture
      TileSet* ts = nullptr;
      amr_status st = get_tiles(t, level, t->shape, t->zslab, &ts);
      if (st != AMR_OK) return st;
      for (bool r : {false, true}) {
        occupancy_grid(t, 1, ts->n, r);
        occupancy_grid(t, 2, ts->n, r);
      }
      HIPCHECK(hipStreamBeginCapture(t->cap_stream, hipStreamCaptureModeThreadLocal));
      st = enqueue_step(t, U, dt_dev, level, flags, t->cap_stream, nullptr, substep);
      hipGraph_t graph = nullptr;
      hipError_t e = hipStreamEndCapture(t->cap_stream, &graph);
      if (st != AMR_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
      }
      if (e != hipSuccess) return AMR_EHIP;
      hipGraphExec_t exec = nullptr;
      if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return AMR_EHIP;
      }
      g.exec = exec;
      g.graph = graph;
      g.U = U;
      g.dt = dt_dev;
      g.level = level;
      g.flags = flags;
      g.shape = t->shape;
      g.zslab = t->zslab;
    }
    HIPCHECK(hipGraphLaunch(g.exec, stream));
  } else {
    amr_status st = enqueue_step(t, U, dt_dev, level, flags, stream, nullptr, substep);
    if (st != AMR_OK) return st;
  }
  if (fuse) {
    t->fused_U = U;
    t->fused_level = level;
  } else if (t->fused_U == U) {
    t->fused_U = nullptr;
    t->fused_level = -2;
  }
  if (level >= 0 && t->has_kids[level]) t->open_mask |= 1u << level;
  if (level > 0) t->half_mask = substep ? t->half_mask & ~(1u << level) : t->half_mask | (1u << level);
  if (level >= 0 && level + 1 < 32) t->half_mask &= ~(1u << (level + 1));  // a new parent step
  return AMR_OK;
}

amr_status amr_cfl_dt(amr_table* t, const double* U, double cfl, int32_t level, double* dt_dev, double* dt_host,
                      hipStream_t stream) {
  if (!t || !U || !dt_dev || !(cfl > 0) || level < -1 || level > t->max_level) return AMR_EINVAL;
  const int lmin = level < 0 ? 0 : level, lmax = level < 0 ? t->max_level : level;
  const unsigned long long* src;
  if (t->fused_U == U && t->fused_level == level) {
    src = t->fused_d;  // maxima of this U were reduced by the last fused stage 2
    // read once: a caller that restores U^n into the same memory (the recovery
    // recipe) gets a fresh scan from the next call
    t->fused_U = nullptr;
    t->fused_level = -2;
  } else {
    TileSet* ts = nullptr;
    amr_status st = get_tiles(t, level, t->shape, t->zslab, &ts);
    if (st != AMR_OK) return st;
    HIPCHECK(launch_fill_u64(stream, t->smax_d, MAX_LEVELS + 1, 0ull));
    if (ts->n > 0) {
      CflArgs a{};
      a.U = U;
      a.patches = t->pdev_d;
      a.tiles = ts->d;
      a.ntiles = ts->n;
      a.tx = SHAPE_TX[t->shape];
      a.ty = SHAPE_TY[t->shape];
      a.fast = t->ph.precision == AMR_PREC_MIXED;
      a.nv = t->ph.nvar;
      a.flag = t->flag_d;
      a.smax = t->smax_d;
      a.c = consts_of(t);
      HIPCHECK(launch_cfl(std::min(ts->n, 8 * t->ncu), stream, a));
    }
    src = t->smax_d;
  }
  // one level: dt_l = cfl / smax_l; all levels: root step of the factor-2 subcycling
  HIPCHECK(launch_cfl_finalize(stream, src, lmin, lmax, level < 0 ? 1 : 0, cfl, dt_dev));
  if (dt_host) {
    HIPCHECK(hipMemcpyAsync(dt_host, dt_dev, sizeof(double), hipMemcpyDeviceToHost, stream));
    int flag = 0;
    HIPCHECK(hipMemcpyAsync(&flag, t->flag_d, sizeof(int), hipMemcpyDeviceToHost, stream));
    HIPCHECK(hipStreamSynchronize(stream));
    if (flag) {
      t->fused_U = nullptr;
      t->fused_level = -2;
      return AMR_EUNPHYSICAL;
    }
  }
  return AMR_OK;
}

amr_status amr_flux_correct(amr_table* t, double* U, int32_t coarse_level, hipStream_t stream) {
  if (!t || !U || coarse_level < 0 || coarse_level > t->max_level) return AMR_EINVAL;
  if (!t->has_kids[coarse_level] || !t->last_dt[coarse_level]) return AMR_ESTATE;
  amr_status st = enqueue_correct(t, U, coarse_level, stream);
  if (st == AMR_OK) t->open_mask &= ~(1u << coarse_level);
  return st;
}

amr_status amr_hydro_advance(amr_table* t, double* U, const double* dt0_dev, uint32_t flags, hipStream_t stream) {
  if (!t || !U || !dt0_dev || flags != 0) return AMR_EINVAL;
  auto enqueue_all = [&](hipStream_t s) -> amr_status {
    HIPCHECK(launch_scale_dt(s, dt0_dev, t->dtl ? t->dtl : nullptr, t->max_level + 1));
    return enqueue_advance(t, U, 0, 0, s);
  };
  if (t->max_level == 0) {  // no hierarchy: one step of the root level with dt0
    return amr_hydro_rk2_step(t, U, dt0_dev, -1, 0, stream);
  }
  t->open_mask = 0;  // a whole root step closes every level's recursion
  t->half_mask = 0;
  for (int l = 0; l <= t->max_level; ++l) {  // tile lists and occupancy before any capture
    TileSet* ts = nullptr;
    amr_status st = get_tiles(t, l, t->shape, t->zslab, &ts);
    if (st != AMR_OK) return st;
    for (bool r : {false, true}) {
      occupancy_grid(t, 1, ts->n, r);
      occupancy_grid(t, 2, ts->n, r);
    }
  }
  if (t->ph.exec == AMR_EXEC_BATCHED) {
    GraphCache& g = t->gadv;
    if (!(g.exec && g.U == U && g.dt == dt0_dev && g.shape == t->shape && g.zslab == t->zslab)) {
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
      if (g.graph) (void)hipGraphDestroy(g.graph);
      g = GraphCache{};
      HIPCHECK(hipStreamBeginCapture(t->cap_stream, hipStreamCaptureModeThreadLocal));
      amr_status st = enqueue_all(t->cap_stream);
      hipGraph_t graph = nullptr;
      hipError_t e = hipStreamEndCapture(t->cap_stream, &graph);
      if (st != AMR_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
      }
      if (e != hipSuccess) return AMR_EHIP;
      hipGraphExec_t exec = nullptr;
      if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return AMR_EHIP;
      }
      g.exec = exec;
      g.graph = graph;
      g.U = U;
      g.dt = dt0_dev;
      g.shape = t->shape;
      g.zslab = t->zslab;
    }
    HIPCHECK(hipGraphLaunch(g.exec, stream));
    return AMR_OK;
  }
  return enqueue_all(stream);
}

amr_status amr_table_status(amr_table* t, hipStream_t stream) {
  if (!t) return AMR_EINVAL;
  int flag = 0;
  HIPCHECK(hipMemcpyAsync(&flag, t->flag_d, sizeof(int), hipMemcpyDeviceToHost, stream));
  HIPCHECK(hipStreamSynchronize(stream));
  // the caller may now rewrite U (the recovery recipe restores U^n): the next
  // amr_cfl_dt scans U instead of reading maxima fused into the last step
  t->fused_U = nullptr;
  t->fused_level = -2;
  if (flag) {
    HIPCHECK(launch_fill_i32(stream, t->flag_d, 1, 0));
    HIPCHECK(hipStreamSynchronize(stream));
    return AMR_EUNPHYSICAL;
  }
  return AMR_OK;
}

amr_status amr_table_last_stage_ms(amr_table* t, float ms[2]) {
  if (!t || !ms) return AMR_EINVAL;
  if (!t->timed_valid) return AMR_ESTATE;
  HIPCHECK(hipEventSynchronize(t->ev[3]));
  HIPCHECK(hipEventElapsedTime(&ms[0], t->ev[0], t->ev[1]));
  HIPCHECK(hipEventElapsedTime(&ms[1], t->ev[2], t->ev[3]));
  return AMR_OK;
}

int32_t amr_table_num_tilings(const amr_table* t) { return t ? NSHAPES : 0; }

amr_status amr_table_set_tiling(amr_table* t, int32_t id, int32_t zslab) {
  if (!t || !shape_ok(t, id) || zslab < 0) return AMR_EINVAL;
  t->shape = id;
  t->zslab = t->ph.ndim == 3 ? zslab : 1;  // 0 = balanced automatic choice
  drop_graph(t);
  return AMR_OK;
}

amr_status amr_table_get_tiling(amr_table* t, int32_t* id, int32_t* zslab) {
  if (!t || !id || !zslab) return AMR_EINVAL;
  *id = t->shape;
  *zslab = t->zslab == 0 ? auto_zslab(t, -1, t->shape) : t->zslab;
  return AMR_OK;
}

amr_status amr_table_tiling_shape(const amr_table* t, int32_t id, int32_t* tx, int32_t* ty) {
  if (!t || !tx || !ty || id < 0 || id >= NSHAPES) return AMR_EINVAL;
  *tx = SHAPE_TX[id];
  *ty = SHAPE_TY[id];
  return AMR_OK;
}

amr_status amr_autotune(amr_table* t, const double* U, const double* dt_dev, int32_t level, int32_t reps,
                        hipStream_t stream, float* ms_best) {
  if (!t || !U || !dt_dev || reps < 1 || level < -1 || level > t->max_level) return AMR_EINVAL;
  if (t->max_level > 0 && level < 0) return AMR_EINVAL;
  // the candidates overwrite the snapshot, U^(1) and the flux registers that an open
  // caller-driven recursion still needs
  if (t->open_mask) return AMR_ESTATE;
  // the latch as the caller left it: candidate runs on the copy must not change it
  int flag_keep = 0;
  HIPCHECK(hipMemcpyAsync(&flag_keep, t->flag_d, sizeof(int), hipMemcpyDeviceToHost, stream));
  HIPCHECK(hipStreamSynchronize(stream));
  double* W = nullptr;
  if (hipMalloc(&W, sizeof(double) * (size_t)t->arena) != hipSuccess) return AMR_ENOMEM;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    (void)hipFree(W);
    return AMR_EHIP;
  }
  int maxnz = 1;
  for (auto& P : t->pdev)
    if (level < 0 || P.level == level) maxnz = std::max(maxnz, P.n[2]);
  std::vector<int> zs;
  if (t->ph.ndim == 3) {
    zs.push_back(0);  // the balanced choice for each shape
    for (int z : {8, 16, 32, 64, 128})
      if (z < maxnz) zs.push_back(z);
    zs.push_back(maxnz);
  } else {
    zs.push_back(1);
  }
  const int keep_shape = t->shape, keep_z = t->zslab;
  const std::vector<const double*> keep_dt = t->last_dt;
  float best = 1e30f;
  int bshape = keep_shape, bz = keep_z;
  amr_status st = AMR_OK;
  for (int shape = 0; shape < NSHAPES && st == AMR_OK; ++shape) {
    if (!shape_ok(t, shape)) continue;
    for (int z : zs) {
      t->shape = shape;
      t->zslab = z;
      drop_graph(t);
      if (hipMemcpyAsync(W, U, sizeof(double) * (size_t)t->arena, hipMemcpyDeviceToDevice, stream) != hipSuccess) {
        st = AMR_EHIP;
        break;
      }
      st = amr_hydro_rk2_step(t, W, dt_dev, level, 0, stream);  // warm-up (and capture)
      if (st != AMR_OK) break;
      (void)hipEventRecord(e0, stream);
      for (int r = 0; r < reps && st == AMR_OK; ++r) st = amr_hydro_rk2_step(t, W, dt_dev, level, 0, stream);
      (void)hipEventRecord(e1, stream);
      if (hipEventSynchronize(e1) != hipSuccess) {
        st = AMR_EHIP;
        break;
      }
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      ms /= reps;
      if (ms < best) {
        best = ms;
        bshape = shape;
        bz = z;
      }
    }
  }
  (void)hipStreamSynchronize(stream);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(W);
  t->shape = st == AMR_OK ? bshape : keep_shape;
  t->zslab = st == AMR_OK ? bz : keep_z;
  drop_graph(t);
  if (t->fused_U == W) {
    t->fused_U = nullptr;
    t->fused_level = -2;
  }
  // the candidates' steps leave no recursion open and no level stepped on the caller's U
  t->open_mask = 0;
  t->half_mask = 0;
  t->last_dt = keep_dt;
  HIPCHECK(launch_fill_i32(stream, t->flag_d, 1, flag_keep));
  HIPCHECK(hipStreamSynchronize(stream));
  if (ms_best) *ms_best = best;
  return st;
}

amr_status amr_regrid_fill(const amr_table* old_t, const double* U_old, amr_table* t, double* U,
                           hipStream_t stream) {
  if (!old_t || !U_old || !t || !U || old_t == t || old_t->ph.nvar != t->ph.nvar || old_t->ph.ndim != t->ph.ndim)
    return AMR_EINVAL;
  const int nd = t->ph.ndim;
  std::vector<CopyOp> cops;
  std::vector<ProlongOp> pops;
  std::vector<int> cfirst(t->max_level + 2, 0), pfirst(t->max_level + 2, 0);
  for (int l = 0; l <= t->max_level; ++l) {
    cfirst[l] = (int)cops.size();
    pfirst[l] = (int)pops.size();
    for (size_t p = 0; p < t->desc.size(); ++p) {
      const amr_patch_desc& D = t->desc[p];
      if (D.level != l) continue;
      std::vector<char> need((size_t)D.n[0] * D.n[1] * D.n[2], 1);
      for (size_t q = 0; q < old_t->desc.size(); ++q) {
        const amr_patch_desc& Q = old_t->desc[q];
        if (Q.level != l) continue;
        CopyOp op{};
        op.dst = (int)p;
        op.src = (int)q;
        bool empty = false;
        for (int e = 0; e < 3; ++e) {
          const int lo = std::max(D.lo[e], Q.lo[e]), hi = std::min(D.lo[e] + D.n[e], Q.lo[e] + Q.n[e]);
          if (e >= nd) {
            op.lo[e] = 0;
            op.sz[e] = 1;
            op.sh[e] = 0;
            continue;
          }
          if (hi <= lo) {
            empty = true;
            break;
          }
          op.lo[e] = lo - D.lo[e];
          op.sz[e] = hi - lo;
          op.sh[e] = D.lo[e] - Q.lo[e];
        }
        if (empty) continue;
        for (int k = 0; k < op.sz[2]; ++k)
          for (int j = 0; j < op.sz[1]; ++j)
            for (int i = 0; i < op.sz[0]; ++i)
              need[((size_t)(op.lo[2] + k) * D.n[1] + op.lo[1] + j) * D.n[0] + op.lo[0] + i] = 0;
        cops.push_back(op);
      }
      bool any = false;
      for (char c : need) any = any || c;
      if (!any) continue;
      if (l == 0) return AMR_EINVAL;  // a new root cell that no old root patch holds
      // the rest is prolonged from the new table's level l-1: boxes of it under each coarse patch
      for (size_t q = 0; q < t->desc.size(); ++q) {
        const amr_patch_desc& Q = t->desc[q];
        if (Q.level != l - 1) continue;
        int ilo[3], isz[3];  // part of D under Q, D-local
        bool empty = false;
        for (int e = 0; e < 3; ++e) {
          if (e >= nd) {
            ilo[e] = 0;
            isz[e] = 1;
            continue;
          }
          const int lo = std::max(D.lo[e], 2 * Q.lo[e]), hi = std::min(D.lo[e] + D.n[e], 2 * (Q.lo[e] + Q.n[e]));
          if (hi <= lo) {
            empty = true;
            break;
          }
          ilo[e] = lo - D.lo[e];
          isz[e] = hi - lo;
        }
        if (empty) continue;
        std::vector<char> sub((size_t)isz[0] * isz[1] * isz[2]);
        for (int k = 0; k < isz[2]; ++k)
          for (int j = 0; j < isz[1]; ++j)
            for (int i = 0; i < isz[0]; ++i) {
              char& m = need[((size_t)(ilo[2] + k) * D.n[1] + ilo[1] + j) * D.n[0] + ilo[0] + i];
              sub[((size_t)k * isz[1] + j) * isz[0] + i] = m;
              m = 0;
            }
        cover_boxes(isz, sub, [&](const int lo[3], const int sz[3]) {
          ProlongOp op{};
          op.dst = (int)p;
          op.src = (int)q;
          for (int e = 0; e < 3; ++e) {
            op.lo[e] = ilo[e] + lo[e];
            op.sz[e] = sz[e];
            op.foff[e] = e < nd ? D.lo[e] : 0;
            op.clo[e] = e < nd ? Q.lo[e] : 0;
          }
          pops.push_back(op);
        });
      }
      amr_status bad = AMR_OK;
      for (char c : need)
        if (c) bad = AMR_EINVAL;  // a fine cell over no coarse patch
      if (bad != AMR_OK) return bad;
    }
  }
  cfirst[t->max_level + 1] = (int)cops.size();
  pfirst[t->max_level + 1] = (int)pops.size();
  // device copies of the op lists and their work lists (freed when the fill has run)
  std::vector<Seg> segs;
  std::vector<int> blk;
  std::vector<WorkList> wc(t->max_level + 1), wp(t->max_level + 1);
  for (int l = 0; l <= t->max_level; ++l) {
    wc[l] = add_work(segs, blk, cops.data() + cfirst[l], cfirst[l + 1] - cfirst[l]);
    wp[l] = add_work(segs, blk, pops.data() + pfirst[l], pfirst[l + 1] - pfirst[l]);
  }
  CopyOp* cops_d = nullptr;
  ProlongOp* pops_d = nullptr;
  Seg* segs_d = nullptr;
  int* blk_d = nullptr;
  amr_status st = AMR_OK;
  auto up = [&](auto** dst, const auto& v) -> bool {
    if (v.empty()) return true;
    using T = typename std::remove_reference<decltype(v)>::type::value_type;
    if (hipMalloc(dst, sizeof(T) * v.size()) != hipSuccess) return false;
    return hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice) == hipSuccess;
  };
  if (!up(&cops_d, cops) || !up(&pops_d, pops) || !up(&segs_d, segs) || !up(&blk_d, blk)) st = AMR_ENOMEM;
  for (int l = 0; l <= t->max_level && st == AMR_OK; ++l) {
    const Work w1{segs_d, blk_d + wc[l].blk_base, wc[l].nblk, 0};
    if (wc[l].nblk > 0 && launch_copy_cells_x(stream, cops_d + cfirst[l], w1, t->pdev_d, old_t->pdev_d, U, U_old,
                                              t->ph.nvar) != hipSuccess)
      st = AMR_EHIP;
    const Work w2{segs_d, blk_d + wp[l].blk_base, wp[l].nblk, 0};
    if (st == AMR_OK && wp[l].nblk > 0 &&
        launch_prolong(stream, pops_d + pfirst[l], w2, t->pdev_d, U, U, U, 0.0, nd, t->ph.nvar) != hipSuccess)
      st = AMR_EHIP;
    // this level's ghosts, read by its children's prolongation stencils
    if (st == AMR_OK && l < t->max_level) {
      st = enqueue_ghosts(t, U, U, l, 0.0, stream, U);
      if (st == AMR_OK && t->has_kids[l] && t->w_phys[l].nblk > 0 &&
          launch_phys(stream, t->phys_d + t->phys_first[l], work_of(t, t->w_phys[l]), t->pdev_d, U, t->ph.nvar) !=
              hipSuccess)
        st = AMR_EHIP;
    }
  }
  if (hipStreamSynchronize(stream) != hipSuccess && st == AMR_OK) st = AMR_EHIP;
  for (void* q : {(void*)cops_d, (void*)pops_d, (void*)segs_d, (void*)blk_d})
    if (q) (void)hipFree(q);
  return st;
}

int64_t amr_table_cells(const amr_table* t, int32_t level) {
  if (!t || level < -1 || level > t->max_level) return -1;
  int64_t n = 0;
  for (const PatchDev& P : t->pdev)
    if (level < 0 || P.level == level) n += (int64_t)P.n[0] * P.n[1] * P.n[2];
  return n;
}

amr_status amr_flag_cells(amr_table* t, double* U, int32_t level, double eps, uint8_t* flags_dev,
                          hipStream_t stream) {
  if (!t || !U || !flags_dev || level < -1 || level > t->max_level || !(eps >= 0.0 && eps < 1e300))
    return AMR_EINVAL;
  auto it = t->cell_lists.find(level);
  if (it == t->cell_lists.end()) {
    CellList cl;
    std::vector<int> pl;
    std::vector<int64_t> co{0};
    for (size_t p = 0; p < t->pdev.size(); ++p) {
      const PatchDev& P = t->pdev[p];
      if (level >= 0 && P.level != level) continue;
      pl.push_back((int)p);
      co.push_back(co.back() + (int64_t)P.n[0] * P.n[1] * P.n[2]);
    }
    cl.npl = (int)pl.size();
    cl.ncells = co.back();
    if (cl.npl > 0) {
      if (hipMalloc(&cl.plist, sizeof(int) * pl.size()) != hipSuccess) return AMR_ENOMEM;
      if (hipMalloc(&cl.cofs, sizeof(int64_t) * co.size()) != hipSuccess) {
        (void)hipFree(cl.plist);
        return AMR_ENOMEM;
      }
      HIPCHECK(hipMemcpy(cl.plist, pl.data(), sizeof(int) * pl.size(), hipMemcpyHostToDevice));
      HIPCHECK(hipMemcpy(cl.cofs, co.data(), sizeof(int64_t) * co.size(), hipMemcpyHostToDevice));
    }
    it = t->cell_lists.emplace(level, cl).first;
  }
  const CellList& cl = it->second;
  if (cl.ncells == 0) return AMR_OK;
  // current ghosts of the flagged levels and of every coarser level (prolongation stencils)
  const int lmax = level < 0 ? t->max_level : level;
  for (int l = 0; l <= lmax; ++l) {
    amr_status st = enqueue_ghosts(t, U, U, l, 1.0, stream, U);  // coarse data: U itself
    if (st != AMR_OK) return st;
    if (l < t->max_level && t->has_kids[l] && t->w_phys[l].nblk > 0)
      HIPCHECK(launch_phys(stream, t->phys_d + t->phys_first[l], work_of(t, t->w_phys[l]), t->pdev_d, U, t->ph.nvar));
  }
  HIPCHECK(launch_flag_cells(stream, cl.plist, cl.cofs, cl.npl, cl.ncells, t->pdev_d, U, eps, flags_dev,
                             t->ph.ndim));
  return AMR_OK;
}

}  // extern "C"
