// amr_cluster.cpp - host-side clustering of refinement flags into the patches of the
// next finer level (factor-2 refinement), for a dynamic block-structured hierarchy
// (Sec. 3: the paper builds its hierarchy on the host).
//
// The rule is the one that places the deep-AMR configuration's levels:
//   * every flagged level-l cell, dilated by one cell along each axis, marks the
//     fine bricks (brick^3 fine cells, aligned on the fine grid) holding its children;
//   * a marked brick is kept if its footprint on level l, dilated by one coarse
//     cell and clipped to the domain, lies on level l (proper nesting: the fine
//     patches' ghost cells and their prolongation stencils stay on level l);
//   * kept bricks are grouped by aligned blocks of block^3 fine cells; a group
//     becomes its bounding box when that box is properly nested, else each half-block
//     sub-group its bounding box, else single bricks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <map>
#include <set>
#include <vector>

#include "../../include/amr_hydro.h"

namespace {

using Key = std::array<int, 3>;

}  // namespace

extern "C" amr_status amr_cluster_flags(const amr_patch_desc* patches, int32_t npatch, int32_t ndim,
                                        const int32_t domain[3], int32_t level, const uint8_t* flags,
                                        int32_t brick, int32_t block, int32_t* boxes, int32_t max_boxes,
                                        int32_t* nboxes) {
  if (!patches || npatch < 1 || ndim < 1 || ndim > 3 || !domain || level < 0 || !flags || !nboxes || brick < 1 ||
      block < brick || block % brick || (block / brick) % 2 || max_boxes < 0 || (max_boxes > 0 && !boxes))
    return AMR_EINVAL;
  int N[3], bd[3];
  for (int d = 0; d < 3; ++d) {
    // (level-l extents must fit an int32 index)
    if (d < ndim && (domain[d] < 1 || level > 30 || ((int64_t)domain[d] << level) > INT32_MAX)) return AMR_EINVAL;
    N[d] = d < ndim ? domain[d] << level : 1;
    bd[d] = d < ndim ? brick : 1;
  }
  const int per = block / brick;
  // level-l coverage as bricks of level-l cells; every level-l patch must be brick-aligned
  std::set<Key> cov;
  for (int p = 0; p < npatch; ++p) {
    const amr_patch_desc& D = patches[p];
    if (D.level != level) continue;
    for (int d = 0; d < ndim; ++d)
      if (D.lo[d] % brick || D.n[d] % brick) return AMR_EINVAL;
    for (int k = D.lo[2] / bd[2]; k < (D.lo[2] + D.n[2]) / bd[2]; ++k)
      for (int j = D.lo[1] / bd[1]; j < (D.lo[1] + D.n[1]) / bd[1]; ++j)
        for (int i = D.lo[0] / bd[0]; i < (D.lo[0] + D.n[0]) / bd[0]; ++i) cov.insert(Key{i, j, k});
  }
  // fine box [lo, hi) nested: its level-l footprint dilated by one cell, clipped to the domain,
  // lies in level-l bricks
  auto nested = [&](const int lo[3], const int hi[3]) {
    int blo[3], bhi[3];
    for (int d = 0; d < 3; ++d) {
      if (d < ndim) {
        const int clo = std::max(lo[d] / 2 - 1, 0), chi = std::min((hi[d] + 1) / 2 + 1, N[d]);
        blo[d] = clo / bd[d];
        bhi[d] = (chi - 1) / bd[d] + 1;
      } else {
        blo[d] = 0;
        bhi[d] = 1;
      }
    }
    for (int k = blo[2]; k < bhi[2]; ++k)
      for (int j = blo[1]; j < bhi[1]; ++j)
        for (int i = blo[0]; i < bhi[0]; ++i)
          if (!cov.count(Key{i, j, k})) return false;
    return true;
  };
  // marked fine bricks
  std::set<Key> cand;
  int64_t w = 0;
  for (int p = 0; p < npatch; ++p) {
    const amr_patch_desc& D = patches[p];
    if (D.level != level) continue;
    for (int k = 0; k < D.n[2]; ++k)
      for (int j = 0; j < D.n[1]; ++j)
        for (int i = 0; i < D.n[0]; ++i, ++w) {
          if (!flags[w]) continue;
          const int c[3] = {D.lo[0] + i, D.lo[1] + j, D.lo[2] + k};
          for (int a = 0; a < ndim; ++a)
            for (int dd = -1; dd <= 1; ++dd) {
              int q[3] = {c[0], c[1], c[2]};
              q[a] += dd;
              if (q[a] < 0 || q[a] >= N[a]) continue;
              Key b;
              for (int d = 0; d < 3; ++d) b[d] = d < ndim ? (2 * q[d]) / bd[d] : 0;
              cand.insert(b);
            }
        }
  }
  std::map<Key, std::vector<Key>> groups;
  for (const Key& b : cand) {
    const int lo[3] = {b[0] * bd[0], b[1] * bd[1], b[2] * bd[2]};
    const int hi[3] = {lo[0] + bd[0], lo[1] + bd[1], lo[2] + bd[2]};
    if (!nested(lo, hi)) continue;
    Key g;
    for (int d = 0; d < 3; ++d) g[d] = d < ndim ? b[d] / per : 0;
    groups[g].push_back(b);
  }
  std::vector<std::array<int, 6>> out;  // lo[3], hi[3]
  auto emit = [&](const std::vector<Key>& bs) {
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      int mn = bs[0][d], mx = bs[0][d];
      for (const Key& b : bs) {
        mn = std::min(mn, b[d]);
        mx = std::max(mx, b[d]);
      }
      lo[d] = mn * bd[d];
      hi[d] = (mx + 1) * bd[d];
    }
    if (!nested(lo, hi)) return false;
    out.push_back({lo[0], lo[1], lo[2], hi[0], hi[1], hi[2]});
    return true;
  };
  for (auto& kv : groups) {
    std::vector<Key>& bs = kv.second;
    std::sort(bs.begin(), bs.end());
    if (emit(bs)) continue;
    std::map<Key, std::vector<Key>> sub;
    for (const Key& b : bs) {
      Key s;
      for (int d = 0; d < 3; ++d) s[d] = d < ndim ? (b[d] % per) / (per / 2) : 0;
      sub[s].push_back(b);
    }
    for (auto& sk : sub) {
      if (emit(sk.second)) continue;
      for (const Key& b : sk.second) emit(std::vector<Key>{b});
    }
  }
  std::sort(out.begin(), out.end());
  *nboxes = (int32_t)out.size();
  if ((int32_t)out.size() > max_boxes) return AMR_EINVAL;
  for (size_t i = 0; i < out.size(); ++i)
    for (int d = 0; d < 3; ++d) {
      boxes[6 * i + d] = out[i][d];
      boxes[6 * i + 3 + d] = out[i][3 + d] - out[i][d];
    }
  return AMR_OK;
}
