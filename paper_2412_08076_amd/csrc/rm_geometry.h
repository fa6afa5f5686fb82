// Host-side geometry of the temporal-blocked FP32 sweeps: the kernel variants, row and
// column windows with their halos, the cost model that picks a configuration before
// tuning, and the tile tables the kernels walk.  Plain C++ (no HIP), so that the
// planning logic can be built and checked on its own, with sanitizers, on any host.
#pragma once

#include <algorithm>
#include <array>
#include <cstdint>
#include <vector>

namespace rmk {

// Tiled kernel variants: strips of R rows (extended tile height 8R) and an LDS row
// stride LW (extended tile width CW <= LW - 2, CW a multiple of 8 chosen at launch; 8 CW
// threads per workgroup).
struct BlockVariant {
  int r, lw;
};
constexpr int kNumBlockVariants = 9;
inline constexpr BlockVariant kBlockVariants[kNumBlockVariants] = {
    {8, 66},    // up to 64 x 64 points
    {16, 66},   // up to 64 x 128
    {8, 130},   // up to 128 x 64
    {13, 66},   // up to 64 x 104
    {16, 130},  // up to 128 x 128
    {12, 98},   // up to 96 x 96
    {13, 106},  // up to 104 x 104
    {32, 66},   // up to 64 x 256: one tile covers n <= 256 vertically (no y halo)
    {32, 98},   // up to 96 x 256
};

// Row-streaming kernel: whole rows of up to kStreamMaxN columns per workgroup, up to
// kStreamMaxT steps per launch; its reverse steps up to kAdjMaxT per launch for
// n <= kAdjStreamMaxN.
constexpr int kStreamMaxN = 1024;
constexpr int kStreamMaxT = 8;
constexpr int kAdjStreamMaxN = 512;
constexpr int kAdjMaxT = 3;

// One extended tile of a block table: origin (x0, y0) of its window in instance
// coordinates, the slot of its residual partial, and the owned rectangle
// [ox0, ox1) x [oy0, oy1) it stores.  inst < 0 marks padding.
struct BTile {
  int32_t inst, x0, y0, slot;
  int32_t ox0, ox1, oy0, oy1;
};

// One workgroup of the mixed-size row-pipeline launch: `count` row windows of one size
// class (tiles first .. first + count - 1 of the launch's tile list, each window L rows
// high), in 1024 / nt sub-groups of nt = 64 ceil(n / 64) threads; sub-groups from
// `count` on have no window and only keep the workgroup's barriers.  cls < 0 marks
// padding.
struct MGroup {
  int32_t first, count, cls, L;
  int32_t nt, pad0, pad1, pad2;
};
constexpr int kMixedThreads = 1024;

}  // namespace rmk

namespace rmgeo {

// Boundary-aware 1D tiling of [0, n) by windows of length len: a window edge on
// the domain boundary needs no halo (the zero border of the LDS tile and the
// zeros published outside the interior are the Dirichlet condition); interior
// edges overlap the neighbouring window by h.  Returns {window start, owned lo,
// owned hi} per window, or nothing when len is too short for the halo.
inline std::vector<std::array<int, 3>> partition(int n, int len, int h) {
  std::vector<std::array<int, 3>> out;
  int o = 0;
  while (true) {
    const int start = o > 0 ? o - h : 0;
    if (start + len >= n) {
      out.push_back({start, o, n});
      break;
    }
    const int hi = start + len - h;
    if (hi <= o) return {};
    out.push_back({start, o, hi});
    o = hi;
  }
  return out;
}

// Kernel shapes: the tiled variants 0 .. kNumBlockVariants - 1, then the row-streaming
// kernel, whose "width" is the height of its row windows (whole rows across).
constexpr int kStreamShape = rmk::kNumBlockVariants;
constexpr int kNumShapes = kStreamShape + 1;

// Geometry of a class (n, variant v, steps per launch T, width cw): the tiles
// across and down.  An instance that fits in one window needs no halo; otherwise
// the halo is T + 1 (one ring more than T steps need, so the residual of the
// final iterate can be formed in the same launch).
inline bool class_geometry(int n, int v, int T, int cw, int& tx, int& ty) {
  if (v == kStreamShape) {
    if (n > rmk::kStreamMaxN || T < 1 || T > rmk::kStreamMaxT || cw < 1) return false;
    tx = 1;
    ty = (int)partition(n, cw, T + 1).size();
    return ty > 0;
  }
  if (v < 0 || v >= rmk::kNumBlockVariants || T < 1) return false;
  const rmk::BlockVariant& bv = rmk::kBlockVariants[v];
  if (cw < 8 || cw % 8 != 0 || cw + 2 > bv.lw) return false;
  const int eh = 8 * bv.r;
  const int h = T + 1;
  tx = (int)partition(n, cw, h).size();
  ty = (int)partition(n, eh, h).size();
  return tx > 0 && ty > 0;
}

// Cost model used before any tuning: the larger of an arithmetic bound
// (redundant halo work included) and an HBM bound (load u, v, f on the extended
// tile, store u, v on the owned one, once per T steps), per inner step.
inline double model_cost(int n, int v, int T, int cw, int count) {
  int tx, ty;
  if (!class_geometry(n, v, T, cw, tx, ty)) return 1e300;
  if (v == kStreamShape) {
    // whole rows in one workgroup: only the row windows overlap; a grid of fewer
    // waves than SIMDs leaves the rest idle
    const int nw = (n + 63) / 64;
    const double rows = std::min<double>((double)ty * cw, (double)n + 2.0 * (ty - 1) * (T + 1));
    const double ext = rows * 64.0 * nw;
    const double fill = std::min(1.0, (double)count * ty * nw / 1024.0);
    const double compute = ext / 2.4e12 / fill;
    const double memory = (12.0 * rows * n + 8.0 * n * (double)n) / T / 5.0e12;
    return std::max(compute, memory) + 4e-6 / T / 256.0;
  }
  const double ext = (double)tx * ty * cw * (double)(8 * rmk::kBlockVariants[v].r);
  const double own = (double)n * n;
  const double compute = ext / 1.6e12;
  const double memory = (12.0 * ext + 8.0 * own) / T / 5.0e12;
  // measured on MI355X: widths that are not multiples of 32 make waves straddle
  // strips (slower LDS and global access), and workgroups wider than 64 columns
  // fit fewer per CU
  const double shape_penalty = (cw % 32 != 0 ? 1.3 : 1.0) * (cw > 64 ? 1.15 : 1.0);
  return std::max(compute, memory) * shape_penalty + 4e-6 / T / 256.0;
}

// Steps per launch tried by the tuner and the cost model.
inline constexpr int kTs[] = {2, 4, 8, 16, 32};

// Tile widths worth trying for (n, v, T): for the few smallest tile counts k
// across, the narrowest multiple of 8 that covers n.
inline std::vector<int> candidate_widths(int n, int v, int T) {
  std::vector<int> out;
  if (v == kStreamShape) {
    // windows for 1 to 10, 12 or 16 row segments per instance
    const int h = T + 1;
    for (int S : {1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 12, 16}) {
      const int len = S == 1 ? n : (n + 2 * (S - 1) * h + S - 1) / S;
      int tx, ty;
      if (class_geometry(n, v, T, len, tx, ty) && ty == S && std::find(out.begin(), out.end(), len) == out.end())
        out.push_back(len);
    }
    return out;
  }
  const int lw = rmk::kBlockVariants[v].lw;
  for (int cw = 8; cw + 2 <= lw && (int)out.size() < 64; cw += 8) {
    int tx, ty;
    if (!class_geometry(n, v, T, cw, tx, ty)) continue;
    // keep cw only if it is the narrowest width with this tile count
    int tx2 = -1, ty2;
    if (cw > 8 && class_geometry(n, v, T, cw - 8, tx2, ty2) && tx2 == tx) continue;
    out.push_back(cw);
  }
  // favour the widest few (fewest tiles) and widths that are multiples of 32
  std::vector<int> keep;
  for (auto it = out.rbegin(); it != out.rend() && (int)keep.size() < 3; ++it) keep.push_back(*it);
  for (int w : out)
    if (w % 32 == 0 && std::find(keep.begin(), keep.end(), w) == keep.end()) keep.push_back(w);
  for (int w : {32, 64, 96, 128}) {
    int tx, ty;
    if (class_geometry(n, v, T, w, tx, ty) && std::find(keep.begin(), keep.end(), w) == keep.end())
      keep.push_back(w);
  }
  return keep;
}

inline void default_class_config(int n, int count, int& shape, int& T, int& cw, int nshapes = kNumShapes) {
  double best = 1e301;
  shape = 0;
  T = 2;
  cw = 64;
  for (int v = 0; v < nshapes; ++v)
    for (int t : kTs)
      for (int w : candidate_widths(n, v, t)) {
        const double c = model_cost(n, v, t, w, count);
        if (c < best * 0.999) {
          best = c;
          shape = v;
          T = t;
          cw = w;
        }
      }
}

// Row-window height of the reverse-step table of a class: enough windows per instance
// for about two waves per SIMD, each window at least four overlaps high.
inline int reverse_window(int n, int count) {
  const int h = rmk::kAdjMaxT + 1;
  const int nw = (n + 63) / 64;
  int want = (2048 + count * nw - 1) / std::max(1, count * nw);
  want = std::max(1, std::min(16, want));
  for (int S = want; S > 1; --S) {
    const int len = (n + 2 * (S - 1) * h + S - 1) / S;
    if (len >= 4 * h && (int)partition(n, len, h).size() == S) return len;
  }
  return n;
}

// Tile table of one configuration of a size class (instances `insts` of size n): every
// tile of every instance, the residual slots of an instance numbered in row-major order
// of its tiles from `slot` on (advanced), its slot range in ranges[2b], ranges[2b + 1],
// and padding tiles (inst = -1, slots after all others).  Row windows are listed
// instance by instance, padded to a multiple of 8.  A tiled table is eight parts of
// equal length, one per XCD under the block remap: the tile rows of the class's k-th
// instance are cut into eight bands of consecutive rows, band j going to part
// (j + k) mod 8.  Any few instances still iterating then keep all eight XCDs busy (an
// instance-major table put a lone instance's tiles on one or two of them), and vertical
// neighbours mostly share an L2.  False for an invalid configuration.
inline bool make_tiles(int n, const std::vector<int>& insts, int shape, int T, int cw, int& slot,
                       std::vector<int>& ranges, std::vector<rmk::BTile>& out) {
  int tx, ty;
  if (!class_geometry(n, shape, T, cw, tx, ty)) return false;
  const bool stream = shape == kStreamShape;
  const int eh = stream ? cw : 8 * rmk::kBlockVariants[shape].r;
  const auto px = stream ? std::vector<std::array<int, 3>>{{0, 0, n}} : partition(n, cw, T + 1);
  const auto py = partition(n, eh, T + 1);
  out.clear();
  if (stream) {
    for (int b : insts) {
      ranges[2 * b] = slot;
      for (const auto& y : py)
        for (const auto& x : px) out.push_back(rmk::BTile{b, x[0], y[0], slot++, x[1], x[2], y[1], y[2]});
      ranges[2 * b + 1] = slot;
    }
    while (out.size() % 8 != 0) out.push_back(rmk::BTile{-1, 0, 0, slot++, 0, 0, 0, 0});
    return true;
  }
  const int rows = (int)py.size(), cols = (int)px.size();
  std::vector<std::vector<rmk::BTile>> part(8);
  for (size_t k = 0; k < insts.size(); ++k) {
    const int b = insts[k];
    ranges[2 * b] = slot;
    for (int j = 0; j < 8; ++j) {
      auto& dst = part[(j + k) % 8];
      for (int r = j * rows / 8; r < (j + 1) * rows / 8; ++r)
        for (int c = 0; c < cols; ++c) {
          const auto& x = px[c];
          const auto& y = py[r];
          dst.push_back(rmk::BTile{b, x[0], y[0], slot + r * cols + c, x[1], x[2], y[1], y[2]});
        }
    }
    slot += rows * cols;
    ranges[2 * b + 1] = slot;
  }
  size_t per = 0;
  for (const auto& q : part) per = std::max(per, q.size());
  for (auto& q : part) {
    while (q.size() < per) q.push_back(rmk::BTile{-1, 0, 0, slot++, 0, 0, 0, 0});
    out.insert(out.end(), q.begin(), q.end());
  }
  return true;
}

// Groups of the mixed-size launch over the row windows of several size classes.  Each
// class contributes its tile table `tiles` (padding entries skipped), whose windows
// are `wlen` rows high (the last of an instance may be lower); the tiles go to `all`
// class by class, and within a class height by height.  Windows of one class with the
// same height share a workgroup, up to kMixedThreads / (64 ceil(n / 64)) of them.
// The list is eight equal parts, one per XCD, each with an eighth of every class's
// groups (padding groups, cls = -1, even them out), the largest n first.
struct MixedClass {
  int cls, n, wlen;
  const std::vector<rmk::BTile>* tiles;
};

inline int window_rows(int n, int wlen, const rmk::BTile& t) { return std::min(n, t.y0 + wlen) - t.y0; }

inline bool make_groups(const std::vector<MixedClass>& classes, std::vector<rmk::BTile>& all,
                        std::vector<rmk::MGroup>& groups) {
  all.clear();
  groups.clear();
  std::vector<std::vector<rmk::MGroup>> per(classes.size());
  for (size_t k = 0; k < classes.size(); ++k) {
    const MixedClass& c = classes[k];
    if (c.n < 1 || c.n > rmk::kStreamMaxN || c.wlen < 1 || c.tiles == nullptr) return false;
    const int nt = 64 * ((c.n + 63) / 64), G = rmk::kMixedThreads / nt;
    // windows of this class by height (heights in order of first appearance)
    std::vector<std::pair<int, std::vector<rmk::BTile>>> byL;
    for (const rmk::BTile& t : *c.tiles) {
      if (t.inst < 0) continue;
      if (t.y0 < 0 || t.y0 >= c.n) return false;
      const int L = window_rows(c.n, c.wlen, t);
      auto it = std::find_if(byL.begin(), byL.end(), [&](const auto& e) { return e.first == L; });
      if (it == byL.end()) {
        byL.push_back({L, {}});
        it = byL.end() - 1;
      }
      it->second.push_back(t);
    }
    // appended height by height, so that the windows of a group are consecutive
    for (const auto& e : byL)
      for (size_t i = 0; i < e.second.size(); i += G) {
        const int cnt = (int)std::min<size_t>(G, e.second.size() - i);
        per[k].push_back(rmk::MGroup{(int32_t)all.size(), cnt, c.cls, e.first, nt, 0, 0, 0});
        all.insert(all.end(), e.second.begin() + i, e.second.begin() + i + cnt);
      }
  }
  // The launch hands XCD k the k-th eighth of the list (xcd_remap): each eighth takes
  // every eighth group of every class (groups k, k + 8, ... of it, padded to the same
  // count), larger classes first, so each XCD gets an equal share of every class and
  // starts its longest workgroups first.
  std::vector<size_t> order(classes.size());
  for (size_t k = 0; k < order.size(); ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return classes[a].n > classes[b].n; });
  const rmk::MGroup pad{0, 0, -1, 0, 64, 0, 0, 0};
  for (int x = 0; x < 8; ++x)
    for (size_t k : order) {
      const size_t q = (per[k].size() + 7) / 8;
      for (size_t j = 0; j < q; ++j) {
        const size_t i = (size_t)x + 8 * j;
        groups.push_back(i < per[k].size() ? per[k][i] : pad);
      }
    }
  return true;
}

}  // namespace rmgeo
