// Checks of the host planning logic of the FP32 sweeps (rm_geometry.h), built with
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_host_sanitized.py.
// For many sizes, kernel shapes, steps per launch and widths:
//   - the windows of a 1D partition own disjoint, contiguous ranges that cover [0, n), and
//     every owned edge inside the domain lies at least the halo h inside its window;
//   - every configuration the cost model or the tuner's candidate list proposes is valid;
//   - a tile table owns every point of every instance exactly once, each owned rectangle
//     lies in its tile's window with the halo, residual slots are numbered consecutively,
//     the per-instance slot ranges partition them and the table is padded to a multiple of 8;
//   - the reverse-step windows split n into the number of windows they promise;
//   - the groups of the mixed-size launch hold every window of every class exactly once,
//     each group windows of one class and one height, no more than its workgroup holds;
//     the list is eight equal parts (one per XCD), each with its class's groups larger
//     classes first and every class's groups spread over the parts within one.
// Exit status 0 when every check holds; the first failure is printed.
#include <cstdio>
#include <algorithm>
#include <array>
#include <cstdlib>
#include <vector>

#include "rm_geometry.h"

using namespace rmgeo;

static int failures = 0;
#define CHECK(cond, ...)                                   \
  do {                                                     \
    if (!(cond)) {                                         \
      std::fprintf(stderr, "check failed: %s: ", #cond);  \
      std::fprintf(stderr, __VA_ARGS__);                   \
      std::fprintf(stderr, "\n");                          \
      if (++failures > 20) std::exit(1);                   \
    }                                                      \
  } while (0)

static void check_partition(int n, int len, int h) {
  const auto w = partition(n, len, h);
  if (w.empty()) {
    // only when the window is too short for the halo (or n is tiny: one window)
    CHECK(len <= 2 * h || len < n, "n=%d len=%d h=%d: empty partition", n, len, h);
    return;
  }
  int next = 0;
  for (size_t k = 0; k < w.size(); ++k) {
    const int start = w[k][0], lo = w[k][1], hi = w[k][2];
    CHECK(lo == next, "n=%d len=%d h=%d: window %zu owns from %d, expected %d", n, len, h, k, lo, next);
    CHECK(lo < hi, "n=%d len=%d h=%d: window %zu owns nothing", n, len, h, k);
    CHECK(start >= 0 && start <= lo, "n=%d len=%d h=%d: window %zu starts at %d", n, len, h, k, start);
    CHECK(lo == 0 || lo - start >= h, "n=%d len=%d h=%d: low halo %d", n, len, h, lo - start);
    const int end = std::min(n, start + len);
    CHECK(hi <= end, "n=%d len=%d h=%d: window %zu owns beyond its end", n, len, h, k);
    CHECK(hi == n || end - hi >= h, "n=%d len=%d h=%d: high halo %d", n, len, h, end - hi);
    next = hi;
  }
  CHECK(next == n, "n=%d len=%d h=%d: partition ends at %d", n, len, h, next);
}

static void check_table(int n, int count, int shape, int T, int cw) {
  int tx = 0, ty = 0;
  if (!class_geometry(n, shape, T, cw, tx, ty)) return;
  std::vector<int> insts;
  const int B = count + 2;  // the class holds every other instance of a larger batch
  for (int b = 1; b < B; b += 2) insts.push_back(b);
  std::vector<int> ranges(2 * (size_t)B, -7);
  std::vector<rmk::BTile> t;
  int slot = 5;
  const bool ok = make_tiles(n, insts, shape, T, cw, slot, ranges, t);
  CHECK(ok, "n=%d shape=%d T=%d cw=%d: valid geometry but no table", n, shape, T, cw);
  if (!ok) return;
  CHECK(t.size() % 8 == 0, "table length %zu", t.size());
  CHECK((int)t.size() >= (int)insts.size() * tx * ty, "table too short");
  const bool stream = shape == kStreamShape;
  const int eh = stream ? cw : 8 * rmk::kBlockVariants[shape].r;
  const int ew = stream ? n : cw;
  const int h = T + 1;
  int expect_slot = 5;
  std::vector<int> owner((size_t)n * n);
  for (int b : insts) {
    CHECK(ranges[2 * b] == expect_slot, "instance %d slots start at %d", b, ranges[2 * b]);
    std::fill(owner.begin(), owner.end(), 0);
    // the instance's slots are its range, each once, in row-major order of its tiles
    std::vector<std::array<int, 3>> mine;  // (slot, y0, x0)
    for (const auto& tl : t)
      if (tl.inst == b) mine.push_back({tl.slot, tl.y0, tl.x0});
    std::sort(mine.begin(), mine.end());
    for (size_t k = 0; k < mine.size(); ++k) {
      CHECK(mine[k][0] == expect_slot + (int)k, "slot %d, expected %d", mine[k][0], expect_slot + (int)k);
      if (k > 0)
        CHECK(mine[k][1] > mine[k - 1][1] || (mine[k][1] == mine[k - 1][1] && mine[k][2] > mine[k - 1][2]),
              "instance %d: slots not in row-major order of its tiles", b);
    }
    for (const auto& tl : t) {
      if (tl.inst != b) continue;
      ++expect_slot;
      CHECK(tl.x0 >= 0 && tl.y0 >= 0, "negative origin");
      CHECK(tl.ox0 >= tl.x0 && tl.ox1 <= std::min(n, tl.x0 + ew), "owned columns outside the window");
      CHECK(tl.oy0 >= tl.y0 && tl.oy1 <= std::min(n, tl.y0 + eh), "owned rows outside the window");
      CHECK(tl.ox0 == 0 || tl.ox0 - tl.x0 >= h, "column halo %d < %d", tl.ox0 - tl.x0, h);
      CHECK(tl.oy0 == 0 || tl.oy0 - tl.y0 >= h, "row halo %d < %d", tl.oy0 - tl.y0, h);
      CHECK(tl.ox1 == n || std::min(n, tl.x0 + ew) - tl.ox1 >= h, "east halo");
      CHECK(tl.oy1 == n || std::min(n, tl.y0 + eh) - tl.oy1 >= h, "north halo");
      for (int y = tl.oy0; y < tl.oy1; ++y)
        for (int x = tl.ox0; x < tl.ox1; ++x) ++owner[(size_t)y * n + x];
    }
    CHECK(ranges[2 * b + 1] == expect_slot, "instance %d slots end at %d", b, ranges[2 * b + 1]);
    for (size_t k = 0; k < owner.size(); ++k)
      if (owner[k] != 1) {
        CHECK(owner[k] == 1, "n=%d shape=%d T=%d cw=%d: point %zu owned %d times", n, shape, T, cw, k, owner[k]);
        break;
      }
  }
  for (int b = 0; b < B; b += 2) CHECK(ranges[2 * b] == -7, "an instance outside the class got a range");
  std::vector<int> pad;
  for (const auto& tl : t)
    if (tl.inst < 0) pad.push_back(tl.slot);
  std::sort(pad.begin(), pad.end());
  for (int s : pad) CHECK(s == expect_slot++, "padding slot %d", s);
  CHECK(slot == expect_slot, "slot counter %d, expected %d", slot, expect_slot);
  if (!stream) {
    // eight parts of equal length (one per XCD under the block remap); an instance with
    // at least eight rows of tiles has tiles in every part
    const size_t per = t.size() / 8;
    for (int b : insts) {
      int parts = 0;
      for (int x = 0; x < 8; ++x) {
        bool any = false;
        for (size_t i = x * per; i < (x + 1) * per; ++i) any = any || t[i].inst == b;
        parts += any ? 1 : 0;
      }
      CHECK(parts == std::min(8, ty), "n=%d shape=%d: instance %d in %d of 8 parts (%d tile rows)", n, shape, b, parts, ty);
    }
  }
}

static void check_groups(const std::vector<int>& ns, const std::vector<int>& counts, int pick) {
  std::vector<std::vector<rmk::BTile>> tabs(ns.size());
  std::vector<MixedClass> mc;
  std::vector<int> wl(ns.size());
  int slot = 0, B = 0;
  for (int c : counts) B += c;
  std::vector<int> ranges(2 * (size_t)B, 0), ninst((size_t)B, 0);
  int b0 = 0;
  for (size_t k = 0; k < ns.size(); ++k) {
    const int n = ns[k];
    const auto ws = candidate_widths(n, kStreamShape, rmk::kStreamMaxT);
    if (ws.empty()) return;
    wl[k] = ws[(size_t)pick % ws.size()];
    std::vector<int> insts;
    for (int j = 0; j < counts[k]; ++j) {
      insts.push_back(b0 + j);
      ninst[(size_t)b0 + j] = n;
    }
    b0 += counts[k];
    CHECK(make_tiles(n, insts, kStreamShape, rmk::kStreamMaxT, wl[k], slot, ranges, tabs[k]), "mixed table n=%d", n);
    mc.push_back(MixedClass{(int)k, n, wl[k], &tabs[k]});
  }
  std::vector<rmk::BTile> all;
  std::vector<rmk::MGroup> g;
  CHECK(make_groups(mc, all, g), "make_groups refused valid classes");
  CHECK(g.size() % 8 == 0, "group list length %zu", g.size());
  std::vector<int> seen((size_t)slot, 0);
  std::vector<std::vector<int>> per_part(ns.size(), std::vector<int>(8, 0));
  const size_t part = g.size() / 8;
  int prev_n = 1 << 30;
  size_t covered = 0;
  for (size_t gi = 0; gi < g.size(); ++gi) {
    const auto& e = g[gi];
    if (gi % part == 0) prev_n = 1 << 30;  // a new XCD part
    if (e.cls < 0) continue;
    CHECK(e.cls < (int)ns.size(), "group class %d", e.cls);
    if (e.cls >= (int)ns.size()) continue;
    ++per_part[(size_t)e.cls][gi / part];
    const int n = ns[(size_t)e.cls];
    CHECK(n <= prev_n, "groups of a part not ordered by size: %d after %d", n, prev_n);
    prev_n = n;
    CHECK(e.nt == 64 * ((n + 63) / 64), "n=%d: sub-group of %d threads", n, e.nt);
    CHECK(e.count >= 1 && e.count * e.nt <= rmk::kMixedThreads, "n=%d: %d windows of %d threads", n, e.count, e.nt);
    CHECK(e.first >= 0 && (size_t)e.first + (size_t)e.count <= all.size(), "group tiles out of range");
    for (int j = 0; j < e.count && (size_t)(e.first + j) < all.size(); ++j) {
      const rmk::BTile& t = all[(size_t)e.first + j];
      CHECK(t.inst >= 0 && t.inst < B && ninst[(size_t)t.inst] == n, "tile of another class in a group of n=%d", n);
      CHECK(window_rows(n, wl[(size_t)e.cls], t) == e.L, "n=%d: window of %d rows in a group of %d", n,
            window_rows(n, wl[(size_t)e.cls], t), e.L);
      CHECK(e.L >= 1 && t.y0 + e.L <= n, "n=%d: window rows [%d, %d)", n, t.y0, t.y0 + e.L);
      if (t.slot >= 0 && t.slot < slot) ++seen[(size_t)t.slot];
      ++covered;
    }
  }
  CHECK(covered == all.size(), "groups cover %zu of %zu windows", covered, all.size());
  for (size_t k = 0; k < ns.size(); ++k) {
    const auto mm = std::minmax_element(per_part[k].begin(), per_part[k].end());
    CHECK(*mm.second - *mm.first <= 1, "n=%d: %d to %d groups per XCD part", ns[k], *mm.first, *mm.second);
  }
  size_t windows = 0;
  for (const auto& tab : tabs)
    for (const auto& t : tab)
      if (t.inst >= 0) {
        ++windows;
        CHECK(seen[(size_t)t.slot] == 1, "window with slot %d grouped %d times", t.slot, seen[(size_t)t.slot]);
      }
  CHECK(windows == all.size(), "%zu windows, %zu in the launch list", windows, all.size());
}

int main() {
  // 1D partitions
  for (int n = 1; n <= 300; ++n)
    for (int h = 1; h <= 9; h += 2)
      for (int len = 1; len <= n + 3; len += (len < 40 ? 1 : 7)) check_partition(n, len, h);
  for (int n : {511, 512, 1000, 1023, 1024, 2047, 4095})
    for (int h : {2, 5, 9, 17})
      for (int len = 2 * h + 1; len <= n; len += 13) check_partition(n, len, h);
  // configurations and tables
  const int sizes[] = {1, 2, 3, 7, 8, 9, 17, 31, 63, 64, 65, 100, 127, 128, 130, 200, 255, 256, 257, 300, 511, 513,
                       700, 1023, 1024};
  for (int n : sizes) {
    for (int count : {1, 3, 26}) {
      int shape = -1, T = 0, cw = 0;
      default_class_config(n, count, shape, T, cw);
      int tx, ty;
      CHECK(class_geometry(n, shape, T, cw, tx, ty), "n=%d count=%d: default configuration invalid", n, count);
      default_class_config(n, count, shape, T, cw, rmk::kNumBlockVariants);
      CHECK(shape < kStreamShape && class_geometry(n, shape, T, cw, tx, ty), "n=%d: default tiled config", n);
    }
    for (int v = 0; v < kNumShapes; ++v)
      for (int T : {1, 2, 3, 4, 5, 6, 7, 8, 16, 32})
        for (int w : candidate_widths(n, v, T)) {
          int tx, ty;
          CHECK(class_geometry(n, v, T, w, tx, ty), "n=%d v=%d T=%d: candidate width %d invalid", n, v, T, w);
          if (n <= 300 || v == kStreamShape) check_table(n, 3, v, T, w);
        }
    if (n <= rmk::kAdjStreamMaxN)
      for (int count : {1, 64, 256}) {
        const int len = reverse_window(n, count);
        CHECK(len >= 1 && len <= n, "reverse window %d for n=%d", len, n);
        if (len < n) check_partition(n, len, rmk::kAdjMaxT + 1);
      }
  }
  // mixed-size launch groups
  for (int pick = 0; pick < 5; ++pick) {
    check_groups({63, 127, 255, 511, 1023}, {205, 128, 102, 51, 26}, pick);
    check_groups({1, 2, 65, 300, 700, 1024}, {3, 1, 17, 5, 2, 1}, pick);
    check_groups({1023, 64, 513}, {1, 40, 3}, pick);
  }
  if (failures == 0) std::printf("plan checks passed\n");
  return failures == 0 ? 0 : 1;
}
