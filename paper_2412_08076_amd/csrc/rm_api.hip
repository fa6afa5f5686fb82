// C-ABI of the long-step Richardson(m) library (declared in include/rm.h):
// contexts, plans (stencil coefficients and tile tables), and the host drivers of
// the unrolled solve, the FP64-refined solve to tolerance, the adjoint and the
// meta network.  All arithmetic on vectors runs in the kernels of rm_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rm.h"
#include "rm_internal.h"
#include "rm_geometry.h"

using rmk::Inst;
using rmk::PlanDev;
using rmk::Tile;
using namespace rmgeo;

namespace {

thread_local std::string g_last_error;

rm_status fail(rm_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

#define RM_HIP(expr)                                                                           \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return fail(RM_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));                 \
  } while (0)

#define RM_TRY(expr)            \
  do {                          \
    rm_status s_ = (expr);      \
    if (s_ != RM_OK) return s_; \
  } while (0)

// Growable device buffer owned by a plan.  Growing synchronises the stream first
// so that no enqueued kernel still references the old allocation.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  rm_status ensure(size_t need, hipStream_t st) {
    if (need <= bytes) return RM_OK;
    if (ptr != nullptr) {
      RM_HIP(hipStreamSynchronize(st));
      RM_HIP(hipFree(ptr));
      ptr = nullptr;
      bytes = 0;
    }
    if (hipMalloc(&ptr, need) != hipSuccess) {
      ptr = nullptr;
      (void)hipGetLastError();
      return fail(RM_ENOMEM, "hipMalloc of " + std::to_string(need) + " bytes failed");
    }
    bytes = need;
    return RM_OK;
  }
  void release() {
    if (ptr != nullptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
  }
  template <typename T>
  T* as() const {
    return static_cast<T*>(ptr);
  }
};

}  // namespace

struct rm_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  // pinned and coherent: (seq << 32) | active count, written by the refined solve's
  // bookkeeping launches; seq numbers those launches over the context's lifetime
  unsigned long long* host_word = nullptr;
  unsigned seq = 0;
  // pinned host staging for the refined solve's per-round reads (grown on demand)
  void* pin = nullptr;
  size_t pin_bytes = 0;
  // the refined solve runs on a stream of its own (graph capture is not
  // possible on a legacy default stream) after waiting for `stream`
  hipStream_t work = nullptr;
  hipEvent_t handoff = nullptr;
  // plans built on this context; rm_destroy detaches them so that a later
  // rm_plan_free does not reach the freed context
  std::vector<rm_plan_s*> plans;
  // this device's address of the file-scope scratch array of rm_residual_noalloc
  double* noalloc_scratch = nullptr;
  // pinned and coherent: (seq << 32) | active instances, per size class, written by the
  // refined solve's bookkeeping launches like the word above (grown on demand)
  unsigned long long* host_cnt = nullptr;
  size_t host_cnt_n = 0;
};

struct rm_plan_s {
  rm_ctx* ctx = nullptr;
  int B = 0;
  int64_t P = 0;
  std::vector<rm_instance> inst;
  std::vector<int64_t> off;
  std::vector<double> coef;   // [B][8]
  std::vector<double> gersh;  // [B]
  std::vector<Tile> tiles;
  std::vector<Inst> insts;
  // device copies
  DevBuf d_tiles, d_inst, d_coef32, d_coef64, d_mu, d_gersh;
  // scratch
  DevBuf partial, red, flags, vecA, vecB, vecC, vecD, vecE, vecF, states, acc, meta;
  // FP32 sweeps: temporal-blocked kernels, one configuration per size class
  struct ClassExec {
    int n = 0;
    int shape = 0;  // kernel shape: tiled variant (index into rmk::kBlockVariants) or row-streaming
    int T = 1;      // steps per launch
    int cw = 64;    // extended tile width (multiple of 8), or row-window height (row-streaming)
    std::vector<int> insts;
    DevBuf tiles;
    int ntiles = 0;
    // Tail configuration: used by the refined solve once few instances are still
    // active.  A row-streaming launch takes about as long for one active instance
    // as for many (each workgroup walks its rows one after another), while the
    // small tiles of a tiled variant cost in proportion to the active instances.
    int tshape = 0, tT = 1, tcw = 64;
    DevBuf ttiles;
    int tntiles = 0;
    // Row windows for the reverse steps of the adjoint (n <= kAdjStreamMaxN), whatever the
    // forward configuration: rcw rows each, overlapping by kAdjMaxT + 1.
    int rcw = 0;
    DevBuf rtiles;
    int rntiles = 0;
    double us = 0.0, tus = 0.0;  // tuned time per inner step, whole class active
    double floor_us = 0.0;       // main configuration with one instance active
  };
  bool use_block = true;
  bool exec_dirty = true;
  int jacobi = 0;  // set per call from RM_FLAG_JACOBI
  int ssor = 0;    // set per call from RM_FLAG_SSOR, with the relaxation factor
  double relax = 1.0;
  std::vector<ClassExec> classes;
  DevBuf d_ranges;  // int [B][2]: slot range of each instance over all class tables
  DevBuf d_tranges; // the same over the tail tables (slots after those of the main tables)
  DevBuf d_cls;     // int [B]: size class of each instance
  DevBuf d_rranges; // the same over the reverse-step tables
  int nslots = 0;
  // mixed-size launch (rm_plan_set_mixed): the main tiles of the classes in it, grouped,
  // and those classes as a bit mask
  bool mixed = false;
  DevBuf d_mtiles, d_mgroups;
  int nmgroups = 0;
  unsigned long long mixed_classes = 0;
  double tail_frac = -1.0;  // active fraction below which the refined solve uses the tails (< 0: measured)
  // two-grid correction: coarse layout, tile and row-group tables, twiddles and
  // coarse scratch, built on first use
  struct TwoGrid {
    bool ready = false;
    int64_t Pc = 0;
    std::vector<int64_t> coff;
    DevBuf d_inst, d_rtiles, d_groups, d_tw, c0, c1, shat, fine2, zero;
    int nrtiles = 0, ngroups = 0, mmax = 0;
    // symbol network: 16 x 16 mode tiles, activations and gradients (16 planes each),
    // the symbol, its log-gradient and the per-tile weight-gradient partials
    DevBuf d_stiles, sa1, sa2, sg1, sg2, ssym, sgz, spart, sgsum;
    int nstiles = 0;
  } tg;
  // flexible GMRES: basis (FP64), preconditioned directions (FP32), work vectors and
  // per-instance state
  struct Fgm {
    DevBuf V, Z, w, t, b32, dbl, ints, partial;
  } fg;
  rmk::TgDev tgdev() const {
    rmk::TgDev g;
    g.inst = tg.d_inst.as<rmk::TgInst>();
    g.tw = tg.d_tw.as<float2>();
    return g;
  }
  PlanDev dev() const {
    PlanDev p;
    p.tiles = d_tiles.as<Tile>();
    p.ntiles = (int)tiles.size();
    p.inst = d_inst.as<Inst>();
    p.B = B;
    p.coef32 = d_coef32.as<float>();
    p.coef64 = d_coef64.as<double>();
    p.mu = d_mu.as<float>();
    p.gersh = d_gersh.as<float>();
    p.jacobi = jacobi;
    return p;
  }
  ~rm_plan_s() {
    for (DevBuf* b : {&d_tiles, &d_inst, &d_coef32, &d_coef64, &d_mu, &d_gersh, &partial, &red, &flags, &vecA,
                      &vecB, &vecC, &vecD, &vecE, &vecF, &states, &acc, &meta, &d_ranges, &d_tranges, &d_rranges, &d_cls, &d_mtiles, &d_mgroups, &tg.d_inst,
                      &tg.d_rtiles, &tg.d_groups, &tg.d_tw, &tg.c0, &tg.c1, &tg.shat, &tg.fine2,
                      &tg.zero, &tg.d_stiles, &tg.sa1, &tg.sa2, &tg.sg1, &tg.sg2, &tg.ssym, &tg.sgz, &tg.spart, &tg.sgsum, &fg.V, &fg.Z, &fg.w, &fg.t, &fg.b32, &fg.dbl, &fg.ints, &fg.partial})
      b->release();
    for (auto& c : classes) {
      c.tiles.release();
      c.ttiles.release();
      c.rtiles.release();
    }
  }
};

namespace {

constexpr int kMaxN = 16384;
constexpr int kMaxM = 64;

// Stencil coefficients of one instance (slots: centre, (+-1,0), (0,+-1),
// (1,1)/(-1,-1), (-1,1)/(1,-1)).
// Q1 (§2.3): C = R diag(1, eps) R^T = [[a, b], [b, c]]; exact element integrals of
// bilinear shape functions on a square give the h-free row below.
// Helmholtz (§3.2): (1/h^2) [0 -1 0; -1 4 - kappa^2 h^2 -1; 0 -1 0], h = 1/(n+1).
void stencil_coefficients(const rm_instance& in, double out[8]) {
  std::fill(out, out + 8, 0.0);
  if (in.op == RM_Q1_ANISO) {
    const double cs = std::cos(in.theta), sn = std::sin(in.theta), e = in.eps;
    const double a = cs * cs + e * sn * sn;
    const double b = (1.0 - e) * sn * cs;
    const double c = sn * sn + e * cs * cs;
    out[0] = 4.0 * (a + c) / 3.0;
    out[1] = (c - 2.0 * a) / 3.0;
    out[2] = (a - 2.0 * c) / 3.0;
    out[3] = -(a + c) / 6.0 - 0.5 * b;
    out[4] = -(a + c) / 6.0 + 0.5 * b;
  } else {
    const double h = 1.0 / (in.n + 1.0);
    const double ih2 = 1.0 / (h * h);
    out[0] = 4.0 * ih2 - in.kappa * in.kappa;
    out[1] = -ih2;
    out[2] = -ih2;
  }
}

rm_status check_ctx_plan(rm_ctx* ctx, const rm_plan_t* plan) {
  if (ctx == nullptr) return fail(RM_EINVAL, "null context");
  if (plan == nullptr) return fail(RM_EINVAL, "null plan");
  if (plan->ctx != ctx) return fail(RM_EINVAL, "plan belongs to another context");
  return RM_OK;
}

rm_status last_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(RM_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return RM_OK;
}

template <typename T>
size_t vec_bytes(const rm_plan_t* p) {
  return (size_t)std::max<int64_t>(p->P, 1) * sizeof(T);
}

// The tail is the main configuration unless that is the row-streaming kernel; then it
// is the cost model's best tiled variant.
void set_default_tail(rm_plan_s::ClassExec& c) {
  if (c.shape == kStreamShape) {
    default_class_config(c.n, (int)c.insts.size(), c.tshape, c.tT, c.tcw, rmk::kNumBlockVariants);
  } else {
    c.tshape = c.shape;
    c.tT = c.T;
    c.tcw = c.cw;
  }
  c.us = c.tus = c.floor_us = 0.0;
}

void init_classes(rm_plan_t* pl) {
  pl->classes.clear();
  std::vector<int> sizes;
  for (const auto& in : pl->inst) sizes.push_back(in.n);
  std::sort(sizes.begin(), sizes.end());
  sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
  for (int n : sizes) {
    rm_plan_s::ClassExec c;
    c.n = n;
    for (int b = 0; b < pl->B; ++b)
      if (pl->inst[b].n == n) c.insts.push_back(b);
    default_class_config(n, (int)c.insts.size(), c.shape, c.T, c.cw);
    set_default_tail(c);
    pl->classes.push_back(std::move(c));
  }
  pl->exec_dirty = true;
}

// Tile table of one configuration of a class; residual slots are numbered from `slot`
// on and each instance's slot range goes to ranges[2b], ranges[2b + 1].
rm_status build_table(const rm_plan_s::ClassExec& c, int shape, int T, int cw, int& slot, std::vector<int>& ranges,
                      DevBuf& tiles, int& ntiles, hipStream_t st, std::vector<rmk::BTile>* keep = nullptr) {
  std::vector<rmk::BTile> local;
  std::vector<rmk::BTile>& t = keep != nullptr ? *keep : local;
  if (!make_tiles(c.n, c.insts, shape, T, cw, slot, ranges, t)) return fail(RM_EINVAL, "invalid kernel configuration");
  ntiles = (int)t.size();
  RM_TRY(tiles.ensure(t.size() * sizeof(rmk::BTile), st));
  RM_HIP(hipStreamSynchronize(st));
  RM_HIP(hipMemcpy(tiles.ptr, t.data(), t.size() * sizeof(rmk::BTile), hipMemcpyHostToDevice));
  return RM_OK;
}

rm_status build_exec(rm_plan_t* pl, hipStream_t st) {
  if (!pl->exec_dirty) return RM_OK;
  std::vector<int> ranges((size_t)pl->B * 2, 0), tranges((size_t)pl->B * 2, 0), rranges((size_t)pl->B * 2, 0);
  // main and tail tables number their residual slots in one sequence, so that one outer
  // iteration may run some classes in their main and others in their tail configuration
  int slot = 0, rslot = 0;
  std::vector<std::vector<rmk::BTile>> main_tabs(pl->classes.size());
  for (size_t ci = 0; ci < pl->classes.size(); ++ci) {
    auto& c = pl->classes[ci];
    RM_TRY(build_table(c, c.shape, c.T, c.cw, slot, ranges, c.tiles, c.ntiles, st, &main_tabs[ci]));
  }
  // the mixed-size launch takes the classes whose main configuration is the 8-step row
  // pipeline, over their main tiles (so the same residual slots and ranges)
  pl->mixed_classes = 0;
  pl->nmgroups = 0;
  if (pl->mixed) {
    std::vector<rmgeo::MixedClass> mc;
    for (size_t ci = 0; ci < pl->classes.size() && ci < 64; ++ci) {
      const auto& c = pl->classes[ci];
      if (c.shape != kStreamShape || c.T != rmk::kStreamMaxT) continue;
      mc.push_back(rmgeo::MixedClass{(int)ci, c.n, c.cw, &main_tabs[ci]});
      pl->mixed_classes |= 1ull << ci;
    }
    if (!mc.empty()) {
      std::vector<rmk::BTile> all;
      std::vector<rmk::MGroup> groups;
      if (!make_groups(mc, all, groups)) return fail(RM_EINVAL, "mixed-size launch: invalid windows");
      RM_TRY(pl->d_mtiles.ensure(all.size() * sizeof(rmk::BTile), st));
      RM_TRY(pl->d_mgroups.ensure(groups.size() * sizeof(rmk::MGroup), st));
      RM_HIP(hipStreamSynchronize(st));
      RM_HIP(hipMemcpy(pl->d_mtiles.ptr, all.data(), all.size() * sizeof(rmk::BTile), hipMemcpyHostToDevice));
      RM_HIP(hipMemcpy(pl->d_mgroups.ptr, groups.data(), groups.size() * sizeof(rmk::MGroup), hipMemcpyHostToDevice));
      pl->nmgroups = (int)groups.size();
    }
  }
  int tslot = slot;
  std::vector<int> cls((size_t)pl->B, 0);
  for (size_t ci = 0; ci < pl->classes.size(); ++ci) {
    auto& c = pl->classes[ci];
    for (int b : c.insts) cls[b] = (int)ci;
    RM_TRY(build_table(c, c.tshape, c.tT, c.tcw, tslot, tranges, c.ttiles, c.tntiles, st));
    c.rcw = 0;
    c.rntiles = 0;
    if (c.n <= rmk::kAdjStreamMaxN) {
      c.rcw = reverse_window(c.n, (int)c.insts.size());
      RM_TRY(build_table(c, kStreamShape, rmk::kAdjMaxT, c.rcw, rslot, rranges, c.rtiles, c.rntiles, st));
    }
  }
  pl->nslots = std::max(slot, std::max(tslot, rslot));
  RM_TRY(pl->d_rranges.ensure(rranges.size() * sizeof(int), st));
  RM_HIP(hipMemcpy(pl->d_rranges.ptr, rranges.data(), rranges.size() * sizeof(int), hipMemcpyHostToDevice));
  RM_TRY(pl->d_ranges.ensure(ranges.size() * sizeof(int), st));
  RM_HIP(hipMemcpy(pl->d_ranges.ptr, ranges.data(), ranges.size() * sizeof(int), hipMemcpyHostToDevice));
  RM_TRY(pl->d_tranges.ensure(tranges.size() * sizeof(int), st));
  RM_HIP(hipMemcpy(pl->d_tranges.ptr, tranges.data(), tranges.size() * sizeof(int), hipMemcpyHostToDevice));
  RM_TRY(pl->d_cls.ensure(cls.size() * sizeof(int), st));
  RM_HIP(hipMemcpy(pl->d_cls.ptr, cls.data(), cls.size() * sizeof(int), hipMemcpyHostToDevice));
  pl->exec_dirty = false;
  return RM_OK;
}

size_t partial_slots(const rm_plan_t* pl) { return std::max<size_t>(pl->tiles.size(), (size_t)pl->nslots); }

// Temporal-blocked sweeps serve the unpreconditioned and Jacobi steps; an SSOR step
// needs its whole tile in one launch.
bool blocked(const rm_plan_t* pl) { return pl->use_block && !pl->ssor; }

// T fused steps of one size class with its main (tail = false) or tail configuration
// (see rmk::launch_block and rmk::launch_stream).
bool launch_class(const rm_plan_s::ClassExec& c, int T, int method, const PlanDev& p, const float* omega,
                  const float* alpha, int m, int s0, const float* f, const float* u, const float* v, float* u_out,
                  float* v_out, const int* active, double* partial2, hipStream_t st, float* states = nullptr,
                  int64_t state_stride = 0, bool tail = false) {
  const int shape = tail ? c.tshape : c.shape, cw = tail ? c.tcw : c.cw, nt = tail ? c.tntiles : c.ntiles;
  const rmk::BTile* tiles = (tail ? c.ttiles : c.tiles).as<rmk::BTile>();
  if (shape == kStreamShape)
    return rmk::launch_stream(T, cw, c.n, method, p, tiles, nt, omega, alpha, m, s0, f, u, v, u_out, v_out, active,
                              partial2, st, states, state_stride);
  return rmk::launch_block(shape, T, cw, method, p, tiles, nt, omega, alpha, m, s0, f, u, v, u_out, v_out, active,
                           partial2, st, states, state_stride);
}

// One inner step over the plan's one-step tile table, plain or SSOR-preconditioned.
template <typename T>
void one_step(const rm_plan_t* pl, const PlanDev& p, int method, const float* omega, const float* alpha, int m, int i,
              const T* f, const T* u, const T* v, T* u_out, T* v_out, const int* active, hipStream_t st) {
  if (pl->ssor)
    rmk::launch_ssor_step<T>(method, p, p.tiles, p.ntiles, omega, alpha, m, i, pl->relax, f, u, v, u_out, v_out,
                             active, st);
  else
    rmk::launch_step<T>(method, p, p.tiles, p.ntiles, omega, alpha, m, i, f, u, v, u_out, v_out, active, st);
}

void adj_one_step(const rm_plan_t* pl, const PlanDev& p, int method, const float* omega, const float* alpha, int m,
                  int i, const float* f, const float* u, const float* v, const float* ub, const float* vb,
                  float* ub_out, float* vb_out, float* fb, double* partial4, hipStream_t st) {
  if (pl->ssor)
    rmk::launch_adj_ssor_step(method, p, omega, alpha, m, i, pl->relax, f, u, v, ub, vb, ub_out, vb_out, fb, partial4,
                              st);
  else
    rmk::launch_adj_step(method, p, omega, alpha, m, i, f, u, v, ub, vb, ub_out, vb_out, fb, partial4, st);
}

// Reverse steps of the adjoint in the row pipeline: when every size class has row windows
// for them (and no SSOR step, whose reverse needs its own kernel).
bool stream_reverse(const rm_plan_t* pl) {
  bool ok = blocked(pl) && !pl->classes.empty();
  for (const auto& cl : pl->classes) ok = ok && cl.rntiles > 0;
  return ok;
}

// Reverse the forward steps nsteps - 1 .. 0 of one segment (latest first).  su(t), sv(t)
// give the state before step t, the weight index of step t is (base + t) mod m, and the
// dot-product partials of step t go to partial + 4 nslot t.  (ubs[cur], vbs[cur]) hold
// the adjoints after the segment on entry and before it on return.  *ranges receives
// the per-instance slot ranges the accumulation must use (null: the one-step tiles).
template <typename SU, typename SV>
rm_status reverse_segment(rm_plan_t* pl, const PlanDev& p, hipStream_t st, int method, const float* omega,
                          const float* alpha, int m, int base, int nsteps, SU su, SV sv, const float* b,
                          float* const ubs[2], float* const vbs[2], int& cur, float* d_b, double* partial, int nslot,
                          const int** ranges) {
  if (stream_reverse(pl)) {
    for (int t = nsteps - 1; t >= 0;) {
      const int tn = std::min(rmk::kAdjMaxT, t + 1);
      rmk::AdjLevels lev{};
      for (int l = 0; l < tn; ++l) {
        lev.u[l] = su(t - l);
        lev.v[l] = sv(t - l);
        lev.part[l] = partial + (size_t)(t - l) * 4 * nslot;
        lev.i[l] = (base + t - l) % m;
      }
      for (auto& cl : pl->classes)
        if (!rmk::launch_adj_stream(tn, cl.rcw, cl.n, method, p, cl.rtiles.as<rmk::BTile>(), cl.rntiles, omega, alpha,
                                    m, lev, b, ubs[cur], vbs[cur], ubs[cur ^ 1], vbs[cur ^ 1], d_b, st))
          return fail(RM_EUNSUPPORTED, "reverse kernel configuration not built");
      cur ^= 1;
      t -= tn;
    }
    *ranges = pl->d_rranges.as<int>();
    return RM_OK;
  }
  for (int t = nsteps - 1; t >= 0; --t) {
    adj_one_step(pl, p, method, omega, alpha, m, (base + t) % m, b, su(t), sv(t), ubs[cur], vbs[cur], ubs[cur ^ 1],
                 vbs[cur ^ 1], d_b, partial + (size_t)t * 4 * nslot, st);
    cur ^= 1;
  }
  *ranges = nullptr;
  return RM_OK;
}

// Preconditioner of this call (validated by validate_weights).
void set_precond(rm_plan_t* pl, const rm_solve_opts* o) {
  pl->jacobi = (o->flags & RM_FLAG_JACOBI) ? 1 : 0;
  pl->ssor = (o->flags & RM_FLAG_SSOR) ? 1 : 0;
  pl->relax = pl->ssor ? o->relax : 1.0;
}

// Advance `nsteps` FP32 inner steps (global step indices s0 ..) on the pingpong
// pair (us, vs), starting from set `cur`; `cur` ends on the set holding the
// result and `flips` counts the swaps (the same for every instance).  Each size
// class advances in its own chunks of at most its T steps, as few as T allows, but
// every class, in its main and in its tail configuration alike, makes a number of
// launches of one common parity, so all classes end on the same set and a solve that
// switches configurations flips the same way throughout.
// When res_partial is given, the residual ||f - A u||^2 of the final iterate is
// left per tile in res_partial and *res_ranges tells the reduction which slots
// belong to which instance (the main tables' ranges; classes in their tail
// configuration use the tail tables' ranges, see uses_tail).  `only_class` >= 0
// restricts the launches to one size class (autotuning); bit c of `tail` selects the
// tail configuration of class c (classes from 64 on always run their main one); bit c
// of `skip` leaves class c out (all of its instances are inactive).
bool uses_tail(unsigned long long tail, size_t ci) { return ci < 64 && ((tail >> ci) & 1ull) != 0; }

rm_status sweep(rm_plan_t* pl, hipStream_t st, int method, int m, int s0, int nsteps, const float* omega,
                const float* alpha, const float* f, float* const us[2], float* const vs[2], int& cur, int& flips,
                const int* active, double* res_partial, const int** res_ranges, int only_class = -1,
                unsigned long long tail = 0, unsigned long long skip = 0) {
  const PlanDev p = pl->dev();
  if (nsteps <= 0) return RM_OK;
  if (!blocked(pl)) {
    for (int k = 0; k < nsteps; ++k) {
      one_step<float>(pl, p, method, omega, alpha, m, (s0 + k) % m, f, us[cur], vs[cur], us[cur ^ 1], vs[cur ^ 1],
                      active, st);
      cur ^= 1;
      ++flips;
    }
    if (res_partial != nullptr) {
      rmk::launch_residual<float>(p, p.tiles, p.ntiles, f, us[cur], nullptr, res_partial, active, st);
      *res_ranges = nullptr;
    }
    return RM_OK;
  }
  RM_TRY(build_exec(pl, st));
  // common parity of the launch counts: the fewest launches when they agree; else the
  // parity of a count that cannot grow (one step per launch), else even
  int par = -1;
  bool mixed = false;
  int fixed_par = -1;
  for (const auto& c : pl->classes)
    for (const int T : {c.T, c.tT}) {
      const int lc = (nsteps + T - 1) / T;
      if (par < 0) par = lc & 1;
      else if ((lc & 1) != par) mixed = true;
      if (lc == nsteps) fixed_par = lc & 1;
    }
  if (mixed) par = fixed_par >= 0 ? fixed_par : 0;
  // chunk plan per class
  std::vector<std::vector<int>> chunks(pl->classes.size());
  int L = 0;
  for (size_t ci = 0; ci < pl->classes.size(); ++ci) {
    if (only_class >= 0 && (int)ci != only_class) continue;
    if (uses_tail(skip, ci)) continue;
    const int T = uses_tail(tail, ci) ? pl->classes[ci].tT : pl->classes[ci].T;
    int lc = (nsteps + T - 1) / T;
    if ((lc & 1) != par) ++lc;
    for (int j = 0; j < lc; ++j) chunks[ci].push_back(nsteps / lc + (j < nsteps % lc ? 1 : 0));
    L = std::max(L, lc);
  }
  // the classes the mixed-size launch advances in this sweep: in the launch's table, in
  // their main configuration and not left out; they share one chunk plan (T = 8)
  unsigned long long in_mixed = 0;
  int mc0 = -1;
  if (pl->mixed && pl->nmgroups > 0 && only_class < 0)
    for (size_t ci = 0; ci < pl->classes.size() && ci < 64; ++ci)
      if (((pl->mixed_classes >> ci) & 1ull) != 0 && !uses_tail(skip, ci) && !uses_tail(tail, ci)) {
        in_mixed |= 1ull << ci;
        if (mc0 < 0) mc0 = (int)ci;
      }
  for (int j = 0; j < L; ++j) {
    const int rd = (cur + j) & 1;
    if (mc0 >= 0 && j < (int)chunks[mc0].size()) {
      int s = s0;
      for (int q = 0; q < j; ++q) s += chunks[mc0][q];
      const bool last = j + 1 == (int)chunks[mc0].size();
      if (!rmk::launch_stream_mixed(chunks[mc0][j], method, p, pl->d_mtiles.as<rmk::BTile>(),
                                    pl->d_mgroups.as<rmk::MGroup>(), pl->nmgroups, ~in_mixed, omega, alpha, m, s, f,
                                    us[rd], vs[rd], us[rd ^ 1], vs[rd ^ 1], active, last ? res_partial : nullptr, st))
        return fail(RM_EUNSUPPORTED, "mixed-size launch not built for this step count");
    }
    for (size_t ci = 0; ci < pl->classes.size(); ++ci) {
      if (j >= (int)chunks[ci].size()) continue;
      if (ci < 64 && ((in_mixed >> ci) & 1ull) != 0) continue;
      auto& c = pl->classes[ci];
      int s = s0;
      for (int q = 0; q < j; ++q) s += chunks[ci][q];
      const bool last = j + 1 == (int)chunks[ci].size();
      if (!launch_class(c, chunks[ci][j], method, p, omega, alpha, m, s, f, us[rd], vs[rd], us[rd ^ 1], vs[rd ^ 1],
                        active, last ? res_partial : nullptr, st, nullptr, 0, uses_tail(tail, ci)))
        return fail(RM_EUNSUPPORTED, "block kernel configuration not built");
    }
  }
  cur ^= par;
  flips += par ? 1 : 2;
  if (res_partial != nullptr) *res_ranges = pl->d_ranges.as<int>();
  return RM_OK;
}

// ---------------------------------------------------------------------------
// unrolled solve: K inner steps from (x, 0)
// ---------------------------------------------------------------------------
template <typename T>
rm_status solve_unroll(rm_ctx* ctx, rm_plan_t* pl, int method, const rm_solve_opts* o, const float* omega,
                       const float* alpha, const T* b, T* x, T* ckpt, double* hist) {
  hipStream_t st = ctx->stream;
  const int64_t P = pl->P;
  RM_TRY(pl->vecA.ensure(vec_bytes<T>(pl), st));
  RM_TRY(pl->vecB.ensure(vec_bytes<T>(pl), st));
  RM_TRY(pl->vecC.ensure(vec_bytes<T>(pl), st));
  RM_TRY(pl->partial.ensure(pl->tiles.size() * 2 * sizeof(double), st));
  T* v0 = pl->vecA.as<T>();
  T* u1 = pl->vecB.as<T>();
  T* v1 = pl->vecC.as<T>();
  T* us[2] = {x, u1};
  T* vs[2] = {v0, v1};
  const PlanDev p = pl->dev();
  if (sizeof(T) == 4) {
    rmk::launch_fill_f32((float*)v0, 0.f, P, st);
    rmk::launch_fill_f32((float*)v1, 0.f, P, st);
  } else {
    rmk::launch_fill_f64((double*)v0, 0.0, P, st);
    rmk::launch_fill_f64((double*)v1, 0.0, P, st);
  }
  const int E = o->ckpt_every;
  if (sizeof(T) == 4) {
    // FP32: temporal-blocked sweeps between checkpoint and history boundaries
    RM_TRY(build_exec(pl, st));
    RM_TRY(pl->partial.ensure(partial_slots(pl) * 2 * sizeof(double), st));
    float* fu[2] = {(float*)us[0], (float*)us[1]};
    float* fv[2] = {(float*)vs[0], (float*)vs[1]};
    int cur = 0, flips = 0;
    for (int s = 0; s < o->K;) {
      if (ckpt != nullptr && E > 0 && s % E == 0) {
        T* slot = ckpt + (int64_t)(s / E) * 2 * P;
        RM_HIP(hipMemcpyAsync(slot, us[cur], P * sizeof(T), hipMemcpyDeviceToDevice, st));
        RM_HIP(hipMemcpyAsync(slot + P, vs[cur], P * sizeof(T), hipMemcpyDeviceToDevice, st));
      }
      int next = (s / o->m + 1) * o->m;
      if (ckpt != nullptr && E > 0) next = std::min(next, (s / E + 1) * E);
      next = std::min(next, o->K);
      const bool want_hist = hist != nullptr && next % o->m == 0;
      const int* ranges = nullptr;
      RM_TRY(sweep(pl, st, method, o->m, s, next - s, omega, alpha, (const float*)b, fu, fv, cur, flips, nullptr,
                   want_hist ? pl->partial.as<double>() : nullptr, &ranges));
      if (want_hist) {
        const int k = next / o->m - 1;
        rmk::launch_reduce_partials(p, pl->partial.as<double>(), hist + (int64_t)k * pl->B, nullptr, 1, nullptr, st,
                                    ranges);
      }
      s = next;
    }
    if (cur == 1) RM_HIP(hipMemcpyAsync(x, u1, P * sizeof(T), hipMemcpyDeviceToDevice, st));
    return last_launch();
  }
  for (int s = 0; s < o->K; ++s) {
    const int cur = s & 1, nxt = cur ^ 1;
    if (ckpt != nullptr && E > 0 && s % E == 0) {
      T* slot = ckpt + (int64_t)(s / E) * 2 * P;
      RM_HIP(hipMemcpyAsync(slot, us[cur], P * sizeof(T), hipMemcpyDeviceToDevice, st));
      RM_HIP(hipMemcpyAsync(slot + P, vs[cur], P * sizeof(T), hipMemcpyDeviceToDevice, st));
    }
    one_step<T>(pl, p, method, omega, alpha, o->m, s % o->m, b, us[cur], vs[cur], us[nxt], vs[nxt], nullptr, st);
    if (hist != nullptr && (s + 1) % o->m == 0) {
      const int k = (s + 1) / o->m - 1;
      rmk::launch_residual<T>(p, p.tiles, p.ntiles, b, us[nxt], nullptr, pl->partial.as<double>(), nullptr, st);
      rmk::launch_reduce_partials(p, pl->partial.as<double>(), hist + (int64_t)k * pl->B, nullptr, 1, nullptr, st);
    }
  }
  if (o->K & 1) RM_HIP(hipMemcpyAsync(x, u1, P * sizeof(T), hipMemcpyDeviceToDevice, st));
  return last_launch();
}

// ---------------------------------------------------------------------------
// FP64 iterative refinement around FP32 inner solves (blocks)
// ---------------------------------------------------------------------------
// One captured outer iteration of the inner solve, replayed with hipGraphLaunch.
struct GraphHolder {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~GraphHolder() {
    if (exec != nullptr) (void)hipGraphExecDestroy(exec);
    if (graph != nullptr) (void)hipGraphDestroy(graph);
  }
};

// Waits until the bookkeeping launch numbered want (or a later one) has published its
// word, spinning on the pinned copy.  After every 20 ms of waiting the stream is
// queried, so that an error or a drained stream without the word ends the wait; the
// query is kept that rare because it can place a marker in the queue, which stalls
// the GPU between launches.
rm_status wait_word(rm_ctx* ctx, hipStream_t st, unsigned want, unsigned long long& w) {
  using clock = std::chrono::steady_clock;
  auto next_query = clock::now() + std::chrono::milliseconds(20);
  for (unsigned spin = 1;; ++spin) {
    w = __atomic_load_n(ctx->host_word, __ATOMIC_ACQUIRE);
    if ((int)((unsigned)(w >> 32) - want) >= 0) return RM_OK;
    if ((spin & 4095u) == 0 && clock::now() >= next_query) {
      const hipError_t e = hipStreamQuery(st);
      if (e == hipSuccess) {
        w = __atomic_load_n(ctx->host_word, __ATOMIC_ACQUIRE);
        if ((int)((unsigned)(w >> 32) - want) >= 0) return RM_OK;
        return fail(RM_EHIP, "the active count was not published");
      }
      if (e != hipErrorNotReady) return fail(RM_EHIP, std::string("hipStreamQuery: ") + hipGetErrorString(e));
      next_query = clock::now() + std::chrono::milliseconds(20);
    }
    __builtin_ia32_pause();
  }
}

rm_status solve_to_tol(rm_ctx* ctx, rm_plan_t* pl, int method, const rm_solve_opts* o, const float* omega,
                       const float* alpha, const double* b, double* x, double* hist, rm_report* rep) {
  if (ctx->work == nullptr) {
    RM_HIP(hipStreamCreateWithFlags(&ctx->work, hipStreamNonBlocking));
    RM_HIP(hipEventCreateWithFlags(&ctx->handoff, hipEventDisableTiming));
  }
  RM_HIP(hipEventRecord(ctx->handoff, ctx->stream));
  RM_HIP(hipStreamWaitEvent(ctx->work, ctx->handoff, 0));
  hipStream_t st = ctx->work;
  const int B = pl->B;
  const int H = o->max_rounds + 1;  // rows of the per-round history
  const size_t fb = vec_bytes<float>(pl);
  RM_TRY(pl->vecA.ensure(fb, st));  // r32
  RM_TRY(pl->vecB.ensure(fb, st));  // d0
  RM_TRY(pl->vecC.ensure(fb, st));  // v0
  RM_TRY(pl->vecD.ensure(fb, st));  // d1
  RM_TRY(pl->vecE.ensure(fb, st));  // v1
  RM_TRY(build_exec(pl, st));
  RM_TRY(pl->partial.ensure(partial_slots(pl) * 2 * sizeof(double), st));
  RM_TRY(pl->red.ensure(((size_t)B * 8 + (size_t)H * B) * sizeof(double), st));
  RM_TRY(pl->flags.ensure(((size_t)B * 13 + 16) * sizeof(int), st));
  const int ncls = (int)pl->classes.size();
  if (ctx->host_cnt_n < (size_t)ncls) {
    RM_HIP(hipStreamSynchronize(st));
    if (ctx->host_cnt != nullptr) (void)hipHostFree(ctx->host_cnt);
    ctx->host_cnt = nullptr;
    ctx->host_cnt_n = 0;
    RM_HIP(hipHostMalloc((void**)&ctx->host_cnt, (size_t)ncls * sizeof(unsigned long long), hipHostMallocCoherent));
    for (int ci = 0; ci < ncls; ++ci) __atomic_store_n(ctx->host_cnt + ci, 0ull, __ATOMIC_RELEASE);
    ctx->host_cnt_n = (size_t)ncls;
  }
  // pinned host copies of the final per-instance results: history [H][B], relres (double),
  // then status, rounds, tot, count (int)
  const size_t pin_need = ((size_t)H + 1) * B * sizeof(double) + 4 * (size_t)B * sizeof(int);
  if (ctx->pin_bytes < pin_need) {
    RM_HIP(hipStreamSynchronize(st));
    if (ctx->pin != nullptr) (void)hipHostFree(ctx->pin);
    ctx->pin = nullptr;
    ctx->pin_bytes = 0;
    RM_HIP(hipHostMalloc(&ctx->pin, pin_need, 0));
    ctx->pin_bytes = pin_need;
  }
  float* r32 = pl->vecA.as<float>();
  float* ds[2] = {pl->vecB.as<float>(), pl->vecD.as<float>()};
  float* vs[2] = {pl->vecC.as<float>(), pl->vecE.as<float>()};
  double* dd = pl->red.as<double>();
  rmk::RoundState rs;
  double* res2 = dd;            // [B]  inner residual^2 after an outer iteration
  rs.rhs2 = dd + B;             // [B]  ||r_j||^2 of the instance's current round
  rs.target2 = dd + 2 * B;      // [B]  inner residual^2 that ends the round
  rs.best2 = dd + 3 * B;        // [B]  smallest inner residual^2 of the round (stagnation)
  rs.prev_rho = dd + 4 * B;     // [B]  rho of the previous round
  rs.relres = dd + 5 * B;       // [B]  the last rho
  rs.history = dd + 8 * B;      // [H][B]
  int* ii = pl->flags.as<int>();
  rs.active = ii;               // [B]  in an inner solve
  rs.count = ii + B;            // [B]  outer iterations of the current round
  rs.status = ii + 2 * B;       // [B]
  rs.pending = ii + 3 * B;      // [B]  round ended, refinement step not yet taken
  rs.since = ii + 4 * B;        // [B]  outer iterations since the last 10 % gain
  rs.gains = ii + 5 * B;        // [B]  10 % gains so far in this round
  rs.tot = ii + 6 * B;          // [B]  outer iterations of the instance's earlier rounds
  rs.round = ii + 7 * B;        // [B]  rounds started
  rs.strikes = ii + 8 * B;      // [B]  rounds that did not halve rho
  rs.start = ii + 9 * B;        // [B]  outer iteration of the solve at which the round began
  int* n_active = ii + 13 * B;  // [1]
  double* partial = pl->partial.as<double>();
  const PlanDev p = pl->dev();
  // stagnation window bounds in outer iterations (about 256 and 4096 inner steps)
  const int stall_min = std::max(16, (256 + o->m - 1) / o->m);
  const int stall_max = std::max(16, (4096 + o->m - 1) / o->m);
  rmk::launch_fill_i32(ii, 0, (int64_t)B * 10, st);
  rmk::launch_fill_i32(rs.pending, 1, B, st);  // every instance starts with a refinement step
  rmk::launch_fill_f64(rs.history, -1.0, (int64_t)H * B, st);
  if (hist != nullptr) rmk::launch_fill_f64(hist, -1.0, (int64_t)o->hist_len * B, st);
  rmk::RoundParams rp{o->tol, o->tol_inner, o->max_rounds, 0};
  int flips_per_outer = 0;
  // Refinement step of every waiting instance before outer iteration g of the solve:
  // x += d of the ended round, r = b - A x in FP64, r32 = fl32(r), d = v = 0 in the buffer
  // set iteration g reads, then the decision.  Each instance runs its rounds on its own:
  // one that ends a round starts the next while the others go on.
  auto refine_step = [&](long long g, bool first) {
    if (!first) rmk::launch_refine_update(p, x, ds[0], ds[1], rs.start, rs.count, flips_per_outer, rs.pending, st);
    const int set = (int)((g * flips_per_outer) & 1);
    rmk::launch_refine_residual(p, b, x, r32, ds[set], vs[set], partial, rs.pending, st);
    rp.start = (int)g;
    rmk::launch_round_decide(p, partial, rp, rs, st);
  };
  refine_step(0, true);

  // one captured outer iteration per combination of main and tail configurations
  std::map<std::pair<unsigned long long, unsigned long long>, GraphHolder> graphs;
  bool use_graph = (o->flags & RM_FLAG_GRAPH) != 0;
  // Per size class: its tail configuration runs once fewer than thr[c] of its
  // instances are not done (0: never; the first 64 classes can switch).
  std::vector<int> thr(ncls, 0);
  for (int ci = 0; ci < ncls && ci < 64; ++ci) {
    const auto& c = pl->classes[ci];
    if (c.tshape == c.shape && c.tT == c.T && c.tcw == c.cw) continue;
    double frac = c.floor_us > 0.0 && c.tus > 0.0 ? c.floor_us / c.tus : 0.35;
    if (pl->tail_frac >= 0.0) frac = pl->tail_frac;
    const int size = (int)c.insts.size();
    thr[ci] = frac >= 1.0 ? size + 1 : (int)std::ceil(frac * size);
  }
  // instances per class not yet done, as last seen (all of them before the first poll)
  std::vector<int> live(ncls, 0);
  for (int ci = 0; ci < ncls; ++ci) live[ci] = (int)pl->classes[ci].insts.size();
  using Config = std::pair<unsigned long long, unsigned long long>;  // (tail mask, skip mask)
  auto config = [&]() {
    Config cf{0ull, 0ull};
    for (int ci = 0; ci < ncls && ci < 64; ++ci) {
      if (live[ci] < thr[ci]) cf.first |= 1ull << ci;
      if (live[ci] == 0) cf.second |= 1ull << ci;
    }
    return cf;
  };
  int cur = 0;
  // one outer iteration: sweep of m steps with the residual fused into its last
  // launch, per-instance reduction, convergence bookkeeping
  auto outer_iteration = [&](Config cf, unsigned seq) -> rm_status {
    int flips = 0;
    const int* ranges = nullptr;
    RM_TRY(sweep(pl, st, method, o->m, 0, o->m, omega, alpha, r32, ds, vs, cur, flips, rs.active, partial, &ranges,
                 -1, cf.first, cf.second));
    flips_per_outer = flips;
    rmk::launch_outer_flags(p, partial, ranges, ranges != nullptr ? pl->d_tranges.as<int>() : nullptr,
                            pl->d_cls.as<int>(), cf.first, ncls, res2, rs.rhs2, rs.target2, rs.best2, rs.since,
                            rs.gains, stall_min, stall_max, o->max_outer, rs.active, rs.count, rs.status, rs.pending,
                            n_active, ctx->host_word, ctx->host_cnt, seq, rs.tot, hist, o->hist_len, st);
    return RM_OK;
  };
  // A class word counts only if a launch of this solve wrote it (its stamp is at least
  // the solve's first launch number), or, after a synchronisation, whatever the stamp
  // (captured launches carry none).
  const unsigned seq0 = ctx->seq + 1u;
  auto read_counts = [&](bool synced) {
    for (int ci = 0; ci < ncls; ++ci) {
      const unsigned long long w = __atomic_load_n(ctx->host_cnt + ci, __ATOMIC_ACQUIRE);
      if (synced || (int)((unsigned)(w >> 32) - seq0) >= 0) live[ci] = (int)(w & 0xffffffffull);
    }
  };
  // every instance's rounds together are capped, so the solve is too
  const long long cap = (long long)(o->max_rounds + 1) * ((long long)o->max_outer + 1) + 2;
  long long issued = 0;  // outer iterations enqueued
  Config cfg = config();
  if (use_graph) {
    // The iteration returns to buffer set 0, so one captured iteration can be replayed;
    // captured on first use per configuration.  Synchronise every check_every replays,
    // read the counts and take the refinement steps of the rounds that ended.
    auto capture = [&](Config g) {
      const int cur0 = cur;
      GraphHolder& gh = graphs[g];
      if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess) {
        const rm_status sc = outer_iteration(g, 0u);
        const hipError_t ec = hipStreamEndCapture(st, &gh.graph);
        if (sc != RM_OK || ec != hipSuccess || cur != cur0 ||
            hipGraphInstantiate(&gh.exec, gh.graph, nullptr, nullptr, 0) != hipSuccess) {
          if (gh.graph != nullptr) (void)hipGraphDestroy(gh.graph);
          gh.graph = nullptr;
          gh.exec = nullptr;
          use_graph = false;
        }
      } else {
        use_graph = false;
      }
      (void)hipGetLastError();
      cur = cur0;
    };
    for (;;) {
      if (use_graph && (graphs.count(cfg) == 0 || graphs[cfg].exec == nullptr)) capture(cfg);
      if (use_graph)
        RM_HIP(hipGraphLaunch(graphs[cfg].exec, st));
      else
        RM_TRY(outer_iteration(cfg, 0u));  // the capture failed: launch directly
      ++issued;
      if (issued % o->check_every == 0 || issued >= cap) {
        RM_HIP(hipStreamSynchronize(st));
        const int left = (int)(__atomic_load_n(ctx->host_word, __ATOMIC_ACQUIRE) & 0xffffffffull);
        const int waiting = (int)(__atomic_load_n(ctx->host_word + 1, __ATOMIC_ACQUIRE) & 0xffffffffull);
        if (left == 0 || issued >= cap) break;
        if (waiting > 0) refine_step(issued, false);
        read_counts(true);
        cfg = config();
      }
    }
  } else {
    // One outer iteration stays queued while the host waits for the words of the
    // iteration before it, so the GPU does not idle for the host's round trip; the
    // configuration of each iteration follows the counts two iterations back.  When that
    // iteration reports rounds waiting for their refinement step, the step is queued
    // before the next iteration (words older than the last step are not taken for it).
    // The context's launch number advances before each launch, so a later solve never
    // mistakes a word of this one for its own.
    long long refined_after = -1;  // the last refinement step ran after this iteration
    auto issue = [&]() -> rm_status {
      ++issued;
      return outer_iteration(cfg, ++ctx->seq);
    };
    RM_TRY(issue());
    for (;;) {
      const bool more = issued < cap;
      if (more) RM_TRY(issue());
      const long long k = more ? issued - 2 : issued - 1;  // the iteration whose words are read
      unsigned long long w = 0;
      RM_TRY(wait_word(ctx, st, more ? ctx->seq - 1u : ctx->seq, w));
      const int left = (int)(w & 0xffffffffull);
      if (left == 0 || !more) break;
      const unsigned long long wp = __atomic_load_n(ctx->host_word + 1, __ATOMIC_ACQUIRE);
      const bool fresh = (int)((unsigned)(wp >> 32) - (unsigned)(seq0 + k)) >= 0;
      if (fresh && (wp & 0xffffffffull) > 0 && k > refined_after) {
        refine_step(issued, false);
        refined_after = issued - 1;
      }
      read_counts(false);
      cfg = config();
    }
  }
  // instances still in a solve or waiting at the cap: mark them as not converged
  double* hist_h = static_cast<double*>(ctx->pin);
  double* relres_h = hist_h + (size_t)H * B;
  int* status_h = reinterpret_cast<int*>(relres_h + B);
  int* rounds_h = status_h + B;
  int* tot_h = rounds_h + B;
  int* cnt_h = tot_h + B;
  RM_HIP(hipMemcpyAsync(hist_h, rs.history, (size_t)H * B * sizeof(double), hipMemcpyDeviceToHost, st));
  RM_HIP(hipMemcpyAsync(relres_h, rs.relres, B * sizeof(double), hipMemcpyDeviceToHost, st));
  RM_HIP(hipMemcpyAsync(status_h, rs.status, B * sizeof(int), hipMemcpyDeviceToHost, st));
  RM_HIP(hipMemcpyAsync(rounds_h, rs.round, B * sizeof(int), hipMemcpyDeviceToHost, st));
  RM_HIP(hipMemcpyAsync(tot_h, rs.tot, B * sizeof(int), hipMemcpyDeviceToHost, st));
  RM_HIP(hipMemcpyAsync(cnt_h, rs.count, B * sizeof(int), hipMemcpyDeviceToHost, st));
  std::vector<int> act_h(B, 0), pend_h(B, 0);
  RM_HIP(hipMemcpyAsync(act_h.data(), rs.active, B * sizeof(int), hipMemcpyDeviceToHost, st));
  RM_HIP(hipMemcpyAsync(pend_h.data(), rs.pending, B * sizeof(int), hipMemcpyDeviceToHost, st));
  RM_HIP(hipStreamSynchronize(st));
  rm_status worst = RM_OK;
  for (int bi = 0; bi < B; ++bi) {
    if ((act_h[bi] || pend_h[bi]) && status_h[bi] == 0) status_h[bi] = RM_ENOTCONV;
    if (status_h[bi] == RM_EDIVERGED) worst = RM_EDIVERGED;
    else if (status_h[bi] == RM_ENOTCONV && worst == RM_OK) worst = RM_ENOTCONV;
  }
  if (rep != nullptr) {
    for (int bi = 0; bi < B; ++bi) {
      if (rep->outer_iters)
        rep->outer_iters[bi] = (int32_t)std::min<long long>((long long)tot_h[bi] + cnt_h[bi], INT32_MAX);
      if (rep->rounds) rep->rounds[bi] = rounds_h[bi];
      if (rep->relres) rep->relres[bi] = relres_h[bi];
      if (rep->status) rep->status[bi] = status_h[bi];
    }
    if (rep->history != nullptr) std::memcpy(rep->history, hist_h, (size_t)H * B * sizeof(double));
  }
  RM_TRY(last_launch());
  if (worst != RM_OK) g_last_error = worst == RM_EDIVERGED ? "an instance diverged" : "an instance hit a cap";
  return worst;
}

rm_status validate_weights(const rm_plan_t* pl, int method, const rm_solve_opts* o, const float* omega,
                           const float* alpha) {
  if (o == nullptr) return fail(RM_EINVAL, "null opts");
  if (method < RM_RICHARDSON || method > RM_NAGEX) return fail(RM_EINVAL, "unknown method");
  if (o->m < 1 || o->m > kMaxM) return fail(RM_EINVAL, "m must be in 1..64");
  if (omega == nullptr) return fail(RM_EINVAL, "null omega");
  if (method != RM_RICHARDSON && alpha == nullptr) return fail(RM_EINVAL, "this method needs alpha");
  if (o->flags & ~(RM_FLAG_GRAPH | RM_FLAG_JACOBI | RM_FLAG_SSOR)) return fail(RM_EINVAL, "unknown flag");
  if ((o->flags & RM_FLAG_JACOBI) && (o->flags & RM_FLAG_SSOR))
    return fail(RM_EINVAL, "RM_FLAG_JACOBI and RM_FLAG_SSOR exclude each other");
  if ((o->flags & RM_FLAG_SSOR) && !(o->relax > 0.0 && o->relax < 2.0))
    return fail(RM_EINVAL, "SSOR needs 0 < relax < 2");
  if (o->flags & (RM_FLAG_JACOBI | RM_FLAG_SSOR))
    for (int b = 0; b < pl->B; ++b)
      if (pl->coef[(size_t)b * 8] == 0.0) return fail(RM_EINVAL, "the preconditioner needs a non-zero diagonal");
  return RM_OK;
}

// ---------------------------------------------------------------------------
// two-grid cycle (smoothing + sine-transform coarse correction)
// ---------------------------------------------------------------------------
rm_status twogrid_layout(rm_plan_t* pl) {
  auto& tg = pl->tg;
  if (!tg.coff.empty()) return RM_OK;
  std::vector<int64_t> coff((size_t)pl->B);
  int64_t c = 0;
  for (int b = 0; b < pl->B; ++b) {
    const int M = pl->inst[b].n + 1;
    if (M < 8 || M > rmk::kTgMaxFFT || (M & (M - 1)) != 0)
      return fail(RM_EUNSUPPORTED, "the two-grid cycle needs n + 1 a power of two in 8..1024 (instance " +
                                       std::to_string(b) + " has n = " + std::to_string(M - 1) + ")");
    const int nc = (M - 2) / 2;
    coff[b] = c;
    c += (int64_t)nc * nc;
  }
  tg.coff = std::move(coff);
  tg.Pc = c;
  return RM_OK;
}

rm_status twogrid_setup(rm_plan_t* pl, hipStream_t st) {
  auto& tg = pl->tg;
  if (tg.ready) return RM_OK;
  RM_TRY(twogrid_layout(pl));
  std::vector<rmk::TgInst> ti((size_t)pl->B);
  std::vector<Tile> rt, grp, stl;
  for (int b = 0; b < pl->B; ++b) {
    const int M = pl->inst[b].n + 1, nc = (M - 2) / 2;
    int lg = 0;
    while ((1 << lg) < M) ++lg;
    ti[b] = rmk::TgInst{tg.coff[b], nc, lg, (float)(1.0 / std::sqrt((double)M)), 0};
    for (int y = 0; y < nc; y += 8)
      for (int x = 0; x < nc; x += 64) rt.push_back(Tile{b, x, y, 0});
    for (int y = 0; y < nc; y += 8) grp.push_back(Tile{b, 0, y, 0});
    for (int y = 0; y < nc; y += 16)
      for (int x = 0; x < nc; x += 16) stl.push_back(Tile{b, x, y, (int)stl.size()});
    tg.mmax = std::max(tg.mmax, M);
  }
  while (rt.size() % 8 != 0) rt.push_back(Tile{-1, 0, 0, 0});
  std::vector<float2> tw(rmk::kTgMaxFFT / 2);
  for (int k = 0; k < rmk::kTgMaxFFT / 2; ++k) {
    const double a = 2.0 * M_PI * k / rmk::kTgMaxFFT;
    tw[k] = make_float2((float)std::cos(a), (float)-std::sin(a));
  }
  RM_TRY(tg.d_inst.ensure(ti.size() * sizeof(rmk::TgInst), st));
  RM_TRY(tg.d_rtiles.ensure(rt.size() * sizeof(Tile), st));
  RM_TRY(tg.d_groups.ensure(grp.size() * sizeof(Tile), st));
  RM_TRY(tg.d_tw.ensure(tw.size() * sizeof(float2), st));
  RM_HIP(hipStreamSynchronize(st));
  RM_HIP(hipMemcpy(tg.d_inst.ptr, ti.data(), ti.size() * sizeof(rmk::TgInst), hipMemcpyHostToDevice));
  RM_HIP(hipMemcpy(tg.d_rtiles.ptr, rt.data(), rt.size() * sizeof(Tile), hipMemcpyHostToDevice));
  RM_HIP(hipMemcpy(tg.d_groups.ptr, grp.data(), grp.size() * sizeof(Tile), hipMemcpyHostToDevice));
  RM_HIP(hipMemcpy(tg.d_tw.ptr, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice));
  RM_TRY(tg.d_stiles.ensure(std::max<size_t>(stl.size(), 1) * sizeof(Tile), st));
  if (!stl.empty())
    RM_HIP(hipMemcpy(tg.d_stiles.ptr, stl.data(), stl.size() * sizeof(Tile), hipMemcpyHostToDevice));
  tg.nstiles = (int)stl.size();
  tg.nrtiles = (int)rt.size();
  tg.ngroups = (int)grp.size();
  const size_t cb = (size_t)std::max<int64_t>(tg.Pc, 1) * sizeof(float);
  RM_TRY(tg.c0.ensure(cb, st));
  RM_TRY(tg.c1.ensure(cb, st));
  tg.ready = true;
  return RM_OK;
}

// u_out = u_in + P S (symbol * (S R (f - A u_in) S)) S   (u_out may equal u_in)
void twogrid_correct(rm_plan_t* pl, hipStream_t st, const float* f, const float* u_in, float* u_out,
                     const float* symbol) {
  const PlanDev p = pl->dev();
  const rmk::TgDev g = pl->tgdev();
  auto& tg = pl->tg;
  float* c0 = tg.c0.as<float>();
  float* c1 = tg.c1.as<float>();
  const Tile* grp = tg.d_groups.as<Tile>();
  rmk::launch_tg_restrict(0, p, g, tg.d_rtiles.as<Tile>(), tg.nrtiles, f, u_in, c0, 1.f, st);
  rmk::launch_tg_dst(0, g, grp, tg.ngroups, tg.mmax, c0, c1, nullptr, nullptr, nullptr, nullptr, st);
  rmk::launch_tg_dst(1, g, grp, tg.ngroups, tg.mmax, c1, c1, symbol, nullptr, nullptr, nullptr, st);
  rmk::launch_tg_dst(2, g, grp, tg.ngroups, tg.mmax, c1, c0, nullptr, nullptr, nullptr, nullptr, st);
  rmk::launch_tg_prolong(p, g, c0, u_in, u_out, st);
}

rm_status twogrid_forward(rm_ctx* ctx, rm_plan_t* pl, int method, const rm_solve_opts* o, const float* omega,
                          const float* alpha, const float* symbol, const float* b, float* x, float* ckpt,
                          double* hist) {
  hipStream_t st = ctx->stream;
  const int64_t P = pl->P;
  RM_TRY(twogrid_setup(pl, st));
  RM_TRY(pl->vecA.ensure(vec_bytes<float>(pl), st));
  RM_TRY(pl->vecB.ensure(vec_bytes<float>(pl), st));
  RM_TRY(pl->vecC.ensure(vec_bytes<float>(pl), st));
  if (pl->use_block) RM_TRY(build_exec(pl, st));
  RM_TRY(pl->partial.ensure(partial_slots(pl) * 2 * sizeof(double), st));
  const PlanDev p = pl->dev();
  float* fu[2] = {x, pl->vecB.as<float>()};
  float* fv[2] = {pl->vecA.as<float>(), pl->vecC.as<float>()};
  int cur = 0, flips = 0;
  for (int k = 0; k < o->K; ++k) {
    if (ckpt != nullptr)
      RM_HIP(hipMemcpyAsync(ckpt + (int64_t)k * P, fu[cur], P * sizeof(float), hipMemcpyDeviceToDevice, st));
    rmk::launch_fill_f32(fv[cur], 0.f, P, st);
    const int* ranges = nullptr;
    RM_TRY(sweep(pl, st, method, o->m, 0, o->m, omega, alpha, b, fu, fv, cur, flips, nullptr, nullptr, &ranges));
    twogrid_correct(pl, st, b, fu[cur], fu[cur], symbol);
    if (hist != nullptr) {
      rmk::launch_residual<float>(p, p.tiles, p.ntiles, b, fu[cur], nullptr, pl->partial.as<double>(), nullptr, st);
      rmk::launch_reduce_partials(p, pl->partial.as<double>(), hist + (int64_t)k * pl->B, nullptr, 1, nullptr, st);
    }
  }
  if (cur == 1) RM_HIP(hipMemcpyAsync(x, fu[1], P * sizeof(float), hipMemcpyDeviceToDevice, st));
  return last_launch();
}

}  // namespace

namespace {

std::string tune_key(const char* arch, const rm_plan_s::ClassExec& c, int m, int method) {
  char buf[256];
  std::snprintf(buf, sizeof buf, "%s n=%d B=%zu m=%d method=%d", arch, c.n, c.insts.size(), m, method);
  return buf;
}

}  // namespace

extern "C" {

// ---------------------------------------------------------------------------
// Scratch of rm_residual_noalloc: the per-tile partial sums live in a file-scope device
// array (one copy per GPU, held until the process ends) instead of plan scratch.  In
// host code `scratch` names a host-side stand-in, never the device memory: its device
// address is taken once per device with hipGetSymbolAddress and kept in
// g_noalloc_addr, and only that address is passed to kernels.
// ---------------------------------------------------------------------------
__device__ __align__(256) double scratch[RM_NOALLOC_MAX_TILES * 2];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
double* g_noalloc_addr[kMaxDevices] = {};

// The device address of `scratch` on `device` (which must be current), looked up on
// the first call for that device.
rm_status noalloc_address(int device, double** out) {
  if (device < 0 || device >= kMaxDevices) return fail(RM_EUNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (g_noalloc_addr[device] == nullptr) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) {
      (void)hipGetLastError();
      return fail(RM_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_noalloc_addr[device] = static_cast<double*>(ptr);
  }
  *out = g_noalloc_addr[device];
  return RM_OK;
}
}  // namespace

const char* rm_status_string(rm_status s) {
  switch (s) {
    case RM_OK: return "ok";
    case RM_EINVAL: return "invalid argument";
    case RM_ENOMEM: return "out of device memory";
    case RM_EHIP: return "HIP runtime error";
    case RM_ENOTCONV: return "not converged within the caps";
    case RM_EDIVERGED: return "diverged";
    case RM_EUNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* rm_last_error(void) { return g_last_error.c_str(); }

rm_status rm_create(rm_ctx** out, int32_t device, void* hip_stream) {
  if (out == nullptr) return fail(RM_EINVAL, "null output handle");
  int ndev = 0;
  RM_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(RM_EINVAL, "no such device");
  RM_HIP(hipSetDevice(device));
  rm_ctx* c = new rm_ctx;
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  // coherent, so that a kernel's system-scope store is what the host reads
  if (hipHostMalloc((void**)&c->host_word, 64, hipHostMallocCoherent) != hipSuccess) {
    delete c;
    return fail(RM_ENOMEM, "pinned host allocation failed");
  }
  __atomic_store_n(c->host_word, 0ull, __ATOMIC_RELEASE);
  const rm_status sa = noalloc_address(device, &c->noalloc_scratch);
  if (sa != RM_OK) {
    (void)hipHostFree(c->host_word);
    delete c;
    return sa;
  }
  *out = c;
  return RM_OK;
}

rm_status rm_destroy(rm_ctx* ctx) {
  if (ctx == nullptr) return RM_OK;
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->work != nullptr) (void)hipStreamSynchronize(ctx->work);
  for (rm_plan_s* pl : ctx->plans) pl->ctx = nullptr;
  if (ctx->host_word != nullptr) (void)hipHostFree(ctx->host_word);
  if (ctx->host_cnt != nullptr) (void)hipHostFree(ctx->host_cnt);
  if (ctx->pin != nullptr) (void)hipHostFree(ctx->pin);
  if (ctx->work != nullptr) (void)hipStreamDestroy(ctx->work);
  if (ctx->handoff != nullptr) (void)hipEventDestroy(ctx->handoff);
  delete ctx;
  return RM_OK;
}

rm_status rm_plan(rm_ctx* ctx, int32_t B, const rm_instance* inst, const int64_t* offsets, rm_plan_t** out) {
  if (ctx == nullptr || out == nullptr) return fail(RM_EINVAL, "null context or output handle");
  if (B < 1 || inst == nullptr) return fail(RM_EINVAL, "need B >= 1 instances");
  for (int b = 0; b < B; ++b) {
    const rm_instance& in = inst[b];
    if (in.n < 1 || in.n > kMaxN) return fail(RM_EINVAL, "instance " + std::to_string(b) + ": n out of range");
    if (in.op == RM_Q1_ANISO) {
      if (!(in.eps > 0.0 && in.eps <= 1.0) || !std::isfinite(in.theta))
        return fail(RM_EINVAL, "instance " + std::to_string(b) + ": eps must be in (0, 1], theta finite");
    } else if (in.op == RM_FD5_HELMHOLTZ) {
      if (!std::isfinite(in.kappa) || in.kappa < 0.0)
        return fail(RM_EINVAL, "instance " + std::to_string(b) + ": kappa must be finite and >= 0");
    } else {
      return fail(RM_EINVAL, "instance " + std::to_string(b) + ": unknown op");
    }
  }
  if (offsets != nullptr) {
    // caller-chosen placement: increasing starts, each instance's n^2 points before the next
    if (offsets[0] < 0) return fail(RM_EINVAL, "offsets[0] must be >= 0");
    for (int b = 0; b < B; ++b)
      if (offsets[b + 1] - offsets[b] < (int64_t)inst[b].n * inst[b].n)
        return fail(RM_EINVAL, "offsets leave instance " + std::to_string(b) + " fewer than n^2 points");
    if (offsets[B] > ((int64_t)1 << 40)) return fail(RM_EINVAL, "offsets beyond 2^40 points");
  }
  RM_HIP(hipSetDevice(ctx->device));
  rm_plan_t* pl = new rm_plan_t;
  pl->ctx = ctx;
  pl->B = B;
  pl->inst.assign(inst, inst + B);
  pl->off.assign(B + 1, offsets != nullptr ? offsets[0] : 0);
  pl->coef.assign((size_t)B * 8, 0.0);
  pl->gersh.assign(B, 0.0);
  std::vector<float> coef32((size_t)B * 8, 0.f), mu((size_t)B * 2), g32(B);
  pl->insts.resize(B);
  for (int b = 0; b < B; ++b) {
    const int n = inst[b].n;
    pl->off[b + 1] = offsets != nullptr ? offsets[b + 1] : pl->off[b] + (int64_t)n * n;
    double* c = &pl->coef[(size_t)b * 8];
    stencil_coefficients(inst[b], c);
    c[5] = c[0] != 0.0 ? 1.0 / c[0] : 0.0;  // 1/D for weighted-Jacobi preconditioning
    pl->gersh[b] = std::fabs(c[0]) + 2.0 * (std::fabs(c[1]) + std::fabs(c[2]) + std::fabs(c[3]) + std::fabs(c[4]));
    for (int k = 0; k < 8; ++k) coef32[(size_t)b * 8 + k] = (float)c[k];
    g32[b] = (float)pl->gersh[b];
    if (inst[b].op == RM_Q1_ANISO) {
      mu[2 * b] = (float)std::log10(inst[b].eps);
      mu[2 * b + 1] = (float)inst[b].theta;
    } else {
      mu[2 * b] = 0.f;
      mu[2 * b + 1] = (float)inst[b].kappa;
    }
    Inst& I = pl->insts[b];
    I.off = pl->off[b];
    I.n = n;
    I.tile_begin = (int)pl->tiles.size();
    for (int y0 = 0; y0 < n; y0 += rmk::TY)
      for (int x0 = 0; x0 < n; x0 += rmk::TX) pl->tiles.push_back(Tile{b, x0, y0, (int)pl->tiles.size()});
    I.tile_end = (int)pl->tiles.size();
    I.pad = 0;
  }
  while (pl->tiles.size() % 8 != 0) pl->tiles.push_back(Tile{-1, 0, 0, (int)pl->tiles.size()});
  pl->P = pl->off[B];
  init_classes(pl);
  hipStream_t st = ctx->stream;
  rm_status s = RM_OK;
  auto up = [&](DevBuf& d, const void* src, size_t bytes) {
    if (s != RM_OK) return;
    s = d.ensure(bytes, st);
    if (s != RM_OK) return;
    if (hipMemcpy(d.ptr, src, bytes, hipMemcpyHostToDevice) != hipSuccess) s = fail(RM_EHIP, "plan upload failed");
  };
  up(pl->d_tiles, pl->tiles.data(), pl->tiles.size() * sizeof(Tile));
  up(pl->d_inst, pl->insts.data(), pl->insts.size() * sizeof(Inst));
  up(pl->d_coef32, coef32.data(), coef32.size() * sizeof(float));
  up(pl->d_coef64, pl->coef.data(), pl->coef.size() * sizeof(double));
  up(pl->d_mu, mu.data(), mu.size() * sizeof(float));
  up(pl->d_gersh, g32.data(), g32.size() * sizeof(float));
  if (s != RM_OK) {
    delete pl;
    return s;
  }
  ctx->plans.push_back(pl);
  *out = pl;
  return RM_OK;
}

rm_status rm_plan_free(rm_plan_t* plan) {
  if (plan == nullptr) return RM_OK;
  if (plan->ctx != nullptr) {
    (void)hipStreamSynchronize(plan->ctx->stream);
    if (plan->ctx->work != nullptr) (void)hipStreamSynchronize(plan->ctx->work);
    auto& v = plan->ctx->plans;
    v.erase(std::remove(v.begin(), v.end(), plan), v.end());
  }
  delete plan;
  return RM_OK;
}

int32_t rm_plan_batch(const rm_plan_t* plan) { return plan == nullptr ? -1 : plan->B; }
int64_t rm_plan_points(const rm_plan_t* plan) { return plan == nullptr ? -1 : plan->P; }

rm_status rm_plan_offsets(const rm_plan_t* plan, int64_t* off) {
  if (plan == nullptr || off == nullptr) return fail(RM_EINVAL, "null argument");
  std::memcpy(off, plan->off.data(), plan->off.size() * sizeof(int64_t));
  return RM_OK;
}

rm_status rm_plan_coefficients(const rm_plan_t* plan, double* coef, double* gersh) {
  if (plan == nullptr) return fail(RM_EINVAL, "null plan");
  for (int b = 0; b < plan->B; ++b) {
    if (coef != nullptr)
      for (int k = 0; k < 5; ++k) coef[b * 5 + k] = plan->coef[(size_t)b * 8 + k];
    if (gersh != nullptr) gersh[b] = plan->gersh[b];
  }
  return RM_OK;
}

rm_status rm_apply_A(rm_ctx* ctx, const rm_plan_t* plan, int32_t dtype, const void* x, void* y) {
  RM_TRY(check_ctx_plan(ctx, plan));
  if (x == nullptr || y == nullptr) return fail(RM_EINVAL, "null vector");
  if (x == y) return fail(RM_EINVAL, "x and y must not overlap");
  const PlanDev p = plan->dev();
  if (dtype == RM_F32)
    rmk::launch_apply<float>(p, p.tiles, p.ntiles, (const float*)x, (float*)y, ctx->stream);
  else if (dtype == RM_F64)
    rmk::launch_apply<double>(p, p.tiles, p.ntiles, (const double*)x, (double*)y, ctx->stream);
  else
    return fail(RM_EINVAL, "unknown dtype");
  return last_launch();
}

rm_status rm_residual(rm_ctx* ctx, const rm_plan_t* plan, int32_t dtype, const void* b, const void* x, void* r,
                      double* r2, double* b2, float* rel2) {
  RM_TRY(check_ctx_plan(ctx, plan));
  if (b == nullptr || x == nullptr) return fail(RM_EINVAL, "null vector");
  if (r != nullptr && r == x) return fail(RM_EINVAL, "r and x must not overlap");
  rm_plan_t* pl = const_cast<rm_plan_t*>(plan);
  RM_TRY(pl->partial.ensure(pl->tiles.size() * 2 * sizeof(double), ctx->stream));
  const PlanDev p = pl->dev();
  double* part = pl->partial.as<double>();
  if (dtype == RM_F32)
    rmk::launch_residual<float>(p, p.tiles, p.ntiles, (const float*)b, (const float*)x, (float*)r, part, nullptr,
                                ctx->stream);
  else if (dtype == RM_F64)
    rmk::launch_residual<double>(p, p.tiles, p.ntiles, (const double*)b, (const double*)x, (double*)r, part,
                                 nullptr, ctx->stream);
  else
    return fail(RM_EINVAL, "unknown dtype");
  if (r2 != nullptr || b2 != nullptr || rel2 != nullptr)
    rmk::launch_reduce_partials(p, part, r2, b2, 1, rel2, ctx->stream);
  return last_launch();
}

rm_status rm_residual_noalloc(rm_ctx* ctx, const rm_plan_t* plan, int32_t dtype, const void* b, const void* x,
                              void* r, double* r2, double* b2, float* rel2) {
  RM_TRY(check_ctx_plan(ctx, plan));
  if (b == nullptr || x == nullptr) return fail(RM_EINVAL, "null vector");
  if (r != nullptr && r == x) return fail(RM_EINVAL, "r and x must not overlap");
  if (dtype != RM_F32 && dtype != RM_F64) return fail(RM_EINVAL, "unknown dtype");
  if (plan->tiles.size() > (size_t)RM_NOALLOC_MAX_TILES)
    return fail(RM_EINVAL, "plan has " + std::to_string(plan->tiles.size()) + " tiles; rm_residual_noalloc holds " +
                               std::to_string(RM_NOALLOC_MAX_TILES));
  if (ctx->noalloc_scratch == nullptr) return fail(RM_EHIP, "no scratch address for this context's device");
  const PlanDev p = plan->dev();
  double* part = ctx->noalloc_scratch;  // every used slot is written by the residual launch before it is read
  if (dtype == RM_F32)
    rmk::launch_residual<float>(p, p.tiles, p.ntiles, (const float*)b, (const float*)x, (float*)r, part, nullptr,
                                ctx->stream);
  else
    rmk::launch_residual<double>(p, p.tiles, p.ntiles, (const double*)b, (const double*)x, (double*)r, part,
                                 nullptr, ctx->stream);
  if (r2 != nullptr || b2 != nullptr || rel2 != nullptr)
    rmk::launch_reduce_partials(p, part, r2, b2, 1, rel2, ctx->stream);
  return last_launch();
}

rm_status rm_solve(rm_ctx* ctx, const rm_plan_t* plan, int32_t method, const rm_solve_opts* opts,
                   const float* omega, const float* alpha, const void* b, void* x, void* ckpt, double* hist,
                   rm_report* rep) {
  RM_TRY(check_ctx_plan(ctx, plan));
  RM_TRY(validate_weights(plan, method, opts, omega, alpha));
  if (b == nullptr || x == nullptr) return fail(RM_EINVAL, "null b or x");
  rm_plan_t* pl = const_cast<rm_plan_t*>(plan);
  set_precond(pl, opts);
  const int m = opts->m;
  if (opts->mode == RM_UNROLL) {
    if (opts->K < 0 || opts->K % m != 0) return fail(RM_EINVAL, "K must be a non-negative multiple of m");
    if (opts->ckpt_every < 0 || (opts->ckpt_every > 0 && opts->K % opts->ckpt_every != 0))
      return fail(RM_EINVAL, "ckpt_every must divide K");
    if (ckpt != nullptr && opts->ckpt_every == 0) return fail(RM_EINVAL, "ckpt given but ckpt_every = 0");
    if (opts->dtype == RM_F32)
      return solve_unroll<float>(ctx, pl, method, opts, omega, alpha, (const float*)b, (float*)x,
                                 (float*)ckpt, hist);
    if (opts->dtype == RM_F64)
      return solve_unroll<double>(ctx, pl, method, opts, omega, alpha, (const double*)b, (double*)x,
                                  (double*)ckpt, hist);
    return fail(RM_EINVAL, "unknown dtype");
  }
  if (opts->mode == RM_TO_TOL) {
    if (ckpt != nullptr) return fail(RM_EINVAL, "RM_TO_TOL takes no ckpt");
    if (opts->hist_len < 0 || (hist != nullptr && opts->hist_len == 0))
      return fail(RM_EINVAL, "RM_TO_TOL with hist needs hist_len >= 1 (and hist_len >= 0 always)");
    if (!(opts->tol > 0.0) || !(opts->tol_inner > 0.0 && opts->tol_inner < 1.0))
      return fail(RM_EINVAL, "need tol > 0 and 0 < tol_inner < 1");
    if (opts->max_outer < 1 || opts->max_rounds < 1 || opts->check_every < 1)
      return fail(RM_EINVAL, "max_outer, max_rounds and check_every must be >= 1");
    const rm_status s = solve_to_tol(ctx, pl, method, opts, omega, alpha, (const double*)b, (double*)x, hist, rep);
    if (s != RM_OK && s != RM_ENOTCONV && s != RM_EDIVERGED && ctx->work != nullptr) {
      // an error left the round loop early: wait for what it had queued on the solve's
      // stream, so that the caller may free x and b, or the context, once this returns
      const std::string keep = g_last_error;
      (void)hipStreamSynchronize(ctx->work);
      g_last_error = keep;
    }
    return s;
  }
  return fail(RM_EINVAL, "unknown mode");
}

rm_status rm_solve_adjoint(rm_ctx* ctx, const rm_plan_t* plan, int32_t method, const rm_solve_opts* opts,
                           const float* omega, const float* alpha, const float* b, const void* ckpt_v,
                           const float* g_uK, const float* g_loss, float* d_omega, float* d_alpha, float* d_b,
                           float* loss) {
  RM_TRY(check_ctx_plan(ctx, plan));
  RM_TRY(validate_weights(plan, method, opts, omega, alpha));
  if (opts->mode != RM_UNROLL) return fail(RM_EINVAL, "the adjoint follows an RM_UNROLL solve");
  if (opts->dtype != RM_F32) return fail(RM_EUNSUPPORTED, "the adjoint runs in FP32 only");
  const int m = opts->m, K = opts->K, E = opts->ckpt_every;
  if (K < 1 || K % m != 0) return fail(RM_EINVAL, "K must be a positive multiple of m");
  if (E < 1 || K % E != 0) return fail(RM_EINVAL, "ckpt_every must be >= 1 and divide K");
  if (b == nullptr || ckpt_v == nullptr || d_omega == nullptr || d_alpha == nullptr)
    return fail(RM_EINVAL, "null b, ckpt, d_omega or d_alpha");
  rm_plan_t* pl = const_cast<rm_plan_t*>(plan);
  set_precond(pl, opts);
  hipStream_t st = ctx->stream;
  const int B = pl->B;
  const int64_t P = pl->P;
  const float* ckpt = static_cast<const float*>(ckpt_v);
  const int na = method == RM_NAGEX ? 2 : 1;  // momentum gradient blocks of d_alpha
  const size_t fbytes = vec_bytes<float>(pl);
  RM_TRY(pl->states.ensure(fbytes * 2 * (size_t)(E + 1), st));
  RM_TRY(pl->vecA.ensure(fbytes, st));  // ub0
  RM_TRY(pl->vecB.ensure(fbytes, st));  // vb0
  RM_TRY(pl->vecC.ensure(fbytes, st));  // ub1
  RM_TRY(pl->vecD.ensure(fbytes, st));  // vb1
  RM_TRY(pl->vecE.ensure(fbytes, st));  // r_K
  if (pl->use_block) RM_TRY(build_exec(pl, st));
  const int nslot = (int)partial_slots(pl);
  RM_TRY(pl->partial.ensure((size_t)nslot * 4 * sizeof(double) * E, st));
  RM_TRY(pl->red.ensure((size_t)B * 4 * sizeof(double), st));
  RM_TRY(pl->acc.ensure((size_t)B * m * (1 + na) * sizeof(double), st));
  float* S = pl->states.as<float>();  // slot t: (u, v) before step c*E + t, t = 1..E; slot 0 unused
                                      // (the checkpoint itself serves as slot 0)
  float* ubs[2] = {pl->vecA.as<float>(), pl->vecC.as<float>()};
  float* vbs[2] = {pl->vecB.as<float>(), pl->vecD.as<float>()};
  float* rK = pl->vecE.as<float>();
  double* partial = pl->partial.as<double>();
  double* r2b2 = pl->red.as<double>();
  double* acc_w = pl->acc.as<double>();
  double* acc_a = acc_w + (size_t)B * m;
  const PlanDev p = pl->dev();
  const int nseg = K / E;
  auto su = [&](int c, int t) -> const float* { return t == 0 ? ckpt + (int64_t)c * 2 * P : S + (int64_t)t * 2 * P; };
  auto sv = [&](int c, int t) -> const float* {
    return t == 0 ? ckpt + (int64_t)c * 2 * P + P : S + (int64_t)t * 2 * P + P;
  };
  // forward recompute of segment c into slots 1..E-1; the last segment also
  // produces slot E, the final state u_K.  The blocked kernels store every
  // intermediate state of a launch and reproduce the one-step kernel bit for bit.
  auto recompute = [&](int c) -> rm_status {
    const int steps = c == nseg - 1 ? E : E - 1;
    if (!blocked(pl)) {
      for (int t = 0; t < steps; ++t) {
        float* uo = S + (int64_t)(t + 1) * 2 * P;
        one_step<float>(pl, p, method, omega, alpha, m, (c * E + t) % m, b, su(c, t), sv(c, t), uo, uo + P, nullptr,
                        st);
      }
      return RM_OK;
    }
    for (auto& cl : pl->classes) {
      for (int s0 = 0; s0 < steps;) {
        const int t = std::min(cl.T, steps - s0);
        float* uo = S + (int64_t)(s0 + t) * 2 * P;
        if (!launch_class(cl, t, method, p, omega, alpha, m, c * E + s0, b, su(c, s0), sv(c, s0), uo, uo + P, nullptr,
                          nullptr, st, S + (int64_t)(s0 + 1) * 2 * P, 2 * P))
          return fail(RM_EUNSUPPORTED, "block kernel configuration not built");
        s0 += t;
      }
    }
    return RM_OK;
  };
  rmk::launch_fill_f64(acc_w, 0.0, (int64_t)B * m * (1 + na), st);
  rmk::launch_fill_f32(vbs[0], 0.f, P, st);
  // terminal values
  RM_TRY(recompute(nseg - 1));
  const float* uK = S + (int64_t)E * 2 * P;
  if (g_uK == nullptr) {
    rmk::launch_residual<float>(p, p.tiles, p.ntiles, b, uK, rK, partial, nullptr, st);
    rmk::launch_reduce_partials(p, partial, r2b2, r2b2 + 1, 2, nullptr, st);
    rmk::launch_adj_terminal(p, b, rK, r2b2, g_loss, ubs[0], d_b, loss, st);
  } else {
    RM_HIP(hipMemcpyAsync(ubs[0], g_uK, P * sizeof(float), hipMemcpyDeviceToDevice, st));
    if (d_b != nullptr) rmk::launch_fill_f32(d_b, 0.f, P, st);
  }
  int cur = 0;
  for (int c = nseg - 1; c >= 0; --c) {
    if (c != nseg - 1) RM_TRY(recompute(c));
    const int* ranges = nullptr;
    RM_TRY(reverse_segment(pl, p, st, method, omega, alpha, m, c * E, E, [&](int t) { return su(c, t); },
                           [&](int t) { return sv(c, t); }, b, ubs, vbs, cur, d_b, partial, nslot, &ranges));
    rmk::launch_adj_accumulate(method, p, partial, nslot, E, c * E, m, acc_w, acc_a, st, ranges);
  }
  rmk::launch_f64_to_f32(acc_w, d_omega, (int64_t)B * m, st);
  rmk::launch_f64_to_f32(acc_a, d_alpha, (int64_t)B * m * na, st);
  return last_launch();
}

namespace {
// Scratch of the symbol network: two activation and two gradient planes of 16 channels,
// the symbol and its log-gradient, per-tile partials of the largest layer.
rm_status symbolnet_prepare(rm_ctx* ctx, rm_plan_t* pl) {
  RM_TRY(twogrid_setup(pl, ctx->stream));
  for (int b = 0; b < pl->B; ++b)
    if (pl->inst[b].op != RM_FD5_HELMHOLTZ) return fail(RM_EINVAL, "the symbol network needs Helmholtz instances");
  auto& tg = pl->tg;
  const size_t planes = (size_t)std::max<int64_t>(tg.Pc, 1) * 16 * sizeof(float);
  const size_t one = (size_t)std::max<int64_t>(tg.Pc, 1) * sizeof(float);
  RM_TRY(tg.sa1.ensure(planes, ctx->stream));
  RM_TRY(tg.sa2.ensure(planes, ctx->stream));
  RM_TRY(tg.ssym.ensure(one, ctx->stream));
  return RM_OK;
}
}  // namespace

int32_t rm_symbolnet_param_count(void) { return rmk::symbolnet_param_count(); }

rm_status rm_symbolnet_forward(rm_ctx* ctx, const rm_plan_t* plan, const float* params, float* symbol) {
  RM_TRY(check_ctx_plan(ctx, plan));
  if (params == nullptr || symbol == nullptr) return fail(RM_EINVAL, "null params or symbol");
  rm_plan_t* pl = const_cast<rm_plan_t*>(plan);
  RM_TRY(symbolnet_prepare(ctx, pl));
  auto& tg = pl->tg;
  rmk::launch_symbolnet_forward(pl->dev(), pl->tgdev(), tg.d_stiles.as<Tile>(), tg.nstiles, tg.Pc, params,
                                tg.sa1.as<float>(), tg.sa2.as<float>(), symbol, ctx->stream);
  return last_launch();
}

rm_status rm_symbolnet_backward(rm_ctx* ctx, const rm_plan_t* plan, const float* params, const float* d_symbol,
                                float* d_params) {
  RM_TRY(check_ctx_plan(ctx, plan));
  if (params == nullptr || d_symbol == nullptr || d_params == nullptr)
    return fail(RM_EINVAL, "null params, d_symbol or d_params");
  rm_plan_t* pl = const_cast<rm_plan_t*>(plan);
  RM_TRY(symbolnet_prepare(ctx, pl));
  auto& tg = pl->tg;
  hipStream_t st = ctx->stream;
  const size_t planes = (size_t)std::max<int64_t>(tg.Pc, 1) * 16 * sizeof(float);
  RM_TRY(tg.sg1.ensure(planes, st));
  RM_TRY(tg.sg2.ensure(planes, st));
  RM_TRY(tg.sgz.ensure((size_t)std::max<int64_t>(tg.Pc, 1) * sizeof(float), st));
  RM_TRY(tg.spart.ensure((size_t)std::max(tg.nstiles, 1) * (16 * 16 * 9 + 16) * sizeof(float), st));
  // FP64 sums of the partials over groups of 64 tiles
  RM_TRY(tg.sgsum.ensure((size_t)std::max((tg.nstiles + 63) / 64, 1) * (16 * 16 * 9 + 16) * sizeof(double), st));
  // the forward activations of these parameters, then the reverse pass
  rmk::launch_symbolnet_forward(pl->dev(), pl->tgdev(), tg.d_stiles.as<Tile>(), tg.nstiles, tg.Pc, params,
                                tg.sa1.as<float>(), tg.sa2.as<float>(), tg.ssym.as<float>(), st);
  rmk::launch_symbolnet_backward(pl->dev(), pl->tgdev(), tg.d_stiles.as<Tile>(), tg.nstiles, tg.Pc, params,
                                 tg.sa1.as<float>(), tg.sa2.as<float>(), tg.ssym.as<float>(), d_symbol,
                                 tg.sgz.as<float>(), tg.sg1.as<float>(), tg.sg2.as<float>(), tg.spart.as<float>(),
                                 tg.sgsum.as<double>(), d_params, st);
  return last_launch();
}

int64_t rm_plan_coarse_points(const rm_plan_t* plan) {
  if (plan == nullptr) return -1;
  rm_plan_t* pl = const_cast<rm_plan_t*>(plan);
  if (twogrid_layout(pl) != RM_OK) return -1;
  return pl->tg.Pc;
}

rm_status rm_plan_coarse_offsets(const rm_plan_t* plan, int64_t* coff) {
  if (plan == nullptr || coff == nullptr) return fail(RM_EINVAL, "null plan or coff");
  rm_plan_t* pl = const_cast<rm_plan_t*>(plan);
  RM_TRY(twogrid_layout(pl));
  std::memcpy(coff, pl->tg.coff.data(), pl->tg.coff.size() * sizeof(int64_t));
  return RM_OK;
}

rm_status rm_twogrid_solve(rm_ctx* ctx, const rm_plan_t* plan, int32_t method, const rm_solve_opts* opts,
                           const float* omega, const float* alpha, const float* symbol, const float* b, float* x,
                           float* ckpt, double* hist) {
  RM_TRY(check_ctx_plan(ctx, plan));
  RM_TRY(validate_weights(plan, method, opts, omega, alpha));
  if (opts->mode != RM_UNROLL || opts->dtype != RM_F32)
    return fail(RM_EUNSUPPORTED, "the two-grid cycle runs as an FP32 RM_UNROLL of K cycles");
  if (opts->K < 0) return fail(RM_EINVAL, "K (cycles) must be >= 0");
  if (symbol == nullptr || b == nullptr || x == nullptr) return fail(RM_EINVAL, "null symbol, b or x");
  rm_plan_t* pl = const_cast<rm_plan_t*>(plan);
  RM_TRY(twogrid_layout(pl));
  set_precond(pl, opts);
  return twogrid_forward(ctx, pl, method, opts, omega, alpha, symbol, b, x, ckpt, hist);
}

rm_status rm_twogrid_adjoint(rm_ctx* ctx, const rm_plan_t* plan, int32_t method, const rm_solve_opts* opts,
                             const float* omega, const float* alpha, const float* symbol, const float* b,
                             const float* ckpt, const float* g_uK, const float* g_loss, float* d_omega,
                             float* d_alpha, float* d_symbol, float* d_b, float* loss) {
  RM_TRY(check_ctx_plan(ctx, plan));
  RM_TRY(validate_weights(plan, method, opts, omega, alpha));
  if (opts->mode != RM_UNROLL || opts->dtype != RM_F32)
    return fail(RM_EUNSUPPORTED, "the two-grid adjoint follows an FP32 RM_UNROLL of K cycles");
  if (opts->K < 1) return fail(RM_EINVAL, "K (cycles) must be >= 1");
  if (symbol == nullptr || b == nullptr || ckpt == nullptr || d_omega == nullptr || d_alpha == nullptr ||
      d_symbol == nullptr)
    return fail(RM_EINVAL, "null symbol, b, ckpt, d_omega, d_alpha or d_symbol");
  rm_plan_t* pl = const_cast<rm_plan_t*>(plan);
  RM_TRY(twogrid_layout(pl));
  set_precond(pl, opts);
  hipStream_t st = ctx->stream;
  RM_TRY(twogrid_setup(pl, st));
  auto& tg = pl->tg;
  const int B = pl->B, m = opts->m, K = opts->K;
  const int64_t P = pl->P;
  const int na = method == RM_NAGEX ? 2 : 1;
  const size_t fbytes = vec_bytes<float>(pl);
  const size_t cbytes = (size_t)std::max<int64_t>(tg.Pc, 1) * sizeof(float);
  RM_TRY(pl->states.ensure(fbytes * 2 * (size_t)(m + 1), st));
  RM_TRY(pl->vecA.ensure(fbytes, st));
  RM_TRY(pl->vecB.ensure(fbytes, st));
  RM_TRY(pl->vecC.ensure(fbytes, st));
  RM_TRY(pl->vecD.ensure(fbytes, st));
  RM_TRY(pl->vecE.ensure(fbytes, st));
  RM_TRY(tg.fine2.ensure(fbytes, st));
  RM_TRY(tg.zero.ensure(fbytes, st));
  RM_TRY(tg.shat.ensure(cbytes, st));
  if (pl->use_block) RM_TRY(build_exec(pl, st));
  const int nslot = (int)partial_slots(pl);
  RM_TRY(pl->partial.ensure((size_t)nslot * 4 * sizeof(double) * m, st));
  RM_TRY(pl->red.ensure((size_t)B * 4 * sizeof(double), st));
  RM_TRY(pl->acc.ensure((size_t)B * m * (1 + na) * sizeof(double), st));
  const PlanDev p = pl->dev();
  const rmk::TgDev g = pl->tgdev();
  float* S = pl->states.as<float>();  // slot t = 1..m: (u, v) after t smoothing steps
  float* ubs[2] = {pl->vecA.as<float>(), pl->vecC.as<float>()};
  float* vbs[2] = {pl->vecB.as<float>(), pl->vecD.as<float>()};
  float* rK = pl->vecE.as<float>();
  float* uK = tg.fine2.as<float>();
  float* zero = tg.zero.as<float>();
  float* c0 = tg.c0.as<float>();
  float* c1 = tg.c1.as<float>();
  float* shat = tg.shat.as<float>();
  const Tile* grp = tg.d_groups.as<Tile>();
  double* partial = pl->partial.as<double>();
  double* r2b2 = pl->red.as<double>();
  double* acc_w = pl->acc.as<double>();
  double* acc_a = acc_w + (size_t)B * m;
  rmk::launch_fill_f32(zero, 0.f, P, st);
  rmk::launch_fill_f64(acc_w, 0.0, (int64_t)B * m * (1 + na), st);
  rmk::launch_fill_f32(d_symbol, 0.f, tg.Pc, st);
  int cur = 0;
  for (int k = K - 1; k >= 0; --k) {
    const float* u0 = ckpt + (int64_t)k * P;
    auto su = [&](int t) -> const float* { return t == 0 ? u0 : S + (int64_t)t * 2 * P; };
    auto sv = [&](int t) -> const float* { return t == 0 ? zero : S + (int64_t)t * 2 * P + P; };
    // recompute the m smoothing states of cycle k
    if (!blocked(pl)) {
      for (int t = 0; t < m; ++t) {
        float* uo = S + (int64_t)(t + 1) * 2 * P;
        one_step<float>(pl, p, method, omega, alpha, m, t, b, su(t), sv(t), uo, uo + P, nullptr, st);
      }
    } else {
      for (auto& cl : pl->classes) {
        for (int s0 = 0; s0 < m;) {
          const int t = std::min(cl.T, m - s0);
          float* uo = S + (int64_t)(s0 + t) * 2 * P;
          if (!launch_class(cl, t, method, p, omega, alpha, m, s0, b, su(s0), sv(s0), uo, uo + P, nullptr, nullptr,
                            st, S + (int64_t)(s0 + 1) * 2 * P, 2 * P))
            return fail(RM_EUNSUPPORTED, "block kernel configuration not built");
          s0 += t;
        }
      }
    }
    const float* uh = su(m);
    if (k == K - 1) {
      // u_K and the terminal adjoint
      twogrid_correct(pl, st, b, uh, uK, symbol);
      if (g_uK == nullptr) {
        rmk::launch_residual<float>(p, p.tiles, p.ntiles, b, uK, rK, partial, nullptr, st);
        rmk::launch_reduce_partials(p, partial, r2b2, r2b2 + 1, 2, nullptr, st);
        rmk::launch_adj_terminal(p, b, rK, r2b2, g_loss, ubs[cur], d_b, loss, st);
      } else {
        RM_HIP(hipMemcpyAsync(ubs[cur], g_uK, P * sizeof(float), hipMemcpyDeviceToDevice, st));
        if (d_b != nullptr) rmk::launch_fill_f32(d_b, 0.f, P, st);
      }
    }
    // sine coefficients of the restricted residual at the smoothed iterate
    rmk::launch_tg_restrict(0, p, g, tg.d_rtiles.as<Tile>(), tg.nrtiles, b, uh, c0, 1.f, st);
    rmk::launch_tg_dst(0, g, grp, tg.ngroups, tg.mmax, c0, c1, nullptr, nullptr, nullptr, nullptr, st);
    rmk::launch_tg_dst(1, g, grp, tg.ngroups, tg.mmax, c1, c1, nullptr, nullptr, shat, nullptr, st);
    // through the correction: c_bar = P^T ub = 4 R ub, symbol gradient, y_bar = C c_bar,
    // r_bar = R^T y_bar, f_bar += r_bar, ub_h = ub - A r_bar
    rmk::launch_tg_restrict(1, p, g, tg.d_rtiles.as<Tile>(), tg.nrtiles, nullptr, ubs[cur], c0, 4.f, st);
    rmk::launch_tg_dst(0, g, grp, tg.ngroups, tg.mmax, c0, c1, nullptr, nullptr, nullptr, nullptr, st);
    rmk::launch_tg_dst(1, g, grp, tg.ngroups, tg.mmax, c1, c1, symbol, shat, nullptr, d_symbol, st);
    rmk::launch_tg_dst(2, g, grp, tg.ngroups, tg.mmax, c1, c0, nullptr, nullptr, nullptr, nullptr, st);
    rmk::launch_tg_adj_correct(p, g, c0, ubs[cur], ubs[cur ^ 1], d_b, st);
    cur ^= 1;
    // through the smoothing, which starts from v = 0 (its adjoint is dropped)
    rmk::launch_fill_f32(vbs[cur], 0.f, P, st);
    const int* ranges = nullptr;
    RM_TRY(reverse_segment(pl, p, st, method, omega, alpha, m, 0, m, su, sv, b, ubs, vbs, cur, d_b, partial, nslot,
                           &ranges));
    rmk::launch_adj_accumulate(method, p, partial, nslot, m, 0, m, acc_w, acc_a, st, ranges);
  }
  rmk::launch_f64_to_f32(acc_w, d_omega, (int64_t)B * m, st);
  rmk::launch_f64_to_f32(acc_a, d_alpha, (int64_t)B * m * na, st);
  return last_launch();
}

rm_status rm_fgmres(rm_ctx* ctx, const rm_plan_t* plan, const rm_fgmres_opts* fo, int32_t method,
                    const rm_solve_opts* inner, const float* omega, const float* alpha, const float* symbol,
                    const double* b, double* x, rm_report* rep) {
  RM_TRY(check_ctx_plan(ctx, plan));
  if (fo == nullptr || b == nullptr || x == nullptr) return fail(RM_EINVAL, "null opts, b or x");
  const int R = fo->restart;
  if (R < 1 || R > 64) return fail(RM_EINVAL, "restart must be in 1..64");
  if (fo->max_iter < 1 || !(fo->tol > 0.0)) return fail(RM_EINVAL, "need max_iter >= 1 and tol > 0");
  rm_plan_t* pl = const_cast<rm_plan_t*>(plan);
  if (inner != nullptr) {
    RM_TRY(validate_weights(plan, method, inner, omega, alpha));
    if (inner->mode != RM_UNROLL || inner->dtype != RM_F32 || inner->K < 1)
      return fail(RM_EINVAL, "the preconditioner is an FP32 RM_UNROLL with K >= 1 (steps, or two-grid cycles)");
    if (symbol != nullptr) RM_TRY(twogrid_layout(pl));
    set_precond(pl, inner);
  } else if (symbol != nullptr) {
    return fail(RM_EINVAL, "a symbol needs inner options");
  }
  hipStream_t st = ctx->stream;
  const int B = pl->B;
  const int64_t P = pl->P;
  const int nslot = (int)pl->tiles.size();
  const size_t pd = (size_t)std::max<int64_t>(P, 1);
  auto& fg = pl->fg;
  RM_TRY(fg.V.ensure(pd * (R + 1) * sizeof(double), st));
  RM_TRY(fg.Z.ensure(pd * R * sizeof(float), st));
  RM_TRY(fg.w.ensure(pd * sizeof(double), st));
  RM_TRY(fg.t.ensure(pd * sizeof(double), st));
  RM_TRY(fg.b32.ensure(pd * sizeof(float), st));
  // doubles: H [B][R][R+1], cs, sn, y [B][R], g [B][R+1], hn2, relres, est [B], r2b2 [B][2]
  const size_t nH = (size_t)B * R * (R + 1), nR = (size_t)B * R, nG = (size_t)B * (R + 1);
  RM_TRY(fg.dbl.ensure((nH + 3 * nR + nG + 5 * (size_t)B) * sizeof(double), st));
  RM_TRY(fg.ints.ensure((size_t)5 * B * sizeof(int), st));
  RM_TRY(fg.partial.ensure((size_t)nslot * (R + 1) * sizeof(double), st));
  double* V = fg.V.as<double>();
  float* Z = fg.Z.as<float>();
  double* w = fg.w.as<double>();
  double* t64 = fg.t.as<double>();
  float* b32 = fg.b32.as<float>();
  double* H = fg.dbl.as<double>();
  double* cs = H + nH;
  double* sn = cs + nR;
  double* yv = sn + nR;
  double* g = yv + nR;
  double* hn2 = g + nG;
  double* relres = hn2 + B;
  double* est = relres + B;
  double* r2b2 = est + B;
  int* iters = fg.ints.as<int>();
  int* jdone = iters + B;
  int* active = jdone + B;
  int* running = active + B;
  int* status = running + B;
  double* partial = fg.partial.as<double>();
  const PlanDev p = pl->dev();
  rmk::launch_fill_i32(iters, 0, B, st);
  rmk::launch_fill_i32(running, 1, B, st);
  rmk::launch_fill_i32(status, RM_ENOTCONV, B, st);
  std::vector<int> h_active((size_t)B), h_round((size_t)B, 0);
  auto any_active = [&]() -> rm_status {
    RM_HIP(hipMemcpyAsync(h_active.data(), active, (size_t)B * sizeof(int), hipMemcpyDeviceToHost, st));
    RM_HIP(hipStreamSynchronize(st));
    return RM_OK;
  };
  auto count = [&]() {
    int c = 0;
    for (int v : h_active) c += v != 0;
    return c;
  };
  for (;;) {
    // true residual, convergence, v_0 = r / beta
    rmk::launch_residual<double>(p, p.tiles, p.ntiles, b, x, V, partial, nullptr, st);
    rmk::launch_reduce_partials(p, partial, r2b2, r2b2 + 1, 2, nullptr, st);
    rmk::launch_fgm_start(B, r2b2, fo->tol, fo->max_iter, iters, running, active, status, relres, g, R + 1, jdone,
                          st);
    rmk::launch_scale(p, V, r2b2, 2, V, active, st);
    RM_TRY(any_active());
    if (count() == 0) break;
    for (int b0 = 0; b0 < B; ++b0) h_round[b0] += h_active[b0] != 0;
    for (int j = 0; j < R; ++j) {
      double* Vj = V + (int64_t)j * P;
      float* Zj = Z + (int64_t)j * P;
      // z_j = M(v_j): the FP32 preconditioner applied to A z = fl32(v_j) from z = 0
      // (instances outside this cycle get a zero right-hand side, whatever Vj holds)
      rmk::launch_to_f32_masked(p, Vj, b32, active, st);
      if (inner == nullptr) {
        RM_HIP(hipMemcpyAsync(Zj, b32, P * sizeof(float), hipMemcpyDeviceToDevice, st));
      } else {
        rmk::launch_fill_f32(Zj, 0.f, P, st);
        if (symbol != nullptr)
          RM_TRY(twogrid_forward(ctx, pl, method, inner, omega, alpha, symbol, b32, Zj, nullptr, nullptr));
        else
          RM_TRY(solve_unroll<float>(ctx, pl, method, inner, omega, alpha, b32, Zj, nullptr, nullptr));
      }
      // w = A z_j in FP64, then two passes of classical Gram-Schmidt against v_0..v_j
      rmk::launch_f32_to_f64(Zj, t64, P, st);
      rmk::launch_apply<double>(p, p.tiles, p.ntiles, t64, w, st);
      double* Hj = H + (int64_t)j * (R + 1);
      const int ldh = R * (R + 1);
      rmk::launch_mdot(p, V, P, j + 1, w, active, partial, nslot, st);
      rmk::launch_mreduce(p, partial, j + 1, nslot, active, Hj, ldh, 0, false, st);
      rmk::launch_maxpy(p, V, P, j + 1, Hj, ldh, 0, w, active, st);
      rmk::launch_mdot(p, V, P, j + 1, w, active, partial, nslot, st);
      rmk::launch_mreduce(p, partial, j + 1, nslot, active, yv, R, 0, false, st);
      rmk::launch_maxpy(p, V, P, j + 1, yv, R, 0, w, active, st);
      rmk::launch_mreduce(p, partial, j + 1, nslot, active, Hj, ldh, 0, true, st);
      rmk::launch_mdot(p, w, P, 1, w, active, partial, nslot, st);
      rmk::launch_mreduce(p, partial, 1, nslot, active, hn2, 1, 0, false, st);
      rmk::launch_scale(p, w, hn2, 1, V + (int64_t)(j + 1) * P, active, st);
      rmk::launch_fgm_givens(B, j, R, H, hn2, cs, sn, g, r2b2, fo->tol, fo->max_iter, iters, jdone, active, est, st);
      RM_TRY(any_active());
      if (count() == 0) break;
    }
    rmk::launch_fgm_backsolve(B, R, H, g, jdone, yv, st);
    rmk::launch_fgm_xupdate(p, Z, P, yv, R, jdone, x, st);
  }
  RM_TRY(last_launch());
  std::vector<int> h_it((size_t)B), h_st((size_t)B);
  std::vector<double> h_rel((size_t)B);
  RM_HIP(hipMemcpy(h_it.data(), iters, (size_t)B * sizeof(int), hipMemcpyDeviceToHost));
  RM_HIP(hipMemcpy(h_st.data(), status, (size_t)B * sizeof(int), hipMemcpyDeviceToHost));
  RM_HIP(hipMemcpy(h_rel.data(), relres, (size_t)B * sizeof(double), hipMemcpyDeviceToHost));
  rm_status worst = RM_OK;
  for (int b0 = 0; b0 < B; ++b0) {
    if (rep != nullptr) {
      if (rep->outer_iters) rep->outer_iters[b0] = h_it[b0];
      if (rep->rounds) rep->rounds[b0] = h_round[b0];
      if (rep->relres) rep->relres[b0] = h_rel[b0];
      if (rep->status) rep->status[b0] = h_st[b0];
    }
    if (h_st[b0] == RM_EDIVERGED) worst = RM_EDIVERGED;
    else if (h_st[b0] == RM_ENOTCONV && worst == RM_OK) worst = RM_ENOTCONV;
  }
  if (worst != RM_OK) g_last_error = "some instances did not reach tol";
  return worst;
}

rm_status rm_plan_set_kernel(rm_plan_t* plan, int32_t n, int32_t shape, int32_t T, int32_t cw) {
  if (plan == nullptr) return fail(RM_EINVAL, "null plan");
  if (shape == -1) {
    plan->use_block = false;
    return RM_OK;
  }
  if (shape < 0 || shape >= kNumShapes) return fail(RM_EINVAL, "unknown kernel variant");
  if (T < 1 || T > 64) return fail(RM_EINVAL, "T must be in 1..64");
  bool hit = false;
  for (auto& c : plan->classes) {
    if (n > 0 && c.n != n) continue;
    int w = cw;
    if (w <= 0) {
      double best = 1e301;
      for (int cand : candidate_widths(c.n, shape, T)) {
        const double cost = model_cost(c.n, shape, T, cand, (int)c.insts.size());
        if (cost < best) {
          best = cost;
          w = cand;
        }
      }
    }
    int tx, ty;
    if (!class_geometry(c.n, shape, T, w, tx, ty))
      return fail(RM_EINVAL, "tile width / halo T + 1 does not fit this kernel variant");
    c.shape = shape;
    c.T = T;
    c.cw = w;
    set_default_tail(c);
    hit = true;
  }
  if (!hit) return fail(RM_EINVAL, "no instance of that size in the plan");
  plan->use_block = true;
  plan->exec_dirty = true;
  return RM_OK;
}

rm_status rm_plan_set_tail_kernel(rm_plan_t* plan, int32_t n, int32_t shape, int32_t T, int32_t cw) {
  if (plan == nullptr) return fail(RM_EINVAL, "null plan");
  if (shape < 0 || shape >= kNumShapes) return fail(RM_EINVAL, "unknown kernel variant");
  bool hit = false;
  for (auto& c : plan->classes) {
    if (n > 0 && c.n != n) continue;
    int w = cw;
    if (w <= 0) {
      double best = 1e301;
      for (int cand : candidate_widths(c.n, shape, T)) {
        const double cost = model_cost(c.n, shape, T, cand, (int)c.insts.size());
        if (cost < best) {
          best = cost;
          w = cand;
        }
      }
    }
    int tx, ty;
    if (!class_geometry(c.n, shape, T, w, tx, ty))
      return fail(RM_EINVAL, "tile width / halo T + 1 does not fit this kernel variant");
    c.tshape = shape;
    c.tT = T;
    c.tcw = w;
    hit = true;
  }
  if (!hit) return fail(RM_EINVAL, "no instance of that size in the plan");
  plan->exec_dirty = true;
  return RM_OK;
}

rm_status rm_plan_get_tail_kernel(const rm_plan_t* plan, int32_t n, int32_t* shape, int32_t* T, int32_t* cw) {
  if (plan == nullptr || shape == nullptr || T == nullptr || cw == nullptr) return fail(RM_EINVAL, "null argument");
  for (const auto& c : plan->classes)
    if (c.n == n) {
      *shape = c.tshape;
      *T = c.tT;
      *cw = c.tcw;
      return RM_OK;
    }
  return fail(RM_EINVAL, "no instance of that size in the plan");
}

rm_status rm_plan_set_mixed(rm_plan_t* plan, int32_t on) {
  if (plan == nullptr) return fail(RM_EINVAL, "null plan");
  if (plan->mixed != (on != 0)) {
    plan->mixed = on != 0;
    plan->exec_dirty = true;
  }
  return RM_OK;
}

rm_status rm_plan_get_mixed(const rm_plan_t* plan, int32_t* on) {
  if (plan == nullptr || on == nullptr) return fail(RM_EINVAL, "null plan or pointer");
  *on = plan->mixed ? 1 : 0;
  return RM_OK;
}

rm_status rm_plan_set_tail_switch(rm_plan_t* plan, double frac) {
  if (plan == nullptr) return fail(RM_EINVAL, "null plan");
  if (!(frac <= 1.0)) return fail(RM_EINVAL, "frac must be <= 1 (negative: automatic)");
  plan->tail_frac = frac;
  return RM_OK;
}

rm_status rm_plan_get_kernel(const rm_plan_t* plan, int32_t n, int32_t* shape, int32_t* T, int32_t* cw) {
  if (plan == nullptr || shape == nullptr || T == nullptr || cw == nullptr) return fail(RM_EINVAL, "null argument");
  if (!plan->use_block) {
    *shape = -1;
    *T = 1;
    *cw = 0;
    return RM_OK;
  }
  for (const auto& c : plan->classes)
    if (c.n == n) {
      *shape = c.shape;
      *T = c.T;
      *cw = c.cw;
      return RM_OK;
    }
  return fail(RM_EINVAL, "no instance of that size in the plan");
}

rm_status rm_tune(rm_ctx* ctx, rm_plan_t* plan, int32_t method, int32_t m, const float* omega, const float* alpha,
                  const float* b, const char* cache_path, double* us_per_step) {
  RM_TRY(check_ctx_plan(ctx, plan));
  if (method < RM_RICHARDSON || method > RM_NAGEX) return fail(RM_EINVAL, "unknown method");
  if (m < 1 || m > kMaxM) return fail(RM_EINVAL, "m must be in 1..64");
  if (omega == nullptr || b == nullptr || (method != RM_RICHARDSON && alpha == nullptr))
    return fail(RM_EINVAL, "null omega, alpha or b");
  plan->jacobi = 0;
  plan->ssor = 0;
  hipStream_t st = ctx->stream;
  hipDeviceProp_t prop;
  RM_HIP(hipGetDeviceProperties(&prop, ctx->device));
  char arch[64];
  std::snprintf(arch, sizeof arch, "%s", prop.gcnArchName);
  for (char* q = arch; *q; ++q)
    if (*q == ':') *q = 0;
  // cached choices
  std::vector<std::pair<std::string, std::string>> cache;
  if (cache_path != nullptr) {
    if (FILE* fh = std::fopen(cache_path, "r")) {
      char line[512];
      while (std::fgets(line, sizeof line, fh)) {
        char key[300], val[200];
        if (std::sscanf(line, " \"%299[^\"]\": %199[^]]", key, val) == 2) cache.emplace_back(key, std::string(val) + "]");
      }
      std::fclose(fh);
    }
  }
  const size_t fb = vec_bytes<float>(plan);
  RM_TRY(plan->vecA.ensure(fb, st));
  RM_TRY(plan->vecB.ensure(fb, st));
  RM_TRY(plan->vecC.ensure(fb, st));
  RM_TRY(plan->vecD.ensure(fb, st));
  float* us_[2] = {plan->vecA.as<float>(), plan->vecB.as<float>()};
  float* vs_[2] = {plan->vecC.as<float>(), plan->vecD.as<float>()};
  for (int k = 0; k < 2; ++k) {
    rmk::launch_fill_f32(us_[k], 0.f, plan->P, st);
    rmk::launch_fill_f32(vs_[k], 0.f, plan->P, st);
  }
  plan->use_block = true;
  hipEvent_t e0, e1;
  RM_HIP(hipEventCreate(&e0));
  RM_HIP(hipEventCreate(&e1));
  double total_us = 0.0;
  const int steps = 16, reps = 3;
  for (size_t ci = 0; ci < plan->classes.size(); ++ci) {
    auto& c = plan->classes[ci];
    const std::string key = tune_key(arch, c, m, method);
    bool found = false;
    for (auto& kv : cache)
      if (kv.first == key) {
        int sh, T, w, tsh, tT, tw;
        double us, tus, fus;
        const int got = std::sscanf(kv.second.c_str(), "[%d, %d, %d, %lf, %d, %d, %d, %lf, %lf]", &sh, &T, &w, &us,
                                    &tsh, &tT, &tw, &tus, &fus);
        int tx, ty;
        if (got >= 4 && class_geometry(c.n, sh, T, w, tx, ty)) {
          c.shape = sh;
          c.T = T;
          c.cw = w;
          set_default_tail(c);
          c.us = us;
          if (got == 9 && class_geometry(c.n, tsh, tT, tw, tx, ty)) {
            c.tshape = tsh;
            c.tT = tT;
            c.tcw = tw;
            c.tus = tus;
            c.floor_us = fus;
          }
          total_us += us;
          found = true;
        }
      }
    if (found) continue;
    // time 16 steps of the class (best of `reps` after one warm-up), with all of its
    // instances active or only those marked in `mask`
    auto time_class = [&](const int* mask, double& t_best) -> rm_status {
      plan->exec_dirty = true;
      t_best = 1e300;
      for (int r = 0; r < reps + 1; ++r) {
        int cur = 0, flips = 0;
        RM_HIP(hipEventRecord(e0, st));
        RM_TRY(sweep(plan, st, method, m, 0, steps, omega, alpha, b, us_, vs_, cur, flips, mask, nullptr, nullptr,
                     (int)ci));
        RM_HIP(hipEventRecord(e1, st));
        RM_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        RM_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (r > 0) t_best = std::min(t_best, (double)ms * 1e3 / steps);
      }
      return RM_OK;
    };
    double best = 1e300, tbest = 1e300;
    int best_s = c.shape, best_T = c.T, best_w = c.cw, tbest_s = c.tshape, tbest_T = c.tT, tbest_w = c.tcw;
    for (int sh = 0; sh < kNumShapes; ++sh)
      for (int T : kTs)
        for (int w : candidate_widths(c.n, sh, T)) {
          c.shape = sh;
          c.T = T;
          c.cw = w;
          double t_best;
          RM_TRY(time_class(nullptr, t_best));
          if (t_best < best) {
            best = t_best;
            best_s = sh;
            best_T = T;
            best_w = w;
          }
          if (sh != kStreamShape && t_best < tbest) {
            tbest = t_best;
            tbest_s = sh;
            tbest_T = T;
            tbest_w = w;
          }
        }
    c.shape = best_s;
    c.T = best_T;
    c.cw = best_w;
    c.us = best;
    c.tshape = tbest_s;
    c.tT = tbest_T;
    c.tcw = tbest_w;
    c.tus = tbest;
    c.floor_us = 0.0;
    if (best_s == kStreamShape && !c.insts.empty()) {
      // the main configuration with a single instance of the class active
      RM_TRY(plan->flags.ensure(((size_t)plan->B * 6 + 16) * sizeof(int), st));
      int* one = plan->flags.as<int>();
      rmk::launch_fill_i32(one, 0, plan->B, st);
      const int on = 1;
      RM_HIP(hipMemcpyAsync(one + c.insts[0], &on, sizeof(int), hipMemcpyHostToDevice, st));
      RM_TRY(time_class(one, c.floor_us));
    }
    total_us += best;
    char val[200];
    std::snprintf(val, sizeof val, "[%d, %d, %d, %.3f, %d, %d, %d, %.3f, %.3f]", best_s, best_T, best_w, best, tbest_s,
                  tbest_T, tbest_w, tbest, c.floor_us);
    cache.emplace_back(key, val);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  plan->exec_dirty = true;
  RM_TRY(build_exec(plan, st));
  if (cache_path != nullptr) {
    if (FILE* fh = std::fopen(cache_path, "w")) {
      std::fprintf(fh, "{\n");
      for (size_t k = 0; k < cache.size(); ++k)
        std::fprintf(fh, "  \"%s\": %s%s\n", cache[k].first.c_str(), cache[k].second.c_str(),
                     k + 1 < cache.size() ? "," : "");
      std::fprintf(fh, "}\n");
      std::fclose(fh);
    }
  }
  if (us_per_step != nullptr) *us_per_step = total_us;
  return last_launch();
}

int32_t rm_meta_param_count(int32_t m) {
  const int H = 64;
  return H * 2 + H + H * H + H + (m + 1) * H + (m + 1);
}

rm_status rm_meta_forward(rm_ctx* ctx, const rm_plan_t* plan, int32_t m, const float* params, float* omega,
                          float* alpha) {
  RM_TRY(check_ctx_plan(ctx, plan));
  if (m < 1 || m > kMaxM) return fail(RM_EINVAL, "m must be in 1..64");
  if (params == nullptr || omega == nullptr || alpha == nullptr) return fail(RM_EINVAL, "null pointer");
  rmk::launch_meta_forward(plan->dev(), m, params, omega, alpha, ctx->stream);
  return last_launch();
}

rm_status rm_meta_backward(rm_ctx* ctx, const rm_plan_t* plan, int32_t m, const float* params,
                           const float* d_omega, const float* d_alpha, float* d_params) {
  RM_TRY(check_ctx_plan(ctx, plan));
  if (m < 1 || m > kMaxM) return fail(RM_EINVAL, "m must be in 1..64");
  if (params == nullptr || d_omega == nullptr || d_alpha == nullptr || d_params == nullptr)
    return fail(RM_EINVAL, "null pointer");
  rm_plan_t* pl = const_cast<rm_plan_t*>(plan);
  RM_TRY(pl->meta.ensure((size_t)pl->B * rm_meta_param_count(m) * sizeof(float), ctx->stream));
  rmk::launch_meta_backward(pl->dev(), m, params, d_omega, d_alpha, pl->meta.as<float>(), d_params, ctx->stream);
  return last_launch();
}

}  // extern "C"
