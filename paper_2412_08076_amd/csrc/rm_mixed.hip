// The mixed-size launch of the forward row pipeline: one launch advances every size
// class that runs the row pipeline, each workgroup taking a group of equally high row
// windows of one class (see rmgeo::make_groups).
#include "rm_stream_run.h"

namespace rmk {

namespace {

// The mixed-size launch: workgroup k takes group groups[k] (after the XCD remap), whose
// windows share a size class and a height; sub-group j (threads j nt .. (j + 1) nt - 1)
// runs window first + j with its own LDS block.  A group of a class whose bit is set
// in leave_out, or whose windows all belong to inactive instances, returns at once
// (the decision is the same for the whole workgroup); otherwise every sub-group runs
// the window's iterations, those without a live window masked.
template <int TL, int METHOD, bool RES>
__global__ __attribute__((amdgpu_flat_work_group_size(kMixedThreads, kMixedThreads))) void k_stream_mixed(
    PlanDev p, const BTile* __restrict__ tiles, const MGroup* __restrict__ groups, int ngroups,
    unsigned long long leave_out, const float* __restrict__ omega, const float* __restrict__ alpha, int m, int s0,
    const float* __restrict__ f, const float* __restrict__ u, const float* __restrict__ v, float* __restrict__ u_out,
    float* __restrict__ v_out, const int* __restrict__ active, double* __restrict__ partial2) {
  extern __shared__ float lds[];
  __shared__ double sh[kMixedThreads / 64];
  const MGroup g = groups[xcd_remap(blockIdx.x, ngroups)];
  if (g.cls < 0 || (g.cls < 64 && ((leave_out >> g.cls) & 1ull) != 0)) return;
  bool any = false;
  for (int j = 0; j < g.count; ++j) any = any || active == nullptr || active[tiles[g.first + j].inst] != 0;
  if (!any) return;
  // G sub-groups of nt threads, and when nt does not divide the workgroup the rest as
  // one narrower sub-group without a window.  A sub-group is whole waves: its index is
  // the same across a wave, so a scalar, and so are its tile, instance, coefficients
  // and step factors.  LDS: block j at j (nt + 5) columns; the last block ends at
  // column G (nt + 5) + (rest + 5) = 1024 + 5 (G + 1) <= 1104 (G = 16 only for nt = 64,
  // which leaves no rest).
  const int G = kMixedThreads / g.nt;
  const int sg = __builtin_amdgcn_readfirstlane(min((int)threadIdx.x / g.nt, G));
  const int NTs = sg < G ? g.nt : kMixedThreads - G * g.nt;
  const int tid = (int)threadIdx.x - sg * g.nt;
  const bool has = sg < g.count;
  const BTile tl = tiles[g.first + (has ? sg : 0)];
  const bool live = has && (active == nullptr || active[tl.inst] != 0);
  constexpr int LS = 2 * (TL + 1) + 1;
  stream_run<TL, METHOD, false, RES, kMixedThreads, 2>(p, tl, g.L, live, NTs, tid, lds + sg * (g.nt + 5) * LS,
                                                       sh + sg * (g.nt / 64), omega, alpha, m, s0, f, u, v, u_out,
                                                       v_out, partial2, nullptr, 0);
}

}  // namespace

bool launch_stream_mixed(int T, int method, const PlanDev& p, const BTile* tiles, const MGroup* groups, int ngroups,
                         unsigned long long leave_out, const float* omega, const float* alpha, int m, int s0,
                         const float* f, const float* u, const float* v, float* u_out, float* v_out,
                         const int* active, double* partial2, hipStream_t st) {
  if (T < 1 || T > kStreamMaxT || ngroups < 1) return false;
  // at most 1024 + 5 * 16 columns of LDS blocks (16 sub-groups of 64 threads)
  const size_t lds = (size_t)(kMixedThreads + 5 * (kMixedThreads / 64)) * (2 * (T + 1) + 1) * sizeof(float);
#define RM_LAUNCH(TT, MM, RR)                                                                                      \
  hipLaunchKernelGGL((k_stream_mixed<TT, MM, RR>), dim3(ngroups), dim3(kMixedThreads), lds, st, p, tiles, groups, \
                     ngroups, leave_out, omega, alpha, m, s0, f, u, v, u_out, v_out, active, partial2)
#define RM_METHOD(TT, MM)                         \
  if (partial2 != nullptr) RM_LAUNCH(TT, MM, true); \
  else RM_LAUNCH(TT, MM, false);
#define RM_T_CASE(TT)                           \
  case TT:                                      \
    switch (method) {                           \
      case M_NAG: RM_METHOD(TT, M_NAG) break;     \
      case M_MOM: RM_METHOD(TT, M_MOM) break;     \
      case M_NAGEX: RM_METHOD(TT, M_NAGEX) break; \
      default: RM_METHOD(TT, M_RICH) break;       \
    }                                           \
    return true;
  switch (T) {
    RM_T_CASE(1)
    RM_T_CASE(2)
    RM_T_CASE(3)
    RM_T_CASE(4)
    RM_T_CASE(5)
    RM_T_CASE(6)
    RM_T_CASE(7)
    RM_T_CASE(8)
    default:
      return false;
  }
#undef RM_T_CASE
#undef RM_METHOD
#undef RM_LAUNCH
}

}  // namespace rmk
