// Row-streaming temporal-blocked steps for gfx950: the kernel that runs one row window
// per workgroup and its launcher (the forward pipeline itself is in rm_stream_run.h),
// and the reverse steps of the adjoint in the same row-pipeline form.
#include <type_traits>

#include "rm_stream_run.h"

#pragma clang fp contract(off)

namespace rmk {

namespace {

// Iterations per unrolled loop body of the reverse pipeline: a multiple of its
// register rings' lengths (3 rows of published values, 2 rows of queued inputs) and
// of the prefetch depth.
constexpr int kUnroll = 6;

// One row window per workgroup (64 ceil(n / 64) threads); windows of inactive
// instances return at once.
template <int TL, int METHOD, bool STORE, bool RES, int MAXT, int PF>
__global__ __attribute__((amdgpu_flat_work_group_size(64, MAXT))) void k_stream(
    PlanDev p, const BTile* __restrict__ tiles, int ntiles, int wlen, const float* __restrict__ omega,
    const float* __restrict__ alpha, int m, int s0, const float* __restrict__ f, const float* __restrict__ u,
    const float* __restrict__ v, float* __restrict__ u_out, float* __restrict__ v_out,
    const int* __restrict__ active, double* __restrict__ partial2, float* __restrict__ states,
    int64_t state_stride) {
  extern __shared__ float lds[];
  __shared__ double sh[MAXT / 64];
  const BTile tl = tiles[xcd_remap(blockIdx.x, ntiles)];
  if (tl.inst < 0) return;
  if (active != nullptr && active[tl.inst] == 0) return;
  const int n = p.inst[tl.inst].n;
  stream_run<TL, METHOD, STORE, RES, MAXT, PF>(p, tl, min(n, tl.y0 + wlen) - tl.y0, true, (int)blockDim.x,
                                               (int)threadIdx.x, lds, sh, omega, alpha, m, s0, f, u, v, u_out,
                                               v_out, partial2, states, state_stride);
}

// PFP: prefetch depth of the plain sweep; PFR: of the launches that also form the residual
// or store the states (more registers).
template <int TL, int MAXT, int PFP, int PFR>
bool launch_stream_tl(int nw, int wlen, int method, const PlanDev& p, const BTile* tiles, int ntiles,
                      const float* omega, const float* alpha, int m, int s0, const float* f, const float* u,
                      const float* v, float* u_out, float* v_out, const int* active, double* partial2,
                      float* states, int64_t state_stride, hipStream_t st) {
  const dim3 grid(ntiles), block(64 * nw);
  const size_t lds = (size_t)(64 * nw + 5) * (2 * (TL + 1) + 1) * sizeof(float);
#define RM_LAUNCH(MM, SS, RR, PF)                                                                                   \
  hipLaunchKernelGGL((k_stream<TL, MM, SS, RR, MAXT, PF>), grid, block, lds, st, p, tiles, ntiles, wlen, omega,   \
                     alpha, m, s0, f, u, v, u_out, v_out, active, partial2, states, state_stride)
#define RM_METHOD(MM)                          \
  if (states != nullptr) RM_LAUNCH(MM, true, false, PFR);  \
  else if (partial2 != nullptr) RM_LAUNCH(MM, false, true, PFR); \
  else RM_LAUNCH(MM, false, false, PFP);
  // the forward recompute that stores every state never asks for the residual
  if (states != nullptr && partial2 != nullptr) return false;
  switch (method) {
    case M_NAG: RM_METHOD(M_NAG) break;
    case M_MOM: RM_METHOD(M_MOM) break;
    case M_NAGEX: RM_METHOD(M_NAGEX) break;
    default: RM_METHOD(M_RICH) break;
  }
  return true;
#undef RM_METHOD
#undef RM_LAUNCH
}


// ---------------------------------------------------------------------------
// Reverse steps (adjoint of a Table-1 unroll) in the same row pipeline.
//
// The reverse of one step is linear in the adjoints (ub, vb) of (u', v'):
//   g = vb + ub,  utb = -w A g,  ub <- ub + utb,  vb <- a g + at utb (per scheme),
//   fb <- fb + w g,
// with the weight gradients <g, r>, <g, v> and <utb, v>, where r = f - A u~ and v are
// the forward state before the step.  Level l = 1..TL takes the l-th step of the
// launch in reverse order: at iteration s it reverses row s - 2l from the g rows
// published by level l - 1 (the loader for l = 1) and from its own forward state,
// which it reads from memory and publishes one row ahead (u~ = u + at v of row
// s - 2l + 2), so that both stencils have their three rows in registers.  ub, vb, f and
// fb travel down the levels in registers; global memory sees the stored forward state
// of every step plus one read and one write of (ub, vb, fb) per launch.  The same
// operations in the same order as the one-step reverse, so ub, vb and fb agree with it
// bit for bit; the dot products are summed over the owned points of each window.
// ---------------------------------------------------------------------------
template <int TL>
struct AdjRegs {
  float gc[TL + 1][3], gm[TL + 1][3], gp[TL + 1][3];  // g published for level l: own, west, east
  float sc[TL + 1][3], sm[TL + 1][3], sp[TL + 1][3];  // u~ of level l's forward state: own, west, east
  float sv[TL + 1][3];                                // v of level l's forward state (own column)
  float qu[TL + 1][2], qv[TL + 1][2], qf[TL + 1][2], qb[TL + 1][2];  // ub, vb, f, fb for level l
  float su[TL + 1][3], svp[TL + 1][3];                // prefetched forward state rows of level l
  float lu[kUnroll], lv[kUnroll], lf[kUnroll], lb[kUnroll];          // prefetched loader rows
};

template <int TL, int METHOD>
__global__ __attribute__((amdgpu_flat_work_group_size(64, 512))) void k_adj_stream(
    PlanDev p, const BTile* __restrict__ tiles, int ntiles, int wlen, const float* __restrict__ omega,
    const float* __restrict__ alpha, int m, AdjLevels lev, const float* __restrict__ f,
    const float* __restrict__ ub, const float* __restrict__ vb, float* __restrict__ ub_out,
    float* __restrict__ vb_out, float* __restrict__ fb) {
  // LDS per column: two row slots per level for g, then two per level for u~ (odd stride)
  constexpr int LS = 4 * TL + 1;
  constexpr int GO = 0, SO = 2 * TL;
  extern __shared__ float lds[];
  __shared__ double sh[3 * kAdjMaxT][8];
  const BTile tl = tiles[xcd_remap(blockIdx.x, ntiles)];
  if (tl.inst < 0) return;
  const Inst in = p.inst[tl.inst];
  const int n = in.n;
  const int NT = blockDim.x;
  const int gx = threadIdx.x;
  const bool colin = gx < n;
  const int gxc = colin ? gx : n - 1;
  const int ys = tl.y0;
  const int L = min(n, ys + wlen) - ys;
  const int own0 = tl.oy0 - ys, own1 = tl.oy1 - ys;
  float c[5];
  load_coef<float>(p, tl.inst, c);
  float fw[TL + 1], fa[TL + 1], fat[TL + 1];
  static_for<1, TL + 1>([&](auto T_) {
    constexpr int l = decltype(T_)::value;
    step_factors<float, METHOD>(p, omega, alpha, m, tl.inst, lev.i[l - 1], fw[l], fa[l], fat[l]);
  });
  for (int e = threadIdx.x; e < (NT + 2) * LS; e += NT) lds[e] = 0.0f;
  float* lbase = lds + gx * LS;  // column gx - 1; own column at + LS, east at + 2 LS
  const int64_t off = in.off;
  const int nn4 = n * n * (int)sizeof(float);
  const bool has_fb = fb != nullptr;
  const __amdgpu_buffer_rsrc_t fb_rs =
      __builtin_amdgcn_make_buffer_rsrc(has_fb ? fb + off : ub_out + off, (short)0, nn4, kBufWord3);
  const __amdgpu_buffer_rsrc_t ub_rs = __builtin_amdgcn_make_buffer_rsrc(ub_out + off, (short)0, nn4, kBufWord3);
  const __amdgpu_buffer_rsrc_t vb_rs = __builtin_amdgcn_make_buffer_rsrc(vb_out + off, (short)0, nn4, kBufWord3);
  AdjRegs<TL> R;
  static_for<0, TL + 1>([&](auto T_) {
    constexpr int l = decltype(T_)::value;
#pragma unroll
    for (int k = 0; k < 3; ++k)
      R.gc[l][k] = R.gm[l][k] = R.gp[l][k] = R.sc[l][k] = R.sm[l][k] = R.sp[l][k] = R.sv[l][k] = 0.0f;
#pragma unroll
    for (int k = 0; k < 2; ++k) R.qu[l][k] = R.qv[l][k] = R.qf[l][k] = R.qb[l][k] = 0.0f;
  });
  // loader rows (ub, vb, f, fb) and forward state rows, clamped into the window
  auto own_row = [&](int r) { return r >= own0 && r < own1 && colin; };
  auto load_top = [&](int r, float& a, float& b2, float& ff, float& bb) {
    const int rc = min(max(r, 0), L - 1);
    const int idx = (ys + rc) * n + gxc;
    a = ub[off + idx];
    b2 = uses_momentum(METHOD) ? vb[off + idx] : 0.0f;
    ff = f[off + idx];
    // fb only on owned points: another window updates the rest in place meanwhile
    const int bo = has_fb && own_row(r) ? ((ys + r) * n + gx) * (int)sizeof(float) : kDropOffset;
    bb = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(fb_rs, bo, 0, 0));
  };
  auto load_state = [&](int l, int r, float& uu, float& vv) {
    const int rc = min(max(r, 0), L - 1);
    const int64_t idx = off + (int64_t)(ys + rc) * n + gxc;
    uu = lev.u[l - 1][idx];
    vv = uses_momentum(METHOD) ? lev.v[l - 1][idx] : 0.0f;
  };
  static_for<0, kUnroll>([&](auto K_) {
    constexpr int k = decltype(K_)::value;
    load_top(k, R.lu[k], R.lv[k], R.lf[k], R.lb[k]);
  });
  // level l publishes state row s - 2 l + 2 at iteration s from prefetch slot s mod 3
  static_for<1, TL + 1>([&](auto T_) {
    constexpr int l = decltype(T_)::value;
#pragma unroll
    for (int k = 0; k < 3; ++k) load_state(l, k - 2 * l + 2, R.su[l][k], R.svp[l][k]);
  });
  double acc[TL + 1][3];
  static_for<0, TL + 1>([&](auto T_) {
    constexpr int l = decltype(T_)::value;
    acc[l][0] = acc[l][1] = acc[l][2] = 0.0;
  });
  __syncthreads();
  const int S = L + 2 * TL;
  auto iter = [&](auto PH_, int s) {
    constexpr int PH = decltype(PH_)::value;
    constexpr int q = pmod(PH + 1, 2);  // LDS slot of the rows published in the previous iteration
    // neighbours of the newest rows (row s - 2 l + 1 of g and of u~)
    static_for<1, TL + 1>([&](auto T_) {
      constexpr int l = decltype(T_)::value;
      constexpr int r3 = pmod(PH - 2 * l + 1, 3);
      R.gm[l][r3] = lbase[GO + (l - 1) * 2 + q];
      R.gp[l][r3] = lbase[2 * LS + GO + (l - 1) * 2 + q];
      R.sm[l][r3] = lbase[SO + (l - 1) * 2 + q];
      R.sp[l][r3] = lbase[2 * LS + SO + (l - 1) * 2 + q];
    });
    static_for<0, TL>([&](auto K_) {
      constexpr int l = TL - decltype(K_)::value;
      constexpr int y3 = pmod(PH - 2 * l, 3), ym3 = pmod(PH - 2 * l - 1, 3), yp3 = pmod(PH - 2 * l + 1, 3);
      constexpr int y2 = pmod(PH, 2);
      const int y = s - 2 * l;
      const bool rowok = (unsigned)y < (unsigned)L;
      const bool mine = own_row(y);
      // reverse of the step at row y
      const float g = R.gc[l][y3];
      const float ag = stencil9<float>(c, R.gc[l][y3], R.gm[l][y3], R.gp[l][y3], R.gc[l][ym3], R.gc[l][yp3],
                                       R.gm[l][ym3], R.gp[l][yp3], R.gp[l][ym3], R.gm[l][yp3]);
      const float utb = -(fw[l] * ag);
      const float r = R.qf[l][y2] - stencil9<float>(c, R.sc[l][y3], R.sm[l][y3], R.sp[l][y3], R.sc[l][ym3],
                                                    R.sc[l][yp3], R.sm[l][ym3], R.sp[l][yp3], R.sp[l][ym3],
                                                    R.sm[l][yp3]);
      const float rv = R.sv[l][y3];
      const double dg = (double)g, dv = (double)rv;
      acc[l][0] += mine ? dg * (double)r : 0.0;
      acc[l][1] += mine ? dg * dv : 0.0;
      acc[l][2] += mine ? (double)utb * dv : 0.0;
      const float nub = R.qu[l][y2] + utb;
      float nvb = 0.0f;
      if (METHOD == M_NAG) nvb = fa[l] * (g + utb);
      if (METHOD == M_MOM) nvb = fa[l] * g;
      if (METHOD == M_NAGEX) nvb = fmadd(fat[l], utb, fa[l] * g);
      const float nfb = fmadd(fw[l], g, R.qb[l][y2]);
      if constexpr (l < TL) {
        const float gn = uses_momentum(METHOD) ? nvb + nub : nub;
        const float pub = rowok && colin ? gn : 0.0f;
        R.gc[l + 1][y3] = pub;
        lbase[LS + GO + l * 2 + y2] = pub;
        R.qu[l + 1][y2] = nub;
        R.qv[l + 1][y2] = nvb;
        R.qf[l + 1][y2] = R.qf[l][y2];
        R.qb[l + 1][y2] = nfb;
      } else {
        const int boff = mine ? ((ys + y) * n + gx) * (int)sizeof(float) : kDropOffset;
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(nub), ub_rs, boff, 0, 0);
        if (uses_momentum(METHOD)) __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(nvb), vb_rs, boff, 0, 0);
        if (has_fb) __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(nfb), fb_rs, boff, 0, 0);
      }
      // forward state of row y + 2 for the next iterations (after the reads of row y - 1)
      {
        constexpr int s3 = pmod(PH, 3);
        const int rq = y + 2;
        const float uu = R.su[l][s3], vv = fresh(R.svp[l][s3]);
        const float x = uses_lookahead(METHOD) ? fmadd(fat[l], vv, uu) : uu;
        const float pub = (unsigned)rq < (unsigned)L && colin ? x : 0.0f;
        R.sc[l][pmod(PH - 2 * l + 2, 3)] = pub;
        R.sv[l][pmod(PH - 2 * l + 2, 3)] = vv;
        lbase[LS + SO + (l - 1) * 2 + y2] = pub;
        load_state(l, rq + 3, R.su[l][s3], R.svp[l][s3]);
      }
    });
    // loader: row s enters level 1
    {
      constexpr int y3 = pmod(PH, 3), y2 = pmod(PH, 2);
      const bool rowok = (unsigned)s < (unsigned)L;
      const float a = fresh(R.lu[PH]), b2 = fresh(R.lv[PH]), ff = fresh(R.lf[PH]), bb = fresh(R.lb[PH]);
      const float gn = uses_momentum(METHOD) ? b2 + a : a;
      const float pub = rowok && colin ? gn : 0.0f;
      R.gc[1][y3] = pub;
      lbase[LS + GO + y2] = pub;
      R.qu[1][y2] = a;
      R.qv[1][y2] = b2;
      R.qf[1][y2] = ff;
      R.qb[1][y2] = bb;
      load_top(s + kUnroll, R.lu[PH], R.lv[PH], R.lf[PH], R.lb[PH]);
    }
    __syncthreads();
  };
#pragma unroll 1
  for (int s = 0; s < S; s += kUnroll) {
    static_for<0, kUnroll>([&](auto PH_) { iter(PH_, s + decltype(PH_)::value); });
  }
  // per level, the three dot products summed over the workgroup in a fixed order
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  static_for<1, TL + 1>([&](auto T_) {
    constexpr int l = decltype(T_)::value;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double x = wave_sum(acc[l][k]);
      if (lane == 0) sh[3 * (l - 1) + k][w] = x;
    }
  });
  __syncthreads();
  if (threadIdx.x < 3 * TL) {
    double sum = 0.0;
    for (int k = 0; k < NT / 64; ++k) sum += sh[threadIdx.x][k];
    const int l = threadIdx.x / 3, k = threadIdx.x % 3;
    double* dst = lev.part[l] + 4 * tl.slot;
    dst[k] = sum;
    if (k == 2) dst[3] = 0.0;
  }
}

template <int TL>
void launch_adj_stream_tl(int nw, int wlen, int method, const PlanDev& p, const BTile* tiles, int ntiles,
                          const float* omega, const float* alpha, int m, const AdjLevels& lev, const float* f,
                          const float* ub, const float* vb, float* ub_out, float* vb_out, float* fb, hipStream_t st) {
  const dim3 grid(ntiles), block(64 * nw);
  const size_t lds = (size_t)(64 * nw + 2) * (4 * TL + 1) * sizeof(float);
#define RM_ADJS(MM)                                                                                               \
  hipLaunchKernelGGL((k_adj_stream<TL, MM>), grid, block, lds, st, p, tiles, ntiles, wlen, omega, alpha, m, lev, \
                     f, ub, vb, ub_out, vb_out, fb)
  switch (method) {
    case M_NAG: RM_ADJS(M_NAG); break;
    case M_MOM: RM_ADJS(M_MOM); break;
    case M_NAGEX: RM_ADJS(M_NAGEX); break;
    default: RM_ADJS(M_RICH); break;
  }
#undef RM_ADJS
}

}  // namespace

bool launch_stream(int T, int wlen, int n, int method, const PlanDev& p, const BTile* tiles, int ntiles,
                   const float* omega, const float* alpha, int m, int s0, const float* f, const float* u,
                   const float* v, float* u_out, float* v_out, const int* active, double* partial2,
                   hipStream_t st, float* states, int64_t state_stride) {
  if (n < 1 || n > kStreamMaxN || wlen < 1 || T < 1 || T > kStreamMaxT) return false;
  const int nw = (n + 63) / 64;
#define RM_T_CASE(TT)                                                                                              \
  case TT:                                                                                                         \
    return nw > 8 ? launch_stream_tl<TT, 1024, 4, 2>(nw, wlen, method, p, tiles, ntiles, omega, alpha, m, s0, f, u, \
                                                     v, u_out, v_out, active, partial2, states, state_stride, st)     \
                  : launch_stream_tl<TT, 512, 4, 4>(nw, wlen, method, p, tiles, ntiles, omega, alpha, m, s0, f, u, v,  \
                                                    u_out, v_out, active, partial2, states, state_stride, st);
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
}

bool launch_adj_stream(int T, int wlen, int n, int method, const PlanDev& p, const BTile* tiles, int ntiles,
                       const float* omega, const float* alpha, int m, const AdjLevels& lev, const float* f,
                       const float* ub, const float* vb, float* ub_out, float* vb_out, float* fb, hipStream_t st) {
  if (n < 1 || n > kAdjStreamMaxN || wlen < 1 || T < 1 || T > kAdjMaxT) return false;
  const int nw = (n + 63) / 64;
  // three levels need 253 registers; a fourth would spill
  switch (T) {
    case 1: launch_adj_stream_tl<1>(nw, wlen, method, p, tiles, ntiles, omega, alpha, m, lev, f, ub, vb, ub_out,
                                    vb_out, fb, st); return true;
    case 2: launch_adj_stream_tl<2>(nw, wlen, method, p, tiles, ntiles, omega, alpha, m, lev, f, ub, vb, ub_out,
                                    vb_out, fb, st); return true;
    case 3: launch_adj_stream_tl<3>(nw, wlen, method, p, tiles, ntiles, omega, alpha, m, lev, f, ub, vb, ub_out,
                                    vb_out, fb, st); return true;
    default: return false;
  }
}

}  // namespace rmk
