// Row-streaming temporal-blocked steps for gfx950: the forward pipeline of one row
// window, shared by the one-window-per-workgroup kernel and the mixed-size launch.
//
// One workgroup of 64 ceil(n / 64) threads (up to 1024) holds whole grid rows of one
// instance (thread = column), so no column halo is needed, and streams down a window
// of rows (the whole height, or one of several overlapping row windows when the batch
// alone does not fill the chip).  The TL inner steps of a launch of a Table-1 scheme
// (Richardson(m), MOM-, NAG- or NAGex-Richardson(m), optionally Jacobi-preconditioned)
// run as a pipeline over the rows: at iteration s the loader brings in row s, and
// step t (1..TL) receives row s - 2t + 1 of what step t - 1 produced in the iteration
// before and completes row s - 2t.  Since no step needs a row produced in the same
// iteration, the TL updates of an iteration are independent and one barrier per
// iteration suffices.
//
// Each step accumulates the stencil of a row as its three input rows arrive: the row
// below (the south row, y - 1) starts the sum, the row itself adds the centre row and
// the row above (y + 1) completes it.  A step therefore keeps only two partial sums
// (rows y + 1 and y + 2) and the (u, v, f) of the two rows it is about to update in
// registers, nine values per column, and the neighbour columns of an arriving row are
// read from LDS once and used at once.  A step publishes each row it produces to LDS
// once (two row slots per step).  Global memory sees one read of (u, v, f) and one
// write of (u, v) per point and launch.
//
// The sum is formed in the order of step_vf (south row, centre row, north row, then
// the weight and the momentum), the order every FP32 sweep kernel uses, so a launch of
// TL steps reproduces TL one-step launches bit for bit.  Rows outside the window
// publish zeros: at the domain edge that is the Dirichlet condition; at a cut between
// windows the error moves inward one row per step, so windows overlap by a halo
// h >= TL (h >= TL + 1 with the residual) and each stores only its owned rows.  With
// partial2 given, ||f - A u||^2 of the final u over the owned rows is formed by one
// more pipeline stage.
#pragma once

#include <type_traits>

#include "rm_device.h"

// every product and sum as written: the kernels that share this order agree bit for bit
#pragma clang fp contract(off)

namespace rmk {

namespace {

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

constexpr int pmod(int a, int b) { return ((a % b) + b) % b; }

// Kinds of iteration of the forward pipeline (see k_stream).
constexpr int K_RUN = 0, K_STEADY = 1, K_FILL = 2;

// A copy in a new register.  A prefetched row lives on in the pipeline's queues after
// the loader consumes it; without the copy the allocator keeps it in the prefetch
// register and moves the next (still in flight) load at the loop edge, which waits for
// the load there.
__device__ __forceinline__ float fresh(float x) {
  float y;
  asm volatile("v_mov_b32 %0, %1" : "=v"(y) : "v"(x));
  return y;
}

// Per-thread registers of the forward pipeline.  Level t = 1..TL is step t; level
// TL + 1 forms the residual.  Partial sums and queued inputs of row r live in slot
// r mod 2; PF rows are prefetched.
template <int TL, int PF>
struct StreamRegs {
  static constexpr int NL = TL + 1;
  float in[NL + 1];      // the row arriving at level t (own column), published by level t - 1
  float acc[NL + 1][2];  // partial stencil sums of level t
  float qu[NL + 1][2];   // u, v, f waiting to be updated by level t
  float qv[NL + 1][2];
  float qf[NL + 1][2];
  float pu[PF], pv[PF], pf[PF];  // prefetched rows
};

// Bounds-checked stores: a raw buffer store whose byte offset is at or beyond the
// descriptor's size is dropped by the hardware, so the stores of the owned points need
// no branch (which would split every iteration into separately scheduled blocks).
constexpr int kBufWord3 = 0x00020000;  // 32-bit data, raw (unswizzled) buffer
constexpr int kDropOffset = 0x7ffffff0;

// The pipeline of one row window: tile tl, L rows, run by the NT threads tid = 0 ..
// NT - 1 (NT = 64 ceil(n / 64), whole waves) with their own LDS block lds and one
// double per wave in sh.  Every thread of the workgroup runs the same number of
// barriers.  A window that is not live (its instance inactive, or no window at all)
// runs without storing anything.
// MAXT: the largest workgroup of the instantiation (512, or 1024 for n > 512, which
// limits a thread to 128 registers); PF: prefetch depth = iterations per unrolled body.
template <int TL, int METHOD, bool STORE, bool RES, int MAXT, int PF>
__device__ __forceinline__ void stream_run(const PlanDev& p, const BTile& tl, int L, bool live, int NT, int tid,
                                           float* lds, double* sh, const float* __restrict__ omega,
                                           const float* __restrict__ alpha, int m, int s0,
                                           const float* __restrict__ f, const float* __restrict__ u,
                                           const float* __restrict__ v, float* __restrict__ u_out,
                                           float* __restrict__ v_out, double* __restrict__ partial2,
                                           float* __restrict__ states, int64_t state_stride) {
  constexpr int NL = TL + 1;
  constexpr int NLV = RES ? NL : TL;  // levels that run
  // LDS: per column, two row slots per level (odd stride: conflict-free across lanes).
  // Block k holds grid column k - 1: block 0 and block n + 1 (never written) are the
  // zero Dirichlet border.  Threads beyond the grid use blocks NT + 2 .. NT + 4 as their
  // west, own and east columns: they read zeros and write where no other thread reads,
  // so what they compute never reaches the grid.
  constexpr int LS = 2 * NL + 1;
  const Inst in = p.inst[tl.inst];
  const int n = in.n;
  const int gx = tid;
  const bool colin = gx < n;
  const int gxc = colin ? gx : n - 1;
  const int ys = tl.y0;
  const int own0 = live ? tl.oy0 - ys : 0, own1 = live ? tl.oy1 - ys : 0;
  float c[5];
  load_coef<float>(p, tl.inst, c);
  // factors of the TL steps: fat[t] is the look-ahead of step t, applied by its producer
  float fw[NL], fa[NL], fat[NL + 1];
  static_for<1, NL>([&](auto T_) {
    constexpr int t = decltype(T_)::value;
    step_factors<float, METHOD>(p, omega, alpha, m, tl.inst, (s0 + t - 1) % m, fw[t], fa[t], fat[t]);
    fw[t] = uniform_f32(fw[t]);  // scaled by 1 / D under Jacobi preconditioning
  });
  for (int e = tid; e < (NT + 5) * LS; e += NT) lds[e] = 0.0f;
  float* lb = lds + (colin ? gx : NT + 2) * LS;  // west column; own column at + LS, east at + 2 LS
  // Rows are read through buffer resources: the column offset is fixed per thread and
  // the row offset is the same for the whole workgroup (a scalar), so a load needs no
  // address arithmetic.  Every row read lies in the field.
  const int nn4 = n * n * (int)sizeof(float);
  const __amdgpu_buffer_rsrc_t fb_in = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(f + in.off), (short)0,
                                                                         nn4, kBufWord3);
  const __amdgpu_buffer_rsrc_t ub_in = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(u + in.off), (short)0,
                                                                         nn4, kBufWord3);
  const __amdgpu_buffer_rsrc_t vb_in = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(v + in.off), (short)0,
                                                                         nn4, kBufWord3);
  const int col4 = gxc * (int)sizeof(float);
  StreamRegs<TL, PF> R;
  static_for<0, NL + 1>([&](auto T_) {
    constexpr int t = decltype(T_)::value;
    R.in[t] = 0.0f;
#pragma unroll
    for (int k = 0; k < 2; ++k) R.acc[t][k] = R.qu[t][k] = R.qv[t][k] = R.qf[t][k] = 0.0f;
  });
  auto load_row = [&](int r, float& lu, float& lv, float& lf) {
    const int row4 = (ys + r) * n * (int)sizeof(float);
    lu = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(ub_in, col4, row4, 0));
    lv = uses_momentum(METHOD) ? __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(vb_in, col4, row4, 0)) : 0.0f;
    lf = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(fb_in, col4, row4, 0));
  };
  __syncthreads();
  double r2 = 0.0;
  const int S = L + 2 * NLV;
  // store offsets: the row part is the same for the whole workgroup, and a thread
  // beyond the grid adds an offset past every field, so one addition forms the offset
  // (at most 0x7ffffff0 + 2^30: no wrap, and always beyond the field when dropped)
  const int colst = colin ? gx * (int)sizeof(float) : 0x40000000;
  const __amdgpu_buffer_rsrc_t ub_out = __builtin_amdgcn_make_buffer_rsrc(u_out + in.off, (short)0, nn4, kBufWord3);
  const __amdgpu_buffer_rsrc_t vb_out = __builtin_amdgcn_make_buffer_rsrc(v_out + in.off, (short)0, nn4, kBufWord3);
  // One iteration.  Phase A, levels from the last to the first (each consumes its
  // arriving row and queue slot before the level below refills them): level t
  // completes row y = s - 2t with the north row (its arriving row y + 1), updates it
  // and passes it on, and adds the centre row of y + 1.  Phase B: level t starts the
  // residual of row y + 2 from its f (queued by level t - 1 in phase A) with the south
  // row.  Kinds of iteration (K): K_RUN masks at run time; K_STEADY: every level's row
  // lies in the window, nothing is masked; K_FILL (s = V, a window at least as long as
  // the fill): the masks are constants, and a level skips phase A while its arriving row
  // y + 1 precedes the zero row -1, and phase B while row y + 2 precedes row 0.  What is
  // skipped would only produce values for rows before the window, which are masked,
  // never stored and never summed; the rows in the window see the same operands.
  auto iter = [&](auto PH_, auto K_, auto V_, int s) {
    constexpr int PH = decltype(PH_)::value;
    constexpr int K = decltype(K_)::value, V = decltype(V_)::value;
    constexpr int y2 = pmod(PH, 2);       // slot of row s - 2t (and of row s - 2t + 2)
    constexpr int y2n = pmod(PH + 1, 2);  // slot of row s - 2t + 1 (the arriving row)
    float Cv[NL + 2], Wv[NL + 2], Ev[NL + 2];
    // phase B of level t: the south row (the arriving row y + 1) starts row y + 2 from the
    // f that level t - 1 queued in its phase A
    auto phase_b = [&](auto T_) {
      constexpr int t = decltype(T_)::value;
      if constexpr (t >= 1 && t <= NLV && !(K == K_FILL && V - 2 * t + 2 < 0)) {
        float a0 = fmadd(-c[2], Cv[t], R.qf[t][y2]);
        a0 = fmadd(-c[3], Wv[t], a0);
        R.acc[t][y2] = fmadd(-c[4], Ev[t], a0);
      }
    };
    static_for<0, NL>([&](auto K_) {
      constexpr int t = NL - decltype(K_)::value;
      if constexpr (t <= NLV && K == K_FILL && V - 2 * t < -1) {
        // the arriving row is row -2 or earlier; phase B reads these zeros as the zero
        // row -1, the south row of row 0
        Cv[t] = Wv[t] = Ev[t] = 0.0f;
      } else if constexpr (t <= NLV) {
        const int y = s - 2 * t;
        const bool rowok = K == K_STEADY ? true : K == K_FILL ? V - 2 * t >= 0 : (unsigned)y < (unsigned)L;
        const bool rowmine = y >= own0 && y < own1;
        const bool mine = rowmine && colin;
        // row y + 1: own column from the register, neighbours from the producer's LDS slot
        const float C = R.in[t];
        const float W = lb[(t - 1) * 2 + y2n];
        const float E = lb[2 * LS + (t - 1) * 2 + y2n];
        Cv[t] = C;
        Wv[t] = W;
        Ev[t] = E;
        float r = fmadd(-c[2], C, R.acc[t][y2]);
        r = fmadd(-c[3], E, r);
        r = fmadd(-c[4], W, r);
        R.acc[t][y2n] = fmadd(-c[1], W + E, fmadd(-c[0], C, R.acc[t][y2n]));
        if constexpr (t == NL) {
          const float rm = mine ? r : 0.0f;
          r2 = __builtin_fma((double)rm, (double)rm, r2);
        } else {
          const float vn = fmadd(fa[t], R.qv[t][y2], fw[t] * r);
          const float un = R.qu[t][y2] + vn;
          if constexpr (t < TL) {
            const float x = uses_lookahead(METHOD) ? fmadd(fat[t + 1], vn, un) : un;
            const float pub = rowok ? x : 0.0f;
            R.in[t + 1] = pub;
            lb[LS + t * 2 + y2] = pub;
            R.qf[t + 1][y2] = R.qf[t][y2];
            R.qu[t + 1][y2] = un;
            R.qv[t + 1][y2] = vn;
            if (STORE && mine) {
              const int64_t gidx = in.off + (int64_t)(ys + y) * n + gx;
              float* su = states + (int64_t)(t - 1) * state_stride;
              su[gidx] = un;
              if (uses_momentum(METHOD)) su[gidx + state_stride / 2] = vn;
            }
          } else {
            const int boff = (rowmine ? (ys + y) * n * (int)sizeof(float) : kDropOffset) + colst;
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(un), ub_out, boff, 0, 0);
            if (uses_momentum(METHOD))
              __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(vn), vb_out, boff, 0, 0);
            if constexpr (RES) {
              const float pub = rowok ? un : 0.0f;
              R.in[NL] = pub;
              lb[LS + TL * 2 + y2] = pub;
              R.qf[NL][y2] = R.qf[t][y2];
            }
          }
        }
      }
      // level t has queued f for level t + 1: its phase B can run
      phase_b(std::integral_constant<int, t + 1>{});
    });
    // loader: row s enters level 1
    {
      const bool rowok = K == K_STEADY || K == K_FILL || (unsigned)s < (unsigned)L;
      const float lu = fresh(R.pu[PH]), lv = fresh(R.pv[PH]), lf = fresh(R.pf[PH]);
      const float x = uses_lookahead(METHOD) ? fmadd(fat[1], lv, lu) : lu;
      const float pub = rowok ? x : 0.0f;
      R.in[1] = pub;
      lb[LS + y2] = pub;
      R.qu[1][y2] = lu;
      R.qv[1][y2] = lv;
      R.qf[1][y2] = lf;
      // unconditional (clamped) so that the loaded registers are not merged with old ones
      load_row(min(s + PF, L - 1), R.pu[PH], R.pv[PH], R.pf[PH]);
    }
    phase_b(std::integral_constant<int, 1>{});
    __syncthreads();
  };
  // fill and drain iterations mask rows outside the window; in between none is
  // With L >= FF the fill (s = 0 .. FF - 1) is unrolled with its masks known (L is the
  // same for the whole workgroup, so every thread takes the same branch).  Only for the
  // longest pipeline of the sweeps; the others and the recompute that stores the states
  // keep the run-time masks.  (An unrolled drain, one copy per value of L - D, costs
  // the kernels their registers: the compiler spills or lowers the occupancy.)
  constexpr int FF = ((2 * NLV + PF - 1) / PF) * PF;
  constexpr bool UNROLLED = TL == kStreamMaxT && !STORE;
  using Run = std::integral_constant<int, K_RUN>;
  using Steady = std::integral_constant<int, K_STEADY>;
  using V0 = std::integral_constant<int, 0>;
  const int F = min(S, FF);
  const int D = F + max(0, (L - F) / PF) * PF;
  int s = 0;
  // The first PF rows are requested inside each branch: on every path to the steady loop
  // they have been consumed, so its loads are waited for only where they are used.
  if (UNROLLED && L >= FF) {
    static_for<0, PF>([&](auto K_) {
      constexpr int k = decltype(K_)::value;
      load_row(k, R.pu[k], R.pv[k], R.pf[k]);
    });
    static_for<0, UNROLLED ? FF : 0>([&](auto S_) {
      constexpr int sc = decltype(S_)::value;
      iter(std::integral_constant<int, sc % PF>{}, std::integral_constant<int, K_FILL>{}, S_, sc);
    });
    s = FF;
  } else {
    // at least one pass (F >= 2 NLV > 0): no path reaches the steady loop with the first
    // prefetched rows still in flight, which would make the compiler wait for every load
    // at the top of each steady pass
    static_for<0, PF>([&](auto K_) {
      constexpr int k = decltype(K_)::value;
      load_row(min(k, L - 1), R.pu[k], R.pv[k], R.pf[k]);
    });
#pragma unroll 1
    do {
      static_for<0, PF>([&](auto PH_) { iter(PH_, Run{}, V0{}, s + decltype(PH_)::value); });
      s += PF;
    } while (s < F);
  }
#pragma unroll 1
  for (; s < D; s += PF)
    static_for<0, PF>([&](auto PH_) { iter(PH_, Steady{}, V0{}, s + decltype(PH_)::value); });
#pragma unroll 1
  for (; s < S; s += PF)
    static_for<0, PF>([&](auto PH_) { iter(PH_, Run{}, V0{}, s + decltype(PH_)::value); });
  if constexpr (RES) {
    r2 = wave_sum(r2);
    if ((tid & 63) == 0) sh[tid >> 6] = r2;
    __syncthreads();
    if (live && tid == 0) {
      double sum = 0.0;
      for (int k = 0; k < NT / 64; ++k) sum += sh[k];
      partial2[2 * tl.slot] = sum;
      partial2[2 * tl.slot + 1] = 0.0;
    }
  }
}

}  // namespace
}  // namespace rmk
