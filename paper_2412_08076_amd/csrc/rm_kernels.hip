// HIP kernels for gfx950 (CDNA4, wave64) of the long-step Richardson(m) hot path.
//
// Operators (arXiv 2412.08076): the Q1 9-point stencil of the anisotropic
// diffusion problem (§2.3) and the 5-point Helmholtz stencil (§3.2), both held as
// five per-instance coefficients: centre, (+-1,0), (0,+-1), (1,1)/(-1,-1) and
// (-1,1)/(1,-1).  Schemes: Richardson(m) and NAG-Richardson(m) (Table 1).
//
// Work decomposition.  Every kernel here walks a plan's tile table: one
// workgroup of 256 threads (4 waves) owns a 64 x 32 output tile of one instance,
// one thread per column and 8 rows per thread.  The inputs of a tile plus a
// one-point halo are staged in LDS; points outside the n x n interior read as 0
// (homogeneous Dirichlet), so ragged tails and boundaries need no special code.
// The block index is remapped so that consecutive tiles land on the same XCD
// (hardware dispatch is round robin over the 8 XCDs), which keeps the halo rows
// shared by neighbouring tiles in one L2.
//
// Reductions (residual norms, adjoint dot products) are formed per tile in FP64
// with a fixed shuffle tree, then summed per instance in tile order by a second
// kernel: results are bitwise reproducible run to run.
//
// All floating-point combinations are written as explicit fused multiply-adds
// with contraction switched off, so the single-step, adjoint-recompute and any
// other kernel that evaluates the same stencil produce identical bits.
#include "rm_device.h"

#pragma clang fp contract(off)

namespace rmk {

namespace {

constexpr int LDS_W = TX + 2;
constexpr int RPT = TY / (WG / TX);  // rows per thread
constexpr int NWAVE = WG / 64;

// One inner step's new momentum at a point, v' = a v + w (f - A s) with the residual
// of residual9, the sequence of step_vf, which every kernel that advances the iteration
// uses, so they agree bit for bit.
template <typename T>
__device__ __forceinline__ T step_v(const T c[5], T w, T a, T f, T v, T C, T W, T E, T S, T N, T SW, T NE, T SE,
                                    T NW) {
  return fmadd(a, v, w * residual9<T>(c, f, C, W, E, S, N, SW, NE, SE, NW));
}

// Stencil at LDS position (lx, ly) of a (TY+2) x LDS_W tile.
template <typename T>
__device__ __forceinline__ T stencil_lds(const T* s, int lx, int ly, const T c[5]) {
  const T* rs = s + (ly - 1) * LDS_W + lx;
  const T* rc = s + ly * LDS_W + lx;
  const T* rn = s + (ly + 1) * LDS_W + lx;
  return stencil9(c, rc[0], rc[-1], rc[1], rs[0], rn[0], rs[-1], rn[1], rs[1], rn[-1]);
}

// f - A s at LDS position (lx, ly), in the order of residual9.
template <typename T>
__device__ __forceinline__ T residual_lds(const T* s, int lx, int ly, const T c[5], T f) {
  const T* rs = s + (ly - 1) * LDS_W + lx;
  const T* rc = s + ly * LDS_W + lx;
  const T* rn = s + (ly + 1) * LDS_W + lx;
  return residual9(c, f, rc[0], rc[-1], rc[1], rs[0], rn[0], rs[-1], rn[1], rs[1], rn[-1]);
}

// Fill the one-point halo ring of the LDS tile with val(gx, gy), or 0 outside the
// n x n interior (val is called at (0, 0) there, so it must not fault on it).
template <typename T, typename F>
__device__ __forceinline__ void stage_halo(T* s, int x0, int y0, int n, F&& val) {
  constexpr int NH = 2 * LDS_W + 2 * TY;
  for (int h = threadIdx.x; h < NH; h += WG) {
    int hx, hy;
    if (h < LDS_W) {
      hx = h; hy = 0;
    } else if (h < 2 * LDS_W) {
      hx = h - LDS_W; hy = TY + 1;
    } else if (h < 2 * LDS_W + TY) {
      hx = 0; hy = 1 + (h - 2 * LDS_W);
    } else {
      hx = TX + 1; hy = 1 + (h - 2 * LDS_W - TY);
    }
    const int gx = x0 + hx - 1, gy = y0 + hy - 1;
    const bool in = (gx >= 0) && (gx < n) && (gy >= 0) && (gy < n);
    const T x = val(in ? gx : 0, in ? gy : 0);   // an in-bounds load behind no branch
    s[hy * LDS_W + hx] = in ? x : T(0);
  }
}

// ---------------------------------------------------------------------------
// y = A x  /  r = b - A x with per-tile ||r||^2, ||b||^2
// ---------------------------------------------------------------------------
template <typename T, int MODE>  // MODE 0: y = A x; MODE 1: residual (+ partials)
__global__ __launch_bounds__(WG) void k_apply(PlanDev p, const Tile* tiles, const T* __restrict__ b,
                                              const T* __restrict__ x, T* __restrict__ y,
                                              double* __restrict__ partial2,
                                              const int* __restrict__ active) {
  __shared__ T s[(TY + 2) * LDS_W];
  __shared__ double sh[NWAVE];
  const Tile tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
  if (tl.inst < 0) return;
  if (active != nullptr && active[tl.inst] == 0) return;
  const Inst in = p.inst[tl.inst];
  const int n = in.n;
  T c[5];
  load_coef<T>(p, tl.inst, c);
  const Field<T> xf(x + in.off, n * n), bf(MODE == 1 ? b + in.off : x + in.off, n * n);
  const int tx = threadIdx.x & 63, ty0 = threadIdx.x >> 6;
  const int gx = tl.x0 + tx;
  // every load on an in-bounds index (0 for points off the grid) and behind no branch
  T rx[RPT], rb[RPT];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int gy = tl.y0 + ty0 + 4 * k;
    const bool in_ = gx < n && gy < n;
    const unsigned idx = in_ ? (unsigned)(gy * n + gx) : 0u;
    rx[k] = xf[idx];
    rb[k] = MODE == 1 ? bf[idx] : T(0);
    rx[k] = in_ ? rx[k] : T(0);
  }
#pragma unroll
  for (int k = 0; k < RPT; ++k) s[(ty0 + 4 * k + 1) * LDS_W + tx + 1] = rx[k];
  stage_halo(s, tl.x0, tl.y0, n, [&](int X, int Y) { return xf[(unsigned)(Y * n + X)]; });
  __syncthreads();
  double r2 = 0.0, b2 = 0.0;
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int ly = ty0 + 4 * k, gy = tl.y0 + ly;
    if (gx < n && gy < n) {
      const int64_t idx = in.off + (int64_t)gy * n + gx;
      if (MODE == 0) {
        y[idx] = stencil_lds(s, tx + 1, ly + 1, c);
      } else {
        const T bv = rb[k];
        const T r = residual_lds(s, tx + 1, ly + 1, c, bv);
        if (y != nullptr) y[idx] = r;
        r2 += (double)r * (double)r;
        b2 += (double)bv * (double)bv;
      }
    }
  }
  if (MODE == 1 && partial2 != nullptr) {
    const double t0 = block_sum(r2, sh);
    __syncthreads();
    const double t1 = block_sum(b2, sh);
    if (threadIdx.x == 0) {
      partial2[2 * tl.pad + 0] = t0;
      partial2[2 * tl.pad + 1] = t1;
    }
  }
}

// ---------------------------------------------------------------------------
// One fused inner step of the Table-1 schemes (last column) in NAGex form:
//   u~ = u + at_i v;  r = f - A u~;  v' = a_i v + w_i r;  u' = u + v'
// with at = a (NAG), at = 0 (MOM), a = at = 0 (Richardson); under weighted-Jacobi
// preconditioning w_i carries the factor 1/D of the constant diagonal.
// ---------------------------------------------------------------------------
template <typename T, int METHOD>
__global__ __launch_bounds__(WG) void k_step(PlanDev p, const Tile* tiles, const float* __restrict__ omega,
                                             const float* __restrict__ alpha, int m, int i,
                                             const T* __restrict__ f, const T* __restrict__ u,
                                             const T* __restrict__ v, T* __restrict__ u_out,
                                             T* __restrict__ v_out, const int* __restrict__ active) {
  __shared__ T s[(TY + 2) * LDS_W];
  const Tile tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
  if (tl.inst < 0) return;
  if (active != nullptr && active[tl.inst] == 0) return;
  const Inst in = p.inst[tl.inst];
  const int n = in.n;
  T c[5];
  load_coef<T>(p, tl.inst, c);
  T w, a, at;
  step_factors<T, METHOD>(p, omega, alpha, m, tl.inst, i, w, a, at);
  const int nn = n * n;
  const Field<T> uf(u + in.off, nn), vf(v + in.off, nn), ff(f + in.off, nn);
  const int tx = threadIdx.x & 63, ty0 = threadIdx.x >> 6;
  const int gx = tl.x0 + tx;
  // every load on an in-bounds index (0 for points off the grid) and behind no branch
  T ru[RPT], rv[RPT], rf[RPT];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int gy = tl.y0 + ty0 + 4 * k;
    const bool in_ = gx < n && gy < n;
    const unsigned idx = in_ ? (unsigned)(gy * n + gx) : 0u;
    const T lu = uf[idx], lv = uses_momentum(METHOD) ? vf[idx] : T(0), lf = ff[idx];
    ru[k] = in_ ? lu : T(0);
    rv[k] = in_ ? lv : T(0);
    rf[k] = in_ ? lf : T(0);
  }
#pragma unroll
  for (int k = 0; k < RPT; ++k)
    s[(ty0 + 4 * k + 1) * LDS_W + tx + 1] = uses_lookahead(METHOD) ? fmadd(at, rv[k], ru[k]) : ru[k];
  if (uses_lookahead(METHOD))
    stage_halo(s, tl.x0, tl.y0, n, [&](int X, int Y) {
      const unsigned e = (unsigned)(Y * n + X);
      return fmadd(at, vf[e], uf[e]);
    });
  else
    stage_halo(s, tl.x0, tl.y0, n, [&](int X, int Y) { return uf[(unsigned)(Y * n + X)]; });
  __syncthreads();
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int ly = ty0 + 4 * k, gy = tl.y0 + ly;
    if (gx < n && gy < n) {
      const T* rs = s + ly * LDS_W + tx + 1;
      const T* rc = rs + LDS_W;
      const T* rn = rc + LDS_W;
      const T vn = step_v(c, w, a, rf[k], rv[k], rc[0], rc[-1], rc[1], rs[0], rn[0], rs[-1], rn[1], rs[1], rn[-1]);
      const int64_t idx = in.off + (int64_t)gy * n + gx;
      u_out[idx] = ru[k] + vn;
      if (uses_momentum(METHOD)) v_out[idx] = vn;
    }
  }
}

// Per-instance fixed-order sum of per-tile partials: one wave per instance.
__global__ __launch_bounds__(64) void k_reduce_partials(PlanDev p, const double* __restrict__ partial2,
                                                        const int* __restrict__ ranges,
                                                        double* __restrict__ out0, double* __restrict__ out1,
                                                        int stride, float* __restrict__ ratio) {
  const int b = blockIdx.x;
  const Inst in = p.inst[b];
  const int t0 = ranges != nullptr ? ranges[2 * b] : in.tile_begin;
  const int t1 = ranges != nullptr ? ranges[2 * b + 1] : in.tile_end;
  double s0 = 0.0, s1 = 0.0;
  for (int t = t0 + (int)threadIdx.x; t < t1; t += 64) {
    s0 += partial2[2 * t];
    s1 += partial2[2 * t + 1];
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  if (threadIdx.x == 0) {
    if (out0 != nullptr) out0[b * stride] = s0;
    if (out1 != nullptr) out1[b * stride] = s1;
    if (ratio != nullptr) ratio[b] = (float)(s0 / s1);
  }
}

// ---------------------------------------------------------------------------
// FP64 iterative refinement
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(WG) void k_refine_residual(PlanDev p, const double* __restrict__ b,
                                                        const double* __restrict__ x, float* __restrict__ r32,
                                                        float* __restrict__ d, float* __restrict__ v,
                                                        double* __restrict__ partial2,
                                                        const int* __restrict__ mask) {
  __shared__ double s[(TY + 2) * LDS_W];
  __shared__ double sh[NWAVE];
  const Tile tl = p.tiles[xcd_remap(blockIdx.x, gridDim.x)];
  if (tl.inst < 0) return;
  if (mask != nullptr && mask[tl.inst] == 0) return;
  const Inst in = p.inst[tl.inst];
  const int n = in.n;
  double c[5];
  load_coef<double>(p, tl.inst, c);
  const double* xi = x + in.off;
  const int tx = threadIdx.x & 63, ty0 = threadIdx.x >> 6;
  const int gx = tl.x0 + tx;
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int ly = ty0 + 4 * k, gy = tl.y0 + ly;
    s[(ly + 1) * LDS_W + tx + 1] = (gx < n && gy < n) ? xi[gy * n + gx] : 0.0;
  }
  stage_halo(s, tl.x0, tl.y0, n, [&](int X, int Y) { return xi[Y * n + X]; });
  __syncthreads();
  double r2 = 0.0, b2 = 0.0;
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int ly = ty0 + 4 * k, gy = tl.y0 + ly;
    if (gx < n && gy < n) {
      const int64_t idx = in.off + (int64_t)gy * n + gx;
      const double bv = b[idx];
      const double r = bv - stencil_lds(s, tx + 1, ly + 1, c);
      r32[idx] = (float)r;
      d[idx] = 0.0f;
      v[idx] = 0.0f;
      r2 += r * r;
      b2 += bv * bv;
    }
  }
  const double t0 = block_sum(r2, sh);
  __syncthreads();
  const double t1 = block_sum(b2, sh);
  if (threadIdx.x == 0) {
    partial2[2 * tl.pad + 0] = t0;
    partial2[2 * tl.pad + 1] = t1;
  }
}

__global__ __launch_bounds__(WG) void k_refine_update(PlanDev p, double* __restrict__ x,
                                                      const float* __restrict__ d0,
                                                      const float* __restrict__ d1,
                                                      const int* __restrict__ start, const int* __restrict__ outer_count,
                                                      int flips, const int* __restrict__ mask) {
  const Tile tl = p.tiles[xcd_remap(blockIdx.x, gridDim.x)];
  if (tl.inst < 0) return;
  if (mask[tl.inst] == 0) return;
  const Inst in = p.inst[tl.inst];
  const int n = in.n;
  const int64_t iters = (int64_t)(start != nullptr ? start[tl.inst] : 0) + outer_count[tl.inst];
  const float* d = ((iters * flips) & 1) ? d1 : d0;
  const int tx = threadIdx.x & 63, ty0 = threadIdx.x >> 6;
  const int gx = tl.x0 + tx;
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int gy = tl.y0 + ty0 + 4 * k;
    if (gx < n && gy < n) {
      const int64_t idx = in.off + (int64_t)gy * n + gx;
      x[idx] = x[idx] + (double)d[idx];
    }
  }
}
// End of one instance's refinement round, one wave per instance waiting for it
// (pending): rho = ||b - A x|| / ||b|| from the refinement residual's tile partials
// (summed in the order of k_reduce_partials), recorded as the round's history entry,
// then either the instance is done (rho <= tol, zero residual, non-finite or diverged,
// the round cap, or a second round that did not halve rho) or its next inner solve
// starts with the target max(tol_inner, tol / (2 rho))^2 ||r||^2 at outer iteration
// rp.start of the solve.
__global__ __launch_bounds__(64) void k_round_decide(PlanDev p, const double* __restrict__ partial2, RoundParams rp,
                                                     RoundState rs) {
  const int b = blockIdx.x;
  if (rs.pending[b] == 0) return;
  const Inst in = p.inst[b];
  double s0 = 0.0, s1 = 0.0;
  for (int t = in.tile_begin + (int)threadIdx.x; t < in.tile_end; t += 64) {
    s0 += partial2[2 * t];
    s1 += partial2[2 * t + 1];
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  if (threadIdx.x != 0) return;
  const int j = rs.round[b];
  const double rho = s1 > 0.0 ? sqrt(s0 / s1) : sqrt(s0);
  rs.relres[b] = rho;
  if (j <= rp.max_rounds) rs.history[(int64_t)j * p.B + b] = rho;
  int fin = 0;
  if (!isfinite(rho) || rs.status[b] == 5) {
    fin = 5;  // RM_EDIVERGED
  } else if (rho <= rp.tol || s0 == 0.0) {
    fin = -1;  // converged
  } else if (j >= rp.max_rounds) {
    fin = 4;  // RM_ENOTCONV: round cap
  } else if (j > 0 && rho > 0.5 * rs.prev_rho[b]) {
    const int k = rs.strikes[b] + 1;
    rs.strikes[b] = k;
    if (k >= 2) fin = 4;  // two rounds without halving the residual
  }
  rs.prev_rho[b] = rho;
  rs.pending[b] = 0;
  if (fin != 0) {
    rs.status[b] = fin > 0 ? fin : 0;
    rs.active[b] = 0;
    return;
  }
  const double tau = fmax(rp.tol_inner, 0.5 * rp.tol / rho);
  rs.target2[b] = tau * tau * s0;
  rs.rhs2[b] = s0;
  rs.best2[b] = s0;
  rs.tot[b] += rs.count[b];
  rs.count[b] = 0;
  rs.since[b] = 0;
  rs.gains[b] = 0;
  rs.start[b] = rp.start;
  rs.round[b] = j + 1;
  rs.active[b] = 1;
}

// The residual of the inner iterate after one outer iteration: res2[b] = the sum of
// instance b's residual partials over the slot range of the configuration its class ran,
// one wave per instance in the order of k_reduce_partials (lane j adds slots t0 + j,
// t0 + j + 64, ..., then a fixed tree over the lanes).  Spread over the whole chip, its
// loads are coalesced; one workgroup summing thousands of scattered slots was bound by
// its single CU's load path.
__global__ __launch_bounds__(64) void k_outer_sums(PlanDev p, const double* __restrict__ partial2,
                                                   const int* __restrict__ ranges, const int* __restrict__ tranges,
                                                   const int* __restrict__ cls, unsigned long long tailmask,
                                                   double* __restrict__ res2) {
  const int b = blockIdx.x;
  const int ci = cls != nullptr ? cls[b] : 0;
  const int* rg = (tranges != nullptr && ci < 64 && ((tailmask >> ci) & 1ull)) ? tranges : ranges;
  const int t0 = rg != nullptr ? rg[2 * b] : p.inst[b].tile_begin;
  const int t1 = rg != nullptr ? rg[2 * b + 1] : p.inst[b].tile_end;
  double s = 0.0;
  for (int t = t0 + (int)threadIdx.x; t < t1; t += 64) s += partial2[2 * t];
  s = wave_sum(s);
  if (threadIdx.x == 0) res2[b] = s;
}

// After one outer iteration of an inner solve: stop instances whose residual
// reached their target, hit the cap, went non-finite or grew beyond 1e6 times
// the right-hand side, or stagnated; count the rest.  Stagnation: no 10 %
// reduction of the best residual for W outer iterations, where W is six times
// the instance's own average spacing of such reductions so far in this round,
// clamped to [stall_min, stall_max] (stall_max before the first reduction):
// an instance at its FP32 floor stops quickly, a slowly converging large one is
// given time.
// Bookkeeping after one outer iteration of the refined solve, in one workgroup with a
// thread per instance: for active instances the count, divergence, target, cap and
// stagnation tests on res2 (formed by k_outer_sums); finally the number still active,
// summed over the threads in a fixed order (no atomics and no counter to clear beforehand).
__global__ __launch_bounds__(1024) void k_outer_flags(
    PlanDev p, const int* __restrict__ cls, int ncls,
    const double* __restrict__ res2, const double* __restrict__ rhs2, const double* __restrict__ target2,
    double* __restrict__ best2, int* __restrict__ since, int* __restrict__ gains, int stall_min, int stall_max,
    int cap, int* __restrict__ active, int* __restrict__ outer_count, int* __restrict__ status,
    int* __restrict__ pending, int* __restrict__ n_active, unsigned long long* __restrict__ host_word,
    unsigned long long* __restrict__ host_cnt, unsigned seq,
    const int* __restrict__ tot, double* __restrict__ hist, int hist_len) {
  __shared__ int kept[16];
  __shared__ int waiting[16];
  extern __shared__ int per_class[];  // [ncls] instances per size class not yet done
  for (int c = threadIdx.x; c < ncls; c += blockDim.x) per_class[c] = 0;
  __syncthreads();
  int mine = 0, pend = 0;
  for (int b = threadIdx.x; b < p.B; b += blockDim.x) {
    const int ci = cls != nullptr ? cls[b] : 0;
    const int act = active[b], cnt = outer_count[b] + 1, sn = since[b], g = gains[b];
    const int pd = pending != nullptr ? pending[b] : 0;
    const double rh = rhs2[b], tg = target2[b], best = best2[b];
    const double r2 = res2[b];
    if (act == 0) {
      // a round that ended earlier and waits for its refinement step
      pend += pd;
      if (pd && ci < ncls) atomicAdd(&per_class[ci], 1);
      continue;
    }
    outer_count[b] = cnt;
    if (hist != nullptr) {
      const int k = tot[b] + cnt - 1;  // outer iterations of this instance over all rounds, from 0
      if (k < hist_len) hist[(int64_t)k * p.B + b] = r2;
    }
    int keep = 1;
    if (!(r2 <= 1e12 * rh)) {  // NaN, Inf or growth
      status[b] = 5;           // RM_EDIVERGED
      keep = 0;
    } else if (r2 <= tg || cnt >= cap) {
      keep = 0;
    } else if (r2 < 0.81 * best) {
      best2[b] = r2;
      since[b] = 0;
      gains[b] = g + 1;
    } else {
      int win = g == 0 ? stall_max : (6 * cnt) / g;
      win = win < stall_min ? stall_min : (win > stall_max ? stall_max : win);
      if (sn + 1 >= win) keep = 0;
      else since[b] = sn + 1;
    }
    active[b] = keep;
    mine += keep;
    // the inner solve of this round has ended: the refinement step takes over
    if (!keep && pending != nullptr) {
      pending[b] = 1;
      ++pend;
    }
    if ((keep || pending != nullptr) && ci < ncls) atomicAdd(&per_class[ci], 1);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    mine += __shfl_xor(mine, o, 64);
    pend += __shfl_xor(pend, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    kept[threadIdx.x >> 6] = mine;
    waiting[threadIdx.x >> 6] = pend;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int total = 0, total_pend = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
      total += kept[k];
      total_pend += waiting[k];
    }
    *n_active = total;
    // straight to the host's pinned copies (system scope, vector stores), each one
    // 64-bit word stamped with the launch number, so the host can tell which launch
    // wrote it without any ordering between the words: the per-class counts of
    // instances not done, the count of rounds waiting for their refinement step, then
    // the count of instances not done (active or waiting)
    if (host_word != nullptr) {
      if (host_cnt != nullptr)
        for (int c = 0; c < ncls; ++c)
          __hip_atomic_store(host_cnt + c, ((unsigned long long)seq << 32) | (unsigned)per_class[c],
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(host_word + 1, ((unsigned long long)seq << 32) | (unsigned)total_pend, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(host_word, ((unsigned long long)seq << 32) | (unsigned)(total + total_pend),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}


template <typename T>
__global__ void k_fill(T* __restrict__ p, T value, int64_t count) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < count;
       k += (int64_t)gridDim.x * blockDim.x)
    p[k] = value;
}

__global__ void k_f64_to_f32(const double* __restrict__ s, float* __restrict__ d, int64_t count) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < count;
       k += (int64_t)gridDim.x * blockDim.x)
    d[k] = (float)s[k];
}

// ---------------------------------------------------------------------------
// Adjoint of the K-step unroll
// ---------------------------------------------------------------------------
// Terminal values for J = sum_b g_b ||r_K||^2 / ||b||^2 with r_K = b - A u_K:
//   ub = -2 g_b / ||b||^2 A r_K,  fb = g_b (2 r_K - 2 L_b b) / ||b||^2.
__global__ __launch_bounds__(WG) void k_adj_terminal(PlanDev p, const float* __restrict__ f,
                                                     const float* __restrict__ rK,
                                                     const double* __restrict__ r2b2,
                                                     const float* __restrict__ g_loss,
                                                     float* __restrict__ ub, float* __restrict__ fb,
                                                     float* __restrict__ loss) {
  __shared__ float s[(TY + 2) * LDS_W];
  const Tile tl = p.tiles[xcd_remap(blockIdx.x, gridDim.x)];
  if (tl.inst < 0) return;
  const int bi = tl.inst;
  const Inst in = p.inst[bi];
  const int n = in.n;
  float c[5];
  load_coef<float>(p, bi, c);
  const double r2 = r2b2[2 * bi], b2 = r2b2[2 * bi + 1];
  const double L = r2 / b2;
  const double g = g_loss != nullptr ? (double)g_loss[bi] : 1.0;
  if (loss != nullptr && tl.pad == in.tile_begin && threadIdx.x == 0) loss[bi] = (float)L;
  const float su = (float)(-2.0 * g / b2);
  const float sr = (float)(2.0 * g / b2);
  const float sb = (float)(-2.0 * g * L / b2);
  const float* ri = rK + in.off;
  const int tx = threadIdx.x & 63, ty0 = threadIdx.x >> 6;
  const int gx = tl.x0 + tx;
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int ly = ty0 + 4 * k, gy = tl.y0 + ly;
    s[(ly + 1) * LDS_W + tx + 1] = (gx < n && gy < n) ? ri[gy * n + gx] : 0.0f;
  }
  stage_halo(s, tl.x0, tl.y0, n, [&](int X, int Y) { return ri[Y * n + X]; });
  __syncthreads();
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int ly = ty0 + 4 * k, gy = tl.y0 + ly;
    if (gx < n && gy < n) {
      const int64_t idx = in.off + (int64_t)gy * n + gx;
      ub[idx] = su * stencil_lds(s, tx + 1, ly + 1, c);
      if (fb != nullptr) fb[idx] = fmadd(sr, s[(ly + 1) * LDS_W + tx + 1], sb * f[idx]);
    }
  }
}

// Reverse of one forward step s (weight index i) of the NAGex-form recurrence, from
// the forward state (u, v) = (u_{s-1}, v_{s-1}) and the adjoints (ub, vb) of
// (u_s, v_s):  g = vb + ub;  r_s = f - A(u + at v);  rb = w g;  fb += rb;
// ut_bar = -A rb (A is symmetric);  ub' = ub + ut_bar;  vb' = a g + at ut_bar
// (NAG: a (g + ut_bar)).  Per tile it leaves <g, r_s>, <g, v> and <ut_bar, v>.
template <int METHOD>
__global__ __launch_bounds__(WG) void k_adj_step(PlanDev p, const float* __restrict__ omega,
                                                 const float* __restrict__ alpha, int m, int i,
                                                 const float* __restrict__ f, const float* __restrict__ u,
                                                 const float* __restrict__ v, const float* __restrict__ ub,
                                                 const float* __restrict__ vb, float* __restrict__ ub_out,
                                                 float* __restrict__ vb_out, float* __restrict__ fb,
                                                 double* __restrict__ partial4) {
  __shared__ float su[(TY + 2) * LDS_W];
  __shared__ float sg[(TY + 2) * LDS_W];
  __shared__ double sh[NWAVE];
  const Tile tl = p.tiles[xcd_remap(blockIdx.x, gridDim.x)];
  if (tl.inst < 0) return;
  const int bi = tl.inst;
  const Inst in = p.inst[bi];
  const int n = in.n;
  float c[5];
  load_coef<float>(p, bi, c);
  float w, a, at;
  step_factors<float, METHOD>(p, omega, alpha, m, bi, i, w, a, at);
  const int nn = n * n;
  const Field<float> uf(u + in.off, nn), vf(v + in.off, nn), ubf(ub + in.off, nn), vbf(vb + in.off, nn);
  const Field<float> ff(f + in.off, nn), fbf(fb != nullptr ? fb + in.off : ub + in.off, nn);
  const int tx = threadIdx.x & 63, ty0 = threadIdx.x >> 6;
  const int gx = tl.x0 + tx;
  // every load on an in-bounds index (0 for points off the grid) and behind no branch
  float rv[RPT], rg[RPT], rub[RPT], rut[RPT], rf[RPT], rfb[RPT];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int gy = tl.y0 + ty0 + 4 * k;
    const bool in_ = gx < n && gy < n;
    const unsigned idx = in_ ? (unsigned)(gy * n + gx) : 0u;
    const float uu = uf[idx], lv = uses_momentum(METHOD) ? vf[idx] : 0.0f, lub = ubf[idx];
    const float vbb = uses_momentum(METHOD) ? vbf[idx] : 0.0f;
    rf[k] = ff[idx];
    rfb[k] = fb != nullptr ? fbf[idx] : 0.0f;
    rv[k] = in_ ? lv : 0.0f;
    rub[k] = in_ ? lub : 0.0f;
    rg[k] = (in_ ? vbb : 0.0f) + rub[k];
    const float u0 = in_ ? uu : 0.0f;
    rut[k] = uses_lookahead(METHOD) ? fmadd(at, rv[k], u0) : u0;
  }
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    su[(ty0 + 4 * k + 1) * LDS_W + tx + 1] = rut[k];
    sg[(ty0 + 4 * k + 1) * LDS_W + tx + 1] = rg[k];
  }
  if (uses_lookahead(METHOD))
    stage_halo(su, tl.x0, tl.y0, n, [&](int X, int Y) {
      const unsigned e = (unsigned)(Y * n + X);
      return fmadd(at, vf[e], uf[e]);
    });
  else
    stage_halo(su, tl.x0, tl.y0, n, [&](int X, int Y) { return uf[(unsigned)(Y * n + X)]; });
  if (uses_momentum(METHOD))
    stage_halo(sg, tl.x0, tl.y0, n, [&](int X, int Y) {
      const unsigned e = (unsigned)(Y * n + X);
      return vbf[e] + ubf[e];
    });
  else
    stage_halo(sg, tl.x0, tl.y0, n, [&](int X, int Y) { return ubf[(unsigned)(Y * n + X)]; });
  __syncthreads();
  double pw = 0.0, pg = 0.0, pl = 0.0;
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int ly = ty0 + 4 * k, gy = tl.y0 + ly;
    if (gx < n && gy < n) {
      const int64_t idx = in.off + (int64_t)gy * n + gx;
      const float r = rf[k] - stencil_lds(su, tx + 1, ly + 1, c);
      const float g = rg[k];
      const float utb = -(w * stencil_lds(sg, tx + 1, ly + 1, c));
      pw += (double)g * (double)r;
      pg += (double)g * (double)rv[k];
      pl += (double)utb * (double)rv[k];
      ub_out[idx] = rub[k] + utb;
      if (METHOD == M_NAG) vb_out[idx] = a * (g + utb);
      if (METHOD == M_MOM) vb_out[idx] = a * g;
      if (METHOD == M_NAGEX) vb_out[idx] = fmadd(at, utb, a * g);
      if (fb != nullptr) fb[idx] = fmadd(w, g, rfb[k]);
    }
  }
  const double t0 = block_sum(pw, sh);
  __syncthreads();
  const double t1 = block_sum(pg, sh);
  __syncthreads();
  const double t2 = block_sum(pl, sh);
  if (threadIdx.x == 0) {
    partial4[4 * tl.pad + 0] = t0;
    partial4[4 * tl.pad + 1] = t1;
    partial4[4 * tl.pad + 2] = t2;
    partial4[4 * tl.pad + 3] = 0.0;
  }
}

template <int METHOD>
__global__ __launch_bounds__(64) void k_adj_accumulate(PlanDev p, const double* __restrict__ partial4, int nslot,
                                                       int E, int s_first, int m, double* __restrict__ acc_w,
                                                       double* __restrict__ acc_a, const int* __restrict__ ranges) {
  const int b = blockIdx.x;
  const Inst in = p.inst[b];
  const double dinv = p.jacobi ? p.coef64[b * 8 + 5] : 1.0;
  const int k0 = ranges != nullptr ? ranges[2 * b] : in.tile_begin;
  const int k1 = ranges != nullptr ? ranges[2 * b + 1] : in.tile_end;
  for (int t = E - 1; t >= 0; --t) {
    const double* q = partial4 + (size_t)t * 4 * nslot;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int k = k0 + (int)threadIdx.x; k < k1; k += 64) {
      s0 += q[4 * k];
      s1 += q[4 * k + 1];
      s2 += q[4 * k + 2];
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    if (threadIdx.x == 0) {
      const int i = (s_first + t) % m;
      acc_w[b * m + i] += dinv * s0;
      if (METHOD == M_NAG) acc_a[b * m + i] += s1 + s2;
      if (METHOD == M_MOM || METHOD == M_NAGEX) acc_a[b * m + i] += s1;
      if (METHOD == M_NAGEX) acc_a[(p.B + b) * m + i] += s2;
    }
  }
}

// ---------------------------------------------------------------------------
// Meta network: (log10 eps, theta) -> tanh 64 -> tanh 64 -> m + 1, head
// omega_i = exp(z_i) / G, alpha_i = sigmoid(z_m).  One wave per instance.
// ---------------------------------------------------------------------------
constexpr int MH = 64;

struct MetaPtrs {
  const float *W1, *b1, *W2, *b2, *W3, *b3;
};
__device__ __forceinline__ MetaPtrs meta_ptrs(const float* P, int m) {
  MetaPtrs q;
  q.W1 = P;
  q.b1 = q.W1 + MH * 2;
  q.W2 = q.b1 + MH;
  q.b2 = q.W2 + MH * MH;
  q.W3 = q.b2 + MH;
  q.b3 = q.W3 + (m + 1) * MH;
  return q;
}

__global__ __launch_bounds__(64) void k_meta_forward(PlanDev p, int m, const float* __restrict__ P,
                                                     float* __restrict__ omega, float* __restrict__ alpha) {
  __shared__ float h1s[MH], h2s[MH];
  const int b = blockIdx.x, j = threadIdx.x;
  const MetaPtrs q = meta_ptrs(P, m);
  const float x0 = p.mu[2 * b], x1 = p.mu[2 * b + 1];
  const float h1 = tanhf(fmadd(q.W1[2 * j + 1], x1, fmadd(q.W1[2 * j], x0, q.b1[j])));
  h1s[j] = h1;
  __syncthreads();
  float acc = q.b2[j];
  for (int k = 0; k < MH; ++k) acc = fmadd(q.W2[j * MH + k], h1s[k], acc);
  h2s[j] = tanhf(acc);
  __syncthreads();
  const float G = p.gersh[b];
  for (int o = j; o <= m; o += 64) {
    float z = q.b3[o];
    for (int k = 0; k < MH; ++k) z = fmadd(q.W3[o * MH + k], h2s[k], z);
    if (o < m) {
      omega[b * m + o] = expf(z) / G;
    } else {
      const float beta = 1.0f / (1.0f + expf(-z));
      for (int t = 0; t < m; ++t) alpha[b * m + t] = beta;
    }
  }
}

__global__ __launch_bounds__(64) void k_meta_backward(PlanDev p, int m, const float* __restrict__ P,
                                                      const float* __restrict__ d_omega,
                                                      const float* __restrict__ d_alpha,
                                                      float* __restrict__ per_inst, int np) {
  __shared__ float h1s[MH], h2s[MH], dzs[65], da2s[MH];
  const int b = blockIdx.x, j = threadIdx.x;
  const MetaPtrs q = meta_ptrs(P, m);
  const float x0 = p.mu[2 * b], x1 = p.mu[2 * b + 1];
  const float h1 = tanhf(fmadd(q.W1[2 * j + 1], x1, fmadd(q.W1[2 * j], x0, q.b1[j])));
  h1s[j] = h1;
  __syncthreads();
  float acc = q.b2[j];
  for (int k = 0; k < MH; ++k) acc = fmadd(q.W2[j * MH + k], h1s[k], acc);
  const float h2 = tanhf(acc);
  h2s[j] = h2;
  __syncthreads();
  const float G = p.gersh[b];
  for (int o = j; o <= m; o += 64) {
    float z = q.b3[o];
    for (int k = 0; k < MH; ++k) z = fmadd(q.W3[o * MH + k], h2s[k], z);
    if (o < m) {
      dzs[o] = d_omega[b * m + o] * (expf(z) / G);
    } else {
      const float beta = 1.0f / (1.0f + expf(-z));
      float s = 0.0f;
      for (int t = 0; t < m; ++t) s += d_alpha[b * m + t];
      dzs[m] = s * beta * (1.0f - beta);
    }
  }
  __syncthreads();
  float* g = per_inst + (int64_t)b * np;
  float* gW1 = g;
  float* gb1 = gW1 + MH * 2;
  float* gW2 = gb1 + MH;
  float* gb2 = gW2 + MH * MH;
  float* gW3 = gb2 + MH;
  float* gb3 = gW3 + (m + 1) * MH;
  for (int o = 0; o <= m; ++o) gW3[o * MH + j] = dzs[o] * h2s[j];
  for (int o = j; o <= m; o += 64) gb3[o] = dzs[o];
  float dh2 = 0.0f;
  for (int o = 0; o <= m; ++o) dh2 = fmadd(dzs[o], q.W3[o * MH + j], dh2);
  const float da2 = dh2 * (1.0f - h2 * h2);
  da2s[j] = da2;
  __syncthreads();
  for (int jj = 0; jj < MH; ++jj) gW2[jj * MH + j] = da2s[jj] * h1s[j];
  gb2[j] = da2;
  float dh1 = 0.0f;
  for (int jj = 0; jj < MH; ++jj) dh1 = fmadd(da2s[jj], q.W2[jj * MH + j], dh1);
  const float da1 = dh1 * (1.0f - h1 * h1);
  gW1[2 * j] = da1 * x0;
  gW1[2 * j + 1] = da1 * x1;
  gb1[j] = da1;
}

__global__ void k_meta_reduce(int B, int np, const float* __restrict__ per_inst, float* __restrict__ d_params) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= np) return;
  double acc = 0.0;
  for (int b = 0; b < B; ++b) acc += (double)per_inst[(int64_t)b * np + k];
  d_params[k] = (float)acc;
}

inline int fill_grid(int64_t count) {
  int64_t g = (count + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T>
void launch_apply(const PlanDev& p, const Tile* tiles, int ntiles, const T* x, T* y, hipStream_t st) {
  hipLaunchKernelGGL((k_apply<T, 0>), dim3(ntiles), dim3(WG), 0, st, p, tiles, (const T*)nullptr, x, y,
                     (double*)nullptr, (const int*)nullptr);
}
template <typename T>
void launch_residual(const PlanDev& p, const Tile* tiles, int ntiles, const T* b, const T* x, T* r,
                     double* partial2, const int* active, hipStream_t st) {
  hipLaunchKernelGGL((k_apply<T, 1>), dim3(ntiles), dim3(WG), 0, st, p, tiles, b, x, r, partial2, active);
}
template <typename T>
void launch_step(int method, const PlanDev& p, const Tile* tiles, int ntiles, const float* omega,
                 const float* alpha, int m, int i, const T* f, const T* u, const T* v, T* u_out, T* v_out,
                 const int* active, hipStream_t st) {
#define RM_STEP(MM)                                                                                           \
  hipLaunchKernelGGL((k_step<T, MM>), dim3(ntiles), dim3(WG), 0, st, p, tiles, omega, alpha, m, i, f, u, v, \
                     u_out, v_out, active)
  switch (method) {
    case M_NAG: RM_STEP(M_NAG); break;
    case M_MOM: RM_STEP(M_MOM); break;
    case M_NAGEX: RM_STEP(M_NAGEX); break;
    default: RM_STEP(M_RICH); break;
  }
#undef RM_STEP
}

template void launch_apply<float>(const PlanDev&, const Tile*, int, const float*, float*, hipStream_t);
template void launch_apply<double>(const PlanDev&, const Tile*, int, const double*, double*, hipStream_t);
template void launch_residual<float>(const PlanDev&, const Tile*, int, const float*, const float*, float*,
                                     double*, const int*, hipStream_t);
template void launch_residual<double>(const PlanDev&, const Tile*, int, const double*, const double*,
                                      double*, double*, const int*, hipStream_t);
template void launch_step<float>(int, const PlanDev&, const Tile*, int, const float*, const float*, int, int,
                                 const float*, const float*, const float*, float*, float*, const int*,
                                 hipStream_t);
template void launch_step<double>(int, const PlanDev&, const Tile*, int, const float*, const float*, int, int,
                                  const double*, const double*, const double*, double*, double*, const int*,
                                  hipStream_t);

void launch_reduce_partials(const PlanDev& p, const double* partial2, double* out0, double* out1, int stride,
                            float* ratio, hipStream_t st, const int* ranges) {
  hipLaunchKernelGGL(k_reduce_partials, dim3(p.B), dim3(64), 0, st, p, partial2, ranges, out0, out1, stride, ratio);
}

void launch_refine_residual(const PlanDev& p, const double* b, const double* x, float* r32, float* d, float* v,
                            double* partial2, const int* round_mask, hipStream_t st) {
  hipLaunchKernelGGL(k_refine_residual, dim3(p.ntiles), dim3(WG), 0, st, p, b, x, r32, d, v, partial2,
                     round_mask);
}

void launch_refine_update(const PlanDev& p, double* x, const float* d0, const float* d1, const int* start,
                          const int* outer_count, int flips, const int* round_mask, hipStream_t st) {
  hipLaunchKernelGGL(k_refine_update, dim3(p.ntiles), dim3(WG), 0, st, p, x, d0, d1, start, outer_count, flips,
                     round_mask);
}

void launch_round_decide(const PlanDev& p, const double* partial2, const RoundParams& rp, RoundState rs,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_round_decide, dim3(p.B), dim3(64), 0, st, p, partial2, rp, rs);
}

void launch_outer_flags(const PlanDev& p, const double* partial2, const int* ranges, const int* tranges,
                        const int* cls, unsigned long long tailmask, int ncls, double* res2, const double* rhs2,
                        const double* target2, double* best2, int* since, int* gains, int stall_min, int stall_max,
                        int cap, int* active, int* outer_count, int* status, int* pending, int* n_active,
                        unsigned long long* host_word, unsigned long long* host_cnt, unsigned seq,
                        const int* tot, double* hist, int hist_len, hipStream_t st) {
  if (p.B > 0)
    hipLaunchKernelGGL(k_outer_sums, dim3(p.B), dim3(64), 0, st, p, partial2, ranges, tranges, cls, tailmask, res2);
  const int threads = 64 * std::min(16, std::max(1, (p.B + 63) / 64));
  hipLaunchKernelGGL(k_outer_flags, dim3(1), dim3(threads), (size_t)std::max(1, ncls) * sizeof(int), st, p, cls,
                     ncls, res2, rhs2, target2, best2, since, gains, stall_min, stall_max, cap, active, outer_count,
                     status, pending, n_active, host_word, host_cnt, seq, tot, hist, hist_len);
}

void launch_fill_i32(int* p, int value, int64_t count, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_fill<int>, dim3(fill_grid(count)), dim3(256), 0, st, p, value, count);
}
void launch_fill_f32(float* p, float value, int64_t count, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_fill<float>, dim3(fill_grid(count)), dim3(256), 0, st, p, value, count);
}
void launch_fill_f64(double* p, double value, int64_t count, hipStream_t st) {
  if (count > 0)
    hipLaunchKernelGGL(k_fill<double>, dim3(fill_grid(count)), dim3(256), 0, st, p, value, count);
}
void launch_f64_to_f32(const double* src, float* dst, int64_t count, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_f64_to_f32, dim3(fill_grid(count)), dim3(256), 0, st, src, dst, count);
}

void launch_adj_terminal(const PlanDev& p, const float* b, const float* rK, const double* r2b2,
                         const float* g_loss, float* ub, float* fb, float* loss, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_terminal, dim3(p.ntiles), dim3(WG), 0, st, p, b, rK, r2b2, g_loss, ub, fb, loss);
}

void launch_adj_step(int method, const PlanDev& p, const float* omega, const float* alpha, int m, int i,
                     const float* f, const float* u, const float* v, const float* ub, const float* vb,
                     float* ub_out, float* vb_out, float* fb, double* partial4, hipStream_t st) {
#define RM_ADJ(MM)                                                                                                \
  hipLaunchKernelGGL(k_adj_step<MM>, dim3(p.ntiles), dim3(WG), 0, st, p, omega, alpha, m, i, f, u, v, ub, vb, \
                     ub_out, vb_out, fb, partial4)
  switch (method) {
    case M_NAG: RM_ADJ(M_NAG); break;
    case M_MOM: RM_ADJ(M_MOM); break;
    case M_NAGEX: RM_ADJ(M_NAGEX); break;
    default: RM_ADJ(M_RICH); break;
  }
#undef RM_ADJ
}

void launch_adj_accumulate(int method, const PlanDev& p, const double* partial4, int nslot, int E, int s_first,
                           int m, double* acc_w, double* acc_a, hipStream_t st, const int* ranges) {
#define RM_ACC(MM)                                                                                                \
  hipLaunchKernelGGL(k_adj_accumulate<MM>, dim3(p.B), dim3(64), 0, st, p, partial4, nslot, E, s_first, m, acc_w, \
                     acc_a, ranges)
  switch (method) {
    case M_NAG: RM_ACC(M_NAG); break;
    case M_MOM: RM_ACC(M_MOM); break;
    case M_NAGEX: RM_ACC(M_NAGEX); break;
    default: RM_ACC(M_RICH); break;
  }
#undef RM_ACC
}

void launch_meta_forward(const PlanDev& p, int m, const float* params, float* omega, float* alpha,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_meta_forward, dim3(p.B), dim3(64), 0, st, p, m, params, omega, alpha);
}

void launch_meta_backward(const PlanDev& p, int m, const float* params, const float* d_omega,
                          const float* d_alpha, float* per_inst, float* d_params, hipStream_t st) {
  const int np = MH * 2 + MH + MH * MH + MH + (m + 1) * MH + (m + 1);
  hipLaunchKernelGGL(k_meta_backward, dim3(p.B), dim3(64), 0, st, p, m, params, d_omega, d_alpha, per_inst,
                     np);
  hipLaunchKernelGGL(k_meta_reduce, dim3((np + 255) / 256), dim3(256), 0, st, p.B, np, per_inst, d_params);
}

}  // namespace rmk
