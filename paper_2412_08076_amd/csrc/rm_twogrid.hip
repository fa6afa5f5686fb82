// Two-grid correction of the Helmholtz multilevel variant (arXiv 2412.08076 §3,
// eqs. dl-him-b and dl-him-h): after the smoothing steps of a Table-1 scheme,
//   u += P S (symbol * (S R (f - A u) S)) S
// with R full weighting onto the coarse grid (n = 2 nc + 1, coarse point (I, J) on
// fine point (2I + 1, 2J + 1)), P bilinear interpolation (P = 4 R^T), and S the
// orthonormal DST-I of the coarse grid, which diagonalises every constant-
// coefficient Dirichlet operator there.  The symbol is per instance, [q][p]
// (row = y mode), like the grid.
//
// Kernels (FP32 fields; the residual behind the correction in FP64):
//   k_tg_restrict  residual of a fine tile (in FP64) from an LDS-staged iterate,
//                  then full weighting (or the weighting of a plain vector, for
//                  P^T = 4 R in the adjoint);
//   k_tg_dst       DST-I along the rows of a coarse field through a radix-2 FFT in
//                  LDS of the odd extension of length M = n + 1, two real rows per
//                  complex FFT.  Pass A transforms along x and writes transposed,
//                  pass B transforms along y, applies the symbol (and in the
//                  adjoint accumulates its gradient) and transforms back in LDS,
//                  pass C transforms along x reading transposed;
//   k_tg_prolong   bilinear interpolation added to u;
//   k_tg_adj_correct  the adjoint on the fine grid: R^T ybar = P ybar / 4 formed in
//                  LDS, ub - A R^T ybar with the stencil summed in FP64, and the
//                  right-hand-side gradient.
// The coarse fields are a few percent of the fine traffic.  A transform pass runs
// about four workgroups per CU, all resident at once, so it lasts one workgroup's
// chain of dependent steps (row loads, FFT stages between barriers, stores).
#include "rm_device.h"

#pragma clang fp contract(off)

namespace rmk {

namespace {

// restriction tile: RT_X x RT_Y coarse points; the residual window around it is
// (2 RT_X + 1) x (2 RT_Y + 1) fine points and needs u on one more ring
constexpr int RT_X = 64, RT_Y = 8;
constexpr int RR_W = 2 * RT_X + 1, RR_H = 2 * RT_Y + 1;
constexpr int RU_W = RR_W + 2, RU_H = RR_H + 2;

// The residual is formed in FP64 from the FP32 iterate: on a smooth, large u the
// terms of f - A u cancel, and FP32 rounding there would be amplified by the symbol
// on the low modes (to ~1e-4 relative at n = 255).  Once formed, the residual is
// rounded to FP32 (relative error eps |r|, harmless) for the full weighting.
template <int MODE>  // 0: rc = scale R (f - A u);  1: rc = scale R u
__global__ __launch_bounds__(WG) void k_tg_restrict(PlanDev p, TgDev g, const Tile* __restrict__ tiles,
                                                    const float* __restrict__ f, const float* __restrict__ u,
                                                    float* __restrict__ rc, float scale) {
  __shared__ float su[MODE == 0 ? RU_H * RU_W : 1];
  __shared__ float sr[RR_H * RR_W];
  const Tile t = tiles[xcd_remap(blockIdx.x, gridDim.x)];
  if (t.inst < 0) return;
  const Inst in = p.inst[t.inst];
  const TgInst gi = g.inst[t.inst];
  const int n = in.n, nc = gi.nc;
  const int fx0 = 2 * t.x0, fy0 = 2 * t.y0;  // fine origin of the residual window
  const Field<float> uf(u + in.off, n * n);
  if (MODE == 0) {
    double c[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) c[k] = p.coef64[t.inst * 8 + k];
    stage<float, RU_W, RU_H, false>(
        fx0 - 1, fy0 - 1, n, [&](unsigned idx) { return uf[idx]; }, [&](int k, int, int, float v) { su[k] = v; });
    __syncthreads();
    const Field<float> fi(f + in.off, n * n);
    constexpr int NR = (RR_H * RR_W + WG - 1) / WG;
    float fv[NR];
    const int t0 = opaque_tid();
#pragma unroll
    for (int j = 0; j < NR; ++j) {   // points off the field read f at 0
      const int k = t0 + j * WG;
      const int ly = k / RR_W, lx = k - ly * RR_W;
      const int gx = fx0 + lx, gy = fy0 + ly;
      fv[j] = fi[(gx < n && gy < n) ? (unsigned)(gy * n + gx) : 0u];
    }
    const int t1 = opaque_tid();
#pragma unroll
    for (int j = 0; j < NR; ++j) {
      const int k = t1 + j * WG;
      const int ly = k / RR_W, lx = k - ly * RR_W;
      const int gx = fx0 + lx, gy = fy0 + ly;
      const bool ok = k < RR_H * RR_W && gx < n && gy < n;
      // points not formed read the stencil at the window's first interior point
      const float* s = su + (ok ? (ly + 1) * RU_W + (lx + 1) : RU_W + 1);
      double acc = c[0] * (double)s[0];
      acc = __builtin_fma(c[1], (double)s[-1] + (double)s[1], acc);
      acc = __builtin_fma(c[2], (double)s[-RU_W] + (double)s[RU_W], acc);
      acc = __builtin_fma(c[3], (double)s[-RU_W - 1] + (double)s[RU_W + 1], acc);
      acc = __builtin_fma(c[4], (double)s[-RU_W + 1] + (double)s[RU_W - 1], acc);
      asm volatile("" : "+v"(acc)::"memory");   // one stencil's LDS reads in flight at a time
      if (k < RR_H * RR_W) sr[k] = ok ? (float)((double)fv[j] - acc) : 0.f;
    }
  } else {
    stage<float, RR_W, RR_H, false>(
        fx0, fy0, n, [&](unsigned idx) { return uf[idx]; }, [&](int k, int, int, float v) { sr[k] = v; });
  }
  __syncthreads();
  const float w = scale * 0.0625f;  // (1/16) [1 2 1; 2 4 2; 1 2 1]
  const int tx = threadIdx.x & 63;
  for (int ty = threadIdx.x >> 6; ty < RT_Y; ty += WG / 64) {
    const int I = t.x0 + tx, J = t.y0 + ty;
    if (I < nc && J < nc) {
      const float* s = sr + (2 * ty + 1) * RR_W + 2 * tx + 1;
      float acc = (s[-RR_W - 1] + s[-RR_W + 1]) + (s[RR_W - 1] + s[RR_W + 1]);
      acc = fmadd(2.f, (s[-1] + s[1]) + (s[-RR_W] + s[RR_W]), acc);
      acc = fmadd(4.f, s[0], acc);
      rc[gi.coff + (int64_t)J * nc + I] = acc * w;
    }
  }
}

// ---------------------------------------------------------------------------
// DST-I through the FFT of the odd extension.  For real rows a, b of length nc
// (M = 2 (nc + 1)) the complex sequence z_t = a_{t-1} + i b_{t-1} (t = 1..nc),
// z_0 = z_{M/2} = 0, z_{M-t} = -z_t has the transform Z_k = 2 Xb_k - 2i Xa_k with
// X the unnormalised DST-I; the orthonormal coefficients are -Im Z_k / sqrt(M)
// (row a) and Re Z_k / sqrt(M) (row b), k = 1..nc.
// ---------------------------------------------------------------------------
constexpr int DG = 8;          // rows per workgroup
constexpr int DPAIR = DG / 2;  // complex FFTs per workgroup
constexpr int DMAX = kTgMaxFFT;
constexpr int DITEMS = DG * (DMAX / 2) / WG;  // coefficients per thread (pass B repack)

__device__ __forceinline__ int bitrev(int t, int lg) { return (int)(__builtin_bitreverse32((unsigned)t) >> (32 - lg)); }

__device__ __forceinline__ float2 cmul(float2 w, float2 x) {
  return make_float2(fmadd(w.x, x.x, -(w.y * x.y)), fmadd(w.x, x.y, w.y * x.x));
}

// S consecutive radix-2 stages l .. l + S - 1 of an in-place decimation-in-time FFT,
// each thread taking 2^S points (stride h = 2^(l-1)) through all S stages in
// registers.  Stage l + s joins pairs at distance 2^s h with the twiddle
// exp(-2 pi i p / 2^(l+s)) of the pair's position p; the first stage of the
// transform (twiddle 1) adds and subtracts without a product.
template <int S>
__device__ __forceinline__ void fft_stages(float2* z, int M, int lg, int l, const float2* tws) {
  constexpr int R = 1 << S;
  const int h = 1 << (l - 1);
  for (int bi = threadIdx.x; bi < DPAIR * (M >> S); bi += WG) {
    const int q = bi >> (lg - S);
    const int b = bi & ((M >> S) - 1);
    const int pos = b & (h - 1);
    const int i0 = q * M + ((b >> (l - 1)) << (l - 1 + S)) + pos;
    float2 a[R];
#pragma unroll
    for (int j = 0; j < R; ++j) a[j] = z[i0 + j * h];
#pragma unroll
    for (int st = 0; st < S; ++st) {
      const int hs = 1 << st;
#pragma unroll
      for (int j0 = 0; j0 < R; j0 += 2 * hs)
#pragma unroll
        for (int mm = 0; mm < hs; ++mm) {
          const float2 e = a[j0 + mm], o = a[j0 + mm + hs];
          const float2 t = (l + st == 1) ? o : cmul(tws[(pos + mm * h) * (M >> (l + st))], o);
          a[j0 + mm] = make_float2(e.x + t.x, e.y + t.y);
          a[j0 + mm + hs] = make_float2(e.x - t.x, e.y - t.y);
        }
    }
#pragma unroll
    for (int j = 0; j < R; ++j) z[i0 + j * h] = a[j];
  }
  __syncthreads();
}

// In-place decimation-in-time FFT of DPAIR sequences of length M = 2^lg stored back
// to back in z, input in bit-reversed order, output in natural order, tws[k] =
// exp(-2 pi i k / M).  The stages go three at a time through registers (one LDS round
// trip per three stages), after one or two first stages when 3 does not divide lg.
__device__ __forceinline__ void fft_pairs(float2* z, int M, int lg, const float2* tws) {
  int l = 1;
  if (lg % 3 == 1) {
    fft_stages<1>(z, M, lg, l, tws);
    l += 1;
  } else if (lg % 3 == 2) {
    fft_stages<2>(z, M, lg, l, tws);
    l += 2;
  }
  for (; l < lg; l += 3) fft_stages<3>(z, M, lg, l, tws);
}

// Place value x of row rr (0..DG-1), position t (1..nc) into the odd extension
// (bit-reversed order).
__device__ __forceinline__ void put_odd(float2* z, int M, int lg, int rr, int t, float x) {
  float* zz = reinterpret_cast<float*>(z);
  const int q = rr >> 1, comp = rr & 1;
  zz[2 * (q * M + bitrev(t, lg)) + comp] = x;
  zz[2 * (q * M + bitrev(M - t, lg)) + comp] = -x;
}

__device__ __forceinline__ void zero_ends(float2* z, int M, int lg) {
  for (int q = threadIdx.x; q < DPAIR; q += WG) {
    z[q * M + 0] = make_float2(0.f, 0.f);                   // t = 0
    z[q * M + bitrev(M >> 1, lg)] = make_float2(0.f, 0.f);  // t = M / 2
  }
}

// Orthonormal coefficient k (1..nc) of row rr after the FFT.
__device__ __forceinline__ float coeff(const float2* z, int M, int rr, int k, float sc) {
  const float2 v = z[(rr >> 1) * M + k];
  return (rr & 1) ? v.x * sc : -v.y * sc;
}

// MODE 0 (A): rows J of in[J][I] -> out[p][J] (transform along I, transposed write)
// MODE 1 (B): rows p of in[p][J] -> transform along J to [p][q]; then
//             shat_out given: store [p][q] and stop;
//             dsym given:     dsym[q][p] += coef[p][q] * shat[p][q];
//             symbol given:   coef[p][q] *= symbol[q][p];
//             transform back along q -> out[p][J]
// MODE 2 (C): rows J gathered from in[p][J] -> out[J][I] (transform along p)
// Dynamic LDS: DPAIR * Mmax sequences plus Mmax / 2 twiddles (float2), Mmax the
// largest n + 1 of the launch.
template <int MODE>
__global__ __launch_bounds__(WG) void k_tg_dst(TgDev g, const Tile* __restrict__ groups, int mmax, const float* in,
                                               float* out, const float* __restrict__ symbol,
                                               const float* __restrict__ shat, float* __restrict__ shat_out,
                                               float* __restrict__ dsym) {
  extern __shared__ float2 lds[];
  float2* z = lds;
  float2* tws = lds + DPAIR * mmax;
  const Tile t = groups[blockIdx.x];
  if (t.inst < 0) return;
  const TgInst gi = g.inst[t.inst];
  const int nc = gi.nc, lg = gi.lg, M = 1 << lg;
  const float sc = gi.scale;
  const int r0 = t.y0;
  const float* src = in + gi.coff;
  float* dst = out + gi.coff;
  for (int k = threadIdx.x; k < (M >> 1); k += WG) tws[k] = g.tw[k * (DMAX / M)];
  // load the group's rows into the odd extensions
  if (MODE == 2) {
    for (int idx = threadIdx.x; idx < DG * nc; idx += WG) {
      const int rr = idx & (DG - 1), c = idx >> 3;
      const int r = r0 + rr;
      put_odd(z, M, lg, rr, c + 1, r < nc ? src[(int64_t)c * nc + r] : 0.f);
    }
  } else {
    for (int rr = 0; rr < DG; ++rr) {
      const int r = r0 + rr;
      for (int c = threadIdx.x; c < nc; c += WG) put_odd(z, M, lg, rr, c + 1, r < nc ? src[(int64_t)r * nc + c] : 0.f);
    }
  }
  zero_ends(z, M, lg);
  __syncthreads();
  fft_pairs(z, M, lg, tws);
  if (MODE == 0) {
    for (int idx = threadIdx.x; idx < DG * nc; idx += WG) {
      const int rr = idx & (DG - 1), k = idx >> 3;
      const int r = r0 + rr;
      if (r < nc) dst[(int64_t)k * nc + r] = coeff(z, M, rr, k + 1, sc);
    }
    return;
  }
  if (MODE == 2) {
    for (int rr = 0; rr < DG; ++rr) {
      const int r = r0 + rr;
      if (r >= nc) break;
      for (int k = threadIdx.x; k < nc; k += WG) dst[(int64_t)r * nc + k] = coeff(z, M, rr, k + 1, sc);
    }
    return;
  }
  // MODE 1: coefficients [p = r0 + rr][q = k]
  if (shat_out != nullptr) {
    for (int rr = 0; rr < DG; ++rr) {
      const int r = r0 + rr;
      if (r >= nc) break;
      for (int k = threadIdx.x; k < nc; k += WG) shat_out[gi.coff + (int64_t)r * nc + k] = coeff(z, M, rr, k + 1, sc);
    }
    return;
  }
  // gather this thread's coefficients, apply the symbol, then rebuild the odd
  // extensions for the inverse transform (all reads happen before the barrier)
  float vals[DITEMS];
#pragma unroll
  for (int j = 0; j < DITEMS; ++j) {
    const int idx = threadIdx.x + j * WG;
    const int rr = idx & (DG - 1), k = idx >> 3;
    const int r = r0 + rr;
    float x = 0.f;
    if (k < nc && r < nc) {
      x = coeff(z, M, rr, k + 1, sc);
      const int64_t qp = gi.coff + (int64_t)k * nc + r;  // [q][p]
      if (dsym != nullptr) dsym[qp] = fmadd(x, shat[gi.coff + (int64_t)r * nc + k], dsym[qp]);
      if (symbol != nullptr) x = x * symbol[qp];
    }
    vals[j] = x;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < DITEMS; ++j) {
    const int idx = threadIdx.x + j * WG;
    const int rr = idx & (DG - 1), k = idx >> 3;
    if (k < nc) put_odd(z, M, lg, rr, k + 1, vals[j]);
  }
  zero_ends(z, M, lg);
  __syncthreads();
  fft_pairs(z, M, lg, tws);
  for (int rr = 0; rr < DG; ++rr) {
    const int r = r0 + rr;
    if (r >= nc) break;
    for (int k = threadIdx.x; k < nc; k += WG) dst[(int64_t)r * nc + k] = coeff(z, M, rr, k + 1, sc);
  }
}

// Coarse window of a fine tile at (x0, y0) (both even): coarse columns from
// x0/2 - 2 and rows from y0/2 - 2, zero outside the coarse grid.  It covers the
// bilinear interpolation of the tile and its one-point halo.
constexpr int CW_W = TX / 2 + 4, CW_H = TY / 2 + 4;

__device__ __forceinline__ void stage_coarse(float* cw, const float* e, int nc, int x0, int y0) {
  const Field<float> ef(e, nc * nc);
  stage<float, CW_W, CW_H, false>(
      x0 / 2 - 2, y0 / 2 - 2, nc, [&](unsigned idx) { return ef[idx]; }, [&](int k, int, int, float v) { cw[k] = v; });
}

// Bilinear interpolation at fine point (i, j) from the window: along each axis an
// odd index sits on coarse (i - 1) / 2, an even one halfway between i/2 - 1 and i/2.
__device__ __forceinline__ float interp(const float* cw, int x0, int y0, int i, int j) {
  const int I0 = x0 / 2 - 2, J0 = y0 / 2 - 2;
  auto row = [&](int J) -> float {
    const float* r = cw + (J - J0) * CW_W - I0;
    if (i & 1) return r[(i - 1) >> 1];
    return 0.5f * (r[(i >> 1) - 1] + r[i >> 1]);
  };
  if (j & 1) return row((j - 1) >> 1);
  return 0.5f * (row((j >> 1) - 1) + row(j >> 1));
}

// uo = ui + P ec (uo may equal ui)
__global__ __launch_bounds__(WG) void k_tg_prolong(PlanDev p, TgDev g, const float* __restrict__ ec,
                                                   const float* ui, float* uo) {
  __shared__ float cw[CW_W * CW_H];
  const Tile tl = p.tiles[xcd_remap(blockIdx.x, gridDim.x)];
  if (tl.inst < 0) return;
  const Inst in = p.inst[tl.inst];
  const TgInst gi = g.inst[tl.inst];
  const int n = in.n;
  stage_coarse(cw, ec + gi.coff, gi.nc, tl.x0, tl.y0);
  __syncthreads();
  const int i = tl.x0 + (threadIdx.x & 63);
  if (i >= n) return;
  const int ty0 = threadIdx.x >> 6;
  constexpr int NY = TY / (WG / 64);
  const Field<float> uif(ui + in.off, n * n), uof(uo + in.off, n * n);
  float uv[NY];
#pragma unroll
  for (int k = 0; k < NY; ++k) uv[k] = uif[(unsigned)(min(tl.y0 + ty0 + 4 * k, n - 1) * n + i)];
#pragma unroll
  for (int k = 0; k < NY; ++k) {   // rows below the field are dropped by the store
    const int j = tl.y0 + ty0 + 4 * k;
    uof.store((unsigned)(j * n + i), uv[k] + interp(cw, tl.x0, tl.y0, i, min(j, n - 1)));
  }
}

// Adjoint of the correction on the fine grid: rb = R^T ybar = P ybar / 4 is formed in
// LDS on the tile and its one-point halo, then ub_out = ub - A rb with the stencil
// summed in FP64 (rb carries the symbol-amplified low modes, and the terms of A rb
// cancel against ub there) and fb += rb on the owned points (fb may be null).
constexpr int AW = TX + 2;
__global__ __launch_bounds__(WG) void k_tg_adj_correct(PlanDev p, TgDev g, const float* __restrict__ ybar,
                                                       const float* __restrict__ ub, float* __restrict__ ub_out,
                                                       float* __restrict__ fb) {
  __shared__ float cw[CW_W * CW_H];
  __shared__ float s[(TY + 2) * AW];
  const Tile tl = p.tiles[xcd_remap(blockIdx.x, gridDim.x)];
  if (tl.inst < 0) return;
  const Inst in = p.inst[tl.inst];
  const TgInst gi = g.inst[tl.inst];
  const int n = in.n;
  stage_coarse(cw, ybar + gi.coff, gi.nc, tl.x0, tl.y0);
  __syncthreads();
  for (int k = threadIdx.x; k < (TY + 2) * AW; k += WG) {
    const int ly = k / AW, lx = k - ly * AW;
    const int gx = tl.x0 + lx - 1, gy = tl.y0 + ly - 1;
    s[k] = (gx >= 0 && gx < n && gy >= 0 && gy < n) ? 0.25f * interp(cw, tl.x0, tl.y0, gx, gy) : 0.f;
  }
  __syncthreads();
  double c[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) c[k] = p.coef64[tl.inst * 8 + k];
  const int tx = threadIdx.x & 63, ty0 = threadIdx.x >> 6;
  const int gx = tl.x0 + tx;
  if (gx >= n) return;
  constexpr int NY = TY / (WG / 64);
  const Field<float> ubf(ub + in.off, n * n), fbf(fb != nullptr ? fb + in.off : ub + in.off, n * n);
  float ubv[NY], fbv[NY];
#pragma unroll
  for (int k = 0; k < NY; ++k) {   // rows below the field load its last row
    const unsigned idx = (unsigned)(min(tl.y0 + ty0 + 4 * k, n - 1) * n + gx);
    ubv[k] = ubf[idx];
    fbv[k] = fb != nullptr ? fbf[idx] : 0.f;
  }
#pragma unroll
  for (int k = 0; k < NY; ++k) {
    const int ly = ty0 + 4 * k, gy = tl.y0 + ly;
    if (gy >= n) break;
    const float* q = s + (ly + 1) * AW + tx + 1;
    double acc = c[0] * (double)q[0];
    acc = __builtin_fma(c[1], (double)q[-1] + (double)q[1], acc);
    acc = __builtin_fma(c[2], (double)q[-AW] + (double)q[AW], acc);
    acc = __builtin_fma(c[3], (double)q[-AW - 1] + (double)q[AW + 1], acc);
    acc = __builtin_fma(c[4], (double)q[-AW + 1] + (double)q[AW - 1], acc);
    const int64_t idx = in.off + (int64_t)gy * n + gx;
    ub_out[idx] = (float)((double)ubv[k] - acc);
    if (fb != nullptr) fb[idx] = fbv[k] + q[0];
  }
}

}  // namespace

// ---- launchers --------------------------------------------------------------
void launch_tg_restrict(int mode, const PlanDev& p, const TgDev& g, const Tile* tiles, int ntiles, const float* f,
                        const float* u, float* rc, float scale, hipStream_t st) {
  if (mode == 0)
    hipLaunchKernelGGL((k_tg_restrict<0>), dim3(ntiles), dim3(WG), 0, st, p, g, tiles, f, u, rc, scale);
  else
    hipLaunchKernelGGL((k_tg_restrict<1>), dim3(ntiles), dim3(WG), 0, st, p, g, tiles, f, u, rc, scale);
}

void launch_tg_dst(int pass, const TgDev& g, const Tile* groups, int ngroups, int mmax, const float* in, float* out,
                   const float* symbol, const float* shat, float* shat_out, float* dsym, hipStream_t st) {
  const size_t lds = (size_t)(DPAIR * mmax + mmax / 2) * sizeof(float2);
  if (pass == 0)
    hipLaunchKernelGGL((k_tg_dst<0>), dim3(ngroups), dim3(WG), lds, st, g, groups, mmax, in, out, symbol, shat,
                       shat_out, dsym);
  else if (pass == 1)
    hipLaunchKernelGGL((k_tg_dst<1>), dim3(ngroups), dim3(WG), lds, st, g, groups, mmax, in, out, symbol, shat,
                       shat_out, dsym);
  else
    hipLaunchKernelGGL((k_tg_dst<2>), dim3(ngroups), dim3(WG), lds, st, g, groups, mmax, in, out, symbol, shat,
                       shat_out, dsym);
}

void launch_tg_prolong(const PlanDev& p, const TgDev& g, const float* ec, const float* ui, float* uo,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_tg_prolong, dim3(p.ntiles), dim3(WG), 0, st, p, g, ec, ui, uo);
}

void launch_tg_adj_correct(const PlanDev& p, const TgDev& g, const float* ybar, const float* ub, float* ub_out,
                           float* fb, hipStream_t st) {
  hipLaunchKernelGGL(k_tg_adj_correct, dim3(p.ntiles), dim3(WG), 0, st, p, g, ybar, ub, ub_out, fb);
}

}  // namespace rmk
