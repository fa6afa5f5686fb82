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
// The coarse fields are a few percent of the fine traffic; the FFT stages are
// LDS-bound at these lengths.
#include "rm_internal.h"

#pragma clang fp contract(off)

namespace rmk {

namespace {

__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

__device__ __forceinline__ int xcd_remap(int bid, int nb) {
  const int per = nb >> 3;
  return (bid & 7) * per + (bid >> 3);
}

// restriction tile: RT_X x RT_Y coarse points; the residual window around it is
// (2 RT_X + 1) x (2 RT_Y + 1) fine points and needs u on one more ring
constexpr int RT_X = 64, RT_Y = 8;
constexpr int RR_W = 2 * RT_X + 1, RR_H = 2 * RT_Y + 1;
constexpr int RU_W = RR_W + 2, RU_H = RR_H + 2;

// The residual is formed in FP64 from the FP32 iterate: on a smooth, large u the
// terms of f - A u cancel, and FP32 rounding there would be amplified by the symbol
// on the low modes (to ~1e-4 relative at n = 255).  Full weighting is summed in FP64
// and rounded to FP32 once.
template <int MODE>  // 0: rc = scale R (f - A u);  1: rc = scale R u
__global__ __launch_bounds__(WG) void k_tg_restrict(PlanDev p, TgDev g, const Tile* __restrict__ tiles,
                                                    const float* __restrict__ f, const float* __restrict__ u,
                                                    float* __restrict__ rc, float scale) {
  __shared__ float su[MODE == 0 ? RU_H * RU_W : 1];
  __shared__ double sr[RR_H * RR_W];
  const Tile t = tiles[xcd_remap(blockIdx.x, gridDim.x)];
  if (t.inst < 0) return;
  const Inst in = p.inst[t.inst];
  const TgInst gi = g.inst[t.inst];
  const int n = in.n, nc = gi.nc;
  const int fx0 = 2 * t.x0, fy0 = 2 * t.y0;  // fine origin of the residual window
  const float* ui = u + in.off;
  if (MODE == 0) {
    double c[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) c[k] = p.coef64[t.inst * 8 + k];
    for (int k = threadIdx.x; k < RU_H * RU_W; k += WG) {
      const int ly = k / RU_W, lx = k - ly * RU_W;
      const int gx = fx0 - 1 + lx, gy = fy0 - 1 + ly;
      su[k] = (gx >= 0 && gx < n && gy >= 0 && gy < n) ? ui[(int64_t)gy * n + gx] : 0.f;
    }
    __syncthreads();
    const float* fi = f + in.off;
    for (int k = threadIdx.x; k < RR_H * RR_W; k += WG) {
      const int ly = k / RR_W, lx = k - ly * RR_W;
      const int gx = fx0 + lx, gy = fy0 + ly;
      double r = 0.0;
      if (gx < n && gy < n) {
        const float* s = su + (ly + 1) * RU_W + (lx + 1);
        double acc = c[0] * (double)s[0];
        acc = __builtin_fma(c[1], (double)s[-1] + (double)s[1], acc);
        acc = __builtin_fma(c[2], (double)s[-RU_W] + (double)s[RU_W], acc);
        acc = __builtin_fma(c[3], (double)s[-RU_W - 1] + (double)s[RU_W + 1], acc);
        acc = __builtin_fma(c[4], (double)s[-RU_W + 1] + (double)s[RU_W - 1], acc);
        r = (double)fi[(int64_t)gy * n + gx] - acc;
      }
      sr[k] = r;
    }
  } else {
    for (int k = threadIdx.x; k < RR_H * RR_W; k += WG) {
      const int ly = k / RR_W, lx = k - ly * RR_W;
      const int gx = fx0 + lx, gy = fy0 + ly;
      sr[k] = (gx < n && gy < n) ? (double)ui[(int64_t)gy * n + gx] : 0.0;
    }
  }
  __syncthreads();
  const double w = (double)scale * 0.0625;  // (1/16) [1 2 1; 2 4 2; 1 2 1]
  const int tx = threadIdx.x & 63;
  for (int ty = threadIdx.x >> 6; ty < RT_Y; ty += WG / 64) {
    const int I = t.x0 + tx, J = t.y0 + ty;
    if (I < nc && J < nc) {
      const double* s = sr + (2 * ty + 1) * RR_W + 2 * tx + 1;
      double acc = (s[-RR_W - 1] + s[-RR_W + 1]) + (s[RR_W - 1] + s[RR_W + 1]);
      acc = __builtin_fma(2.0, (s[-1] + s[1]) + (s[-RR_W] + s[RR_W]), acc);
      acc = __builtin_fma(4.0, s[0], acc);
      rc[gi.coff + (int64_t)J * nc + I] = (float)(acc * w);
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
constexpr int DG = 16;         // rows per workgroup
constexpr int DPAIR = DG / 2;  // complex FFTs per workgroup
constexpr int DMAX = kTgMaxFFT;
constexpr int DITEMS = DG * (DMAX / 2) / WG;  // coefficients per thread (pass B repack)

__device__ __forceinline__ int bitrev(int t, int lg) { return (int)(__builtin_bitreverse32((unsigned)t) >> (32 - lg)); }

// In-place radix-2 decimation-in-time FFT of DPAIR sequences of length M = 2^lg
// stored back to back in z, input in bit-reversed order, output in natural order.
// tw[k] = exp(-2 pi i k / DMAX), k < DMAX / 2.
__device__ __forceinline__ void fft_pairs(float2* z, int M, int lg, const float2* __restrict__ tw) {
  const int nb = DPAIR * (M >> 1);
  for (int l = 1; l <= lg; ++l) {
    const int half = 1 << (l - 1);
    const int tws = DMAX >> l;
    for (int bi = threadIdx.x; bi < nb; bi += WG) {
      const int q = bi >> (lg - 1);
      const int b = bi & ((M >> 1) - 1);
      const int pos = b & (half - 1);
      const int i0 = q * M + ((b >> (l - 1)) << l) + pos;
      const int i1 = i0 + half;
      const float2 w = tw[pos * tws];
      const float2 x1 = z[i1];
      const float2 x0 = z[i0];
      const float tr = fmadd(w.x, x1.x, -(w.y * x1.y));
      const float ti = fmadd(w.x, x1.y, w.y * x1.x);
      z[i0] = make_float2(x0.x + tr, x0.y + ti);
      z[i1] = make_float2(x0.x - tr, x0.y - ti);
    }
    __syncthreads();
  }
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
    z[q * M + 0] = make_float2(0.f, 0.f);            // t = 0
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
template <int MODE>
__global__ __launch_bounds__(WG) void k_tg_dst(TgDev g, const Tile* __restrict__ groups, const float* in,
                                               float* out, const float* __restrict__ symbol,
                                               const float* __restrict__ shat, float* __restrict__ shat_out,
                                               float* __restrict__ dsym) {
  __shared__ float2 z[DPAIR * DMAX];
  const Tile t = groups[blockIdx.x];
  if (t.inst < 0) return;
  const TgInst gi = g.inst[t.inst];
  const int nc = gi.nc, lg = gi.lg, M = 1 << lg;
  const float sc = gi.scale;
  const int r0 = t.y0;
  const float* src = in + gi.coff;
  float* dst = out + gi.coff;
  // load the group's rows into the odd extensions
  if (MODE == 2) {
    for (int idx = threadIdx.x; idx < DG * nc; idx += WG) {
      const int rr = idx & (DG - 1), c = idx >> 4;
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
  fft_pairs(z, M, lg, g.tw);
  if (MODE == 0) {
    for (int idx = threadIdx.x; idx < DG * nc; idx += WG) {
      const int rr = idx & (DG - 1), k = idx >> 4;
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
    const int rr = idx & (DG - 1), k = idx >> 4;
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
    const int rr = idx & (DG - 1), k = idx >> 4;
    if (k < nc) put_odd(z, M, lg, rr, k + 1, vals[j]);
  }
  zero_ends(z, M, lg);
  __syncthreads();
  fft_pairs(z, M, lg, g.tw);
  for (int rr = 0; rr < DG; ++rr) {
    const int r = r0 + rr;
    if (r >= nc) break;
    for (int k = threadIdx.x; k < nc; k += WG) dst[(int64_t)r * nc + k] = coeff(z, M, rr, k + 1, sc);
  }
}

// Bilinear interpolation of the coarse field e at fine point (i, j) (zero outside):
// along each axis an odd index sits on coarse (i - 1) / 2, an even one halfway between
// i/2 - 1 and i/2.
__device__ __forceinline__ float interp_row(const float* e, int nc, int J, int i) {
  auto at = [&](int I) { return (I >= 0 && I < nc) ? e[(int64_t)J * nc + I] : 0.f; };
  if (i & 1) return at((i - 1) >> 1);
  return 0.5f * (at((i >> 1) - 1) + at(i >> 1));
}

__device__ __forceinline__ float interp(const float* e, int nc, int i, int j) {
  if (j & 1) return interp_row(e, nc, (j - 1) >> 1, i);
  const int Ja = (j >> 1) - 1, Jb = j >> 1;
  const float a = Ja >= 0 ? interp_row(e, nc, Ja, i) : 0.f;
  const float b = Jb < nc ? interp_row(e, nc, Jb, i) : 0.f;
  return 0.5f * (a + b);
}

// uo = ui + P ec (uo may equal ui)
__global__ __launch_bounds__(WG) void k_tg_prolong(PlanDev p, TgDev g, const float* __restrict__ ec,
                                                   const float* ui, float* uo) {
  const Tile tl = p.tiles[xcd_remap(blockIdx.x, gridDim.x)];
  if (tl.inst < 0) return;
  const Inst in = p.inst[tl.inst];
  const TgInst gi = g.inst[tl.inst];
  const int n = in.n, nc = gi.nc;
  const float* e = ec + gi.coff;
  const int i = tl.x0 + (threadIdx.x & 63);
  if (i >= n) return;
  const int ty0 = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < TY / (WG / 64); ++k) {
    const int j = tl.y0 + ty0 + 4 * k;
    if (j >= n) break;
    const int64_t idx = in.off + (int64_t)j * n + i;
    uo[idx] = ui[idx] + interp(e, nc, i, j);
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
  __shared__ float s[(TY + 2) * AW];
  const Tile tl = p.tiles[xcd_remap(blockIdx.x, gridDim.x)];
  if (tl.inst < 0) return;
  const Inst in = p.inst[tl.inst];
  const TgInst gi = g.inst[tl.inst];
  const int n = in.n, nc = gi.nc;
  const float* e = ybar + gi.coff;
  for (int k = threadIdx.x; k < (TY + 2) * AW; k += WG) {
    const int ly = k / AW, lx = k - ly * AW;
    const int gx = tl.x0 + lx - 1, gy = tl.y0 + ly - 1;
    s[k] = (gx >= 0 && gx < n && gy >= 0 && gy < n) ? 0.25f * interp(e, nc, gx, gy) : 0.f;
  }
  __syncthreads();
  double c[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) c[k] = p.coef64[tl.inst * 8 + k];
  const int tx = threadIdx.x & 63, ty0 = threadIdx.x >> 6;
  const int gx = tl.x0 + tx;
  if (gx >= n) return;
#pragma unroll
  for (int k = 0; k < TY / (WG / 64); ++k) {
    const int ly = ty0 + 4 * k, gy = tl.y0 + ly;
    if (gy >= n) break;
    const float* q = s + (ly + 1) * AW + tx + 1;
    double acc = c[0] * (double)q[0];
    acc = __builtin_fma(c[1], (double)q[-1] + (double)q[1], acc);
    acc = __builtin_fma(c[2], (double)q[-AW] + (double)q[AW], acc);
    acc = __builtin_fma(c[3], (double)q[-AW - 1] + (double)q[AW + 1], acc);
    acc = __builtin_fma(c[4], (double)q[-AW + 1] + (double)q[AW - 1], acc);
    const int64_t idx = in.off + (int64_t)gy * n + gx;
    ub_out[idx] = (float)((double)ub[idx] - acc);
    if (fb != nullptr) fb[idx] += q[0];
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

void launch_tg_dst(int pass, const TgDev& g, const Tile* groups, int ngroups, const float* in, float* out,
                   const float* symbol, const float* shat, float* shat_out, float* dsym, hipStream_t st) {
  if (pass == 0)
    hipLaunchKernelGGL((k_tg_dst<0>), dim3(ngroups), dim3(WG), 0, st, g, groups, in, out, symbol, shat, shat_out,
                       dsym);
  else if (pass == 1)
    hipLaunchKernelGGL((k_tg_dst<1>), dim3(ngroups), dim3(WG), 0, st, g, groups, in, out, symbol, shat, shat_out,
                       dsym);
  else
    hipLaunchKernelGGL((k_tg_dst<2>), dim3(ngroups), dim3(WG), 0, st, g, groups, in, out, symbol, shat, shat_out,
                       dsym);
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
