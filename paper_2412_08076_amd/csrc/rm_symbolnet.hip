// Symbol network of the two-grid Helmholtz cycle (§3: the meta network behind Lambda~ of
// the spectral correction, eq. dl-him-h; the exponential takes the log form that §3.2 uses
// for the smoother weight), forward and backward, FP32.
//
// Per instance, on the coarse mode grid (nc x nc, mode (p, q) at [q-1][p-1]):
//   features  X = (lam h^2 / 8, p / (nc + 1), q / (nc + 1)), lam the fine-grid eigenvalue
//             (4/h^2)(sin^2(p pi h/2) + sin^2(q pi h/2)) - kappa^2, h = 1/(n+1) (FP64);
//   a1 = tanh(conv(X; W1, b1)),  a2 = tanh(conv(a1; W2, b2)),  z = conv(a2; W3, b3),
//   symbol = lam / (lam^2 + 1) exp(z),
// with 3 x 3 cross-correlations, zero padding, 3 -> 16 -> 16 -> 1 channels.  Parameters in
// one flat vector, W1[16][3][3][3], b1[16], W2[16][16][3][3], b2[16], W3[1][16][3][3], b3[1].
//
// Each workgroup takes a 16 x 16 tile of one instance's modes and stages its input
// channels with a one-point halo in LDS; the weights are the same for every thread and
// are read as scalars.  Activations are stored channel-planar over the packed coarse
// vector (channel c of coarse point k at c * Pc + k).  The backward pass forms the input
// gradient through the transposed convolution and the tanh derivative, and per tile the
// partial sums of every weight's gradient (thread = (output, input) channel pair, the nine
// kernel offsets in registers); the weights themselves are staged in LDS, transposed so
// that the weights one staged value multiplies are consecutive words.  The partials are
// summed in FP64 in a fixed order (each group of SN_TG consecutive tiles in tile order,
// then the groups in order), so the gradient is the same on every run.
#include "rm_device.h"

#pragma clang fp contract(off)

namespace rmk {

namespace {

constexpr int SN_T = 16;            // tile edge (coarse modes)
constexpr int SN_H = SN_T + 2;      // with the halo
constexpr int SN_PL = SN_H * SN_H + 1;  // LDS plane stride (odd: channel planes on distinct banks)
constexpr int SN_C = 16;            // hidden channels
constexpr int SN_TG = 64;           // tiles per group of the weight-gradient reduction
constexpr int SN_W1 = 0, SN_B1 = SN_W1 + SN_C * 3 * 9, SN_W2 = SN_B1 + SN_C, SN_B2 = SN_W2 + SN_C * SN_C * 9,
              SN_W3 = SN_B2 + SN_C, SN_B3 = SN_W3 + SN_C * 9, SN_NP = SN_B3 + 1;

// The fine-grid eigenvalue of mode (p, q) (1-based) of instance b, in FP64.
__device__ __forceinline__ double sn_lambda(const PlanDev& p, int b, int pp, int qq) {
  const int n = p.inst[b].n;
  const double kappa = (double)p.mu[2 * b + 1];
  const double h = 1.0 / (double)(n + 1);
  const double sp = sin((double)pp * M_PI * h * 0.5), sq = sin((double)qq * M_PI * h * 0.5);
  return (4.0 / (h * h)) * (sp * sp + sq * sq) - kappa * kappa;
}

// Stage CIN channels of the input around tile (x0, y0) of instance b into lds[ci][j][i]
// (= point (x0 - 1 + i, y0 - 1 + j)), zero outside the nc x nc grid; the input is either
// the features (FEAT) or channel planes of a coarse field.
template <int CIN, bool FEAT>
__device__ __forceinline__ void sn_stage(const PlanDev& p, int b, int nc, int64_t coff, int64_t Pc, int x0, int y0,
                                         const float* __restrict__ src, float* lds) {
  const double h = 1.0 / (double)(p.inst[b].n + 1);
  for (int e = threadIdx.x; e < SN_H * SN_H; e += SN_T * SN_T) {
    const int j = e / SN_H, i = e - j * SN_H;
    const int x = x0 - 1 + i, y = y0 - 1 + j;
    const bool in = (unsigned)x < (unsigned)nc && (unsigned)y < (unsigned)nc;
    if constexpr (FEAT) {
      float f0 = 0.f, f1 = 0.f, f2 = 0.f;
      if (in) {
        f0 = (float)(sn_lambda(p, b, x + 1, y + 1) * h * h * 0.125);
        f1 = (float)(x + 1) / (float)(nc + 1);
        f2 = (float)(y + 1) / (float)(nc + 1);
      }
      lds[e] = f0;
      lds[SN_PL + e] = f1;
      lds[2 * SN_PL + e] = f2;
    } else {
      const int64_t k = coff + (int64_t)(in ? y : 0) * nc + (in ? x : 0);
#pragma unroll
      for (int c = 0; c < CIN; ++c) lds[c * SN_PL + e] = in ? src[c * Pc + k] : 0.0f;
    }
  }
}

// Forward layer: out = act(conv(in)) for COUT channels (MODE 0: tanh to channel planes;
// MODE 1: the symbol, COUT = 1).
template <int CIN, int COUT, bool FEAT, int MODE>
__global__ __launch_bounds__(SN_T* SN_T) void k_sn_forward(PlanDev p, TgDev g, const Tile* __restrict__ tiles,
                                                           int64_t Pc, const float* __restrict__ params, int woff,
                                                           int boff, const float* __restrict__ in,
                                                           float* __restrict__ out) {
  __shared__ float lds[CIN * SN_PL];
  __shared__ float wl[CIN * 9 * COUT + COUT];  // [ci][k][co], then the biases
  const Tile tl = tiles[blockIdx.x];
  if (tl.inst < 0) return;
  const TgInst gi = g.inst[tl.inst];
  const int nc = gi.nc;
  for (int e = threadIdx.x; e < CIN * 9 * COUT; e += SN_T * SN_T) {
    const int co = e / (CIN * 9), r = e - co * CIN * 9;  // r = ci * 9 + k
    wl[r * COUT + co] = params[woff + e];
  }
  if (threadIdx.x < COUT) wl[CIN * 9 * COUT + threadIdx.x] = params[boff + threadIdx.x];
  sn_stage<CIN, FEAT>(p, tl.inst, nc, gi.coff, Pc, tl.x0, tl.y0, in, lds);
  __syncthreads();
  const int tx = threadIdx.x % SN_T, ty = threadIdx.x / SN_T;
  const int x = tl.x0 + tx, y = tl.y0 + ty;
  if (x >= nc || y >= nc) return;
  float acc[COUT];
#pragma unroll
  for (int co = 0; co < COUT; ++co) acc[co] = wl[CIN * 9 * COUT + co];
#pragma unroll 1
  for (int ci = 0; ci < CIN; ++ci)
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const float v = lds[ci * SN_PL + (ty + k / 3) * SN_H + tx + k % 3];
      const float* w = wl + (ci * 9 + k) * COUT;
#pragma unroll
      for (int co = 0; co < COUT; ++co) acc[co] = fmadd(w[co], v, acc[co]);
    }
  const int64_t kk = gi.coff + (int64_t)y * nc + x;
  if constexpr (MODE == 0) {
#pragma unroll
    for (int co = 0; co < COUT; ++co) out[co * Pc + kk] = tanhf(acc[co]);
  } else {
    const double lam = sn_lambda(p, tl.inst, x + 1, y + 1);
    out[kk] = (float)(lam / (lam * lam + 1.0) * exp((double)acc[0]));
  }
}

// gz = d_symbol * symbol (d symbol / d z = symbol).
__global__ void k_sn_gz(int64_t Pc, const float* __restrict__ dsym, const float* __restrict__ sym,
                        float* __restrict__ gz) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < Pc; k += (int64_t)gridDim.x * blockDim.x)
    gz[k] = dsym[k] * sym[k];
}

// Backward layer: with gout the gradient at this layer's pre-activation output (COUT
// channels) and in its input (CIN channels, or the features): per tile, the partial
// gradients of the layer's weights and biases (part[tile][COUT * CIN * 9 + COUT]); with
// GIN, gin = (W^T * gout) (1 - in^2), the gradient at the previous layer's
// pre-activation output.
template <int CIN, int COUT, bool FEAT, bool GIN>
__global__ __launch_bounds__(SN_T* SN_T) void k_sn_backward(PlanDev p, TgDev g, const Tile* __restrict__ tiles,
                                                            int64_t Pc, const float* __restrict__ params, int woff,
                                                            const float* __restrict__ in,
                                                            const float* __restrict__ gout, float* __restrict__ gin,
                                                            float* __restrict__ part) {
  constexpr int NPL = COUT * CIN * 9 + COUT;
  __shared__ float lin[CIN * SN_PL];
  __shared__ float lg[COUT * SN_PL];
  __shared__ float wl[GIN ? COUT * 9 * CIN : 1];  // [co][k][ci]
  const Tile tl = tiles[blockIdx.x];
  float* my = part + (int64_t)blockIdx.x * NPL;
  if (tl.inst < 0) {
    for (int e = threadIdx.x; e < NPL; e += SN_T * SN_T) my[e] = 0.0f;
    return;
  }
  const TgInst gi = g.inst[tl.inst];
  const int nc = gi.nc;
  if constexpr (GIN)
    for (int e = threadIdx.x; e < COUT * CIN * 9; e += SN_T * SN_T) {
      const int co = e / (CIN * 9), r = e - co * CIN * 9, ci = r / 9, k = r - ci * 9;
      wl[(co * 9 + k) * CIN + ci] = params[woff + e];
    }
  sn_stage<CIN, FEAT>(p, tl.inst, nc, gi.coff, Pc, tl.x0, tl.y0, in, lin);
  sn_stage<COUT, false>(p, tl.inst, nc, gi.coff, Pc, tl.x0, tl.y0, gout, lg);
  __syncthreads();
  // weight gradients: thread (co, ci), all nine offsets, over the tile's points row by row
  const int t = threadIdx.x;
  if (t < COUT * CIN) {
    const int co = t / CIN, ci = t - co * CIN;
    float s[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) s[k] = 0.0f;
    float sb = 0.0f;
    for (int ty = 0; ty < SN_T; ++ty) {
#pragma unroll
      for (int tx = 0; tx < SN_T; ++tx) {
        // gout at interior point (tx, ty) sits at (tx + 1, ty + 1) of the staged tile
        const float gv = lg[co * SN_PL + (ty + 1) * SN_H + tx + 1];
        sb += gv;
#pragma unroll
        for (int k = 0; k < 9; ++k) s[k] = fmadd(gv, lin[ci * SN_PL + (ty + k / 3) * SN_H + tx + k % 3], s[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) my[(co * CIN + ci) * 9 + k] = s[k];
    if (ci == 0) my[COUT * CIN * 9 + co] = sb;
  }
  if constexpr (GIN) {
    const int tx = threadIdx.x % SN_T, ty = threadIdx.x / SN_T;
    const int x = tl.x0 + tx, y = tl.y0 + ty;
    if (x < nc && y < nc) {
      float acc[CIN];
#pragma unroll
      for (int ci = 0; ci < CIN; ++ci) acc[ci] = 0.0f;
#pragma unroll 1
      for (int co = 0; co < COUT; ++co)
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          // out(y', x') reads in(y' + ky - 1, x' + kx - 1): in(y, x) collects from y' = y - ky + 1
          const float gv = lg[co * SN_PL + (ty + 2 - k / 3) * SN_H + tx + 2 - k % 3];
          const float* w = wl + (co * 9 + k) * CIN;
#pragma unroll
          for (int ci = 0; ci < CIN; ++ci) acc[ci] = fmadd(w[ci], gv, acc[ci]);
        }
      const int64_t kk = gi.coff + (int64_t)y * nc + x;
#pragma unroll
      for (int ci = 0; ci < CIN; ++ci) {
        const float a = lin[ci * SN_PL + (ty + 1) * SN_H + tx + 1];
        gin[ci * Pc + kk] = acc[ci] * (1.0f - a * a);
      }
    }
  }
}

// gsum[g][k] = sum over the tiles t of group g (t = g SN_TG .. , in order) of part[t][k],
// k < npl, in FP64 (grid: parameter blocks x groups).
__global__ void k_sn_reduce_groups(const float* __restrict__ part, int ntiles, int npl, double* __restrict__ gsum) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x, g = blockIdx.y;
  if (k >= npl) return;
  const int t0 = g * SN_TG, t1 = min(ntiles, t0 + SN_TG);
  double s = 0.0;
  for (int t = t0; t < t1; ++t) s += (double)part[(int64_t)t * npl + k];
  gsum[(int64_t)g * npl + k] = s;
}

// d[k] = sum over the groups g (in order) of gsum[g][k], rounded to FP32 (zero without tiles).
__global__ void k_sn_reduce(const double* __restrict__ gsum, int ngroups, int npl, float* __restrict__ d) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= npl) return;
  double s = 0.0;
  for (int g = 0; g < ngroups; ++g) s += gsum[(int64_t)g * npl + k];
  d[k] = (float)s;
}

// The sum over the tiles of part[t][k] into d[k] (two kernels, see above).
void sn_reduce(const float* part, double* gsum, int ntiles, int npl, float* d, hipStream_t st) {
  const int ng = (ntiles + SN_TG - 1) / SN_TG;
  if (ng > 0)
    hipLaunchKernelGGL(k_sn_reduce_groups, dim3((npl + 255) / 256, ng), dim3(256), 0, st, part, ntiles, npl, gsum);
  hipLaunchKernelGGL(k_sn_reduce, dim3((npl + 255) / 256), dim3(256), 0, st, (const double*)gsum, ng, npl, d);
}

}  // namespace

int symbolnet_param_count() { return SN_NP; }

void launch_symbolnet_forward(const PlanDev& p, const TgDev& g, const Tile* tiles, int ntiles, int64_t Pc,
                              const float* params, float* a1, float* a2, float* symbol, hipStream_t st) {
  if (ntiles == 0) return;  // no instance has a coarse grid
  hipLaunchKernelGGL((k_sn_forward<3, SN_C, true, 0>), dim3(ntiles), dim3(SN_T * SN_T), 0, st, p, g, tiles, Pc,
                     params, SN_W1, SN_B1, (const float*)nullptr, a1);
  hipLaunchKernelGGL((k_sn_forward<SN_C, SN_C, false, 0>), dim3(ntiles), dim3(SN_T * SN_T), 0, st, p, g, tiles, Pc,
                     params, SN_W2, SN_B2, (const float*)a1, a2);
  hipLaunchKernelGGL((k_sn_forward<SN_C, 1, false, 1>), dim3(ntiles), dim3(SN_T * SN_T), 0, st, p, g, tiles, Pc,
                     params, SN_W3, SN_B3, (const float*)a2, symbol);
}

void launch_symbolnet_backward(const PlanDev& p, const TgDev& g, const Tile* tiles, int ntiles, int64_t Pc,
                               const float* params, const float* a1, const float* a2, const float* symbol,
                               const float* d_symbol, float* gz, float* g1, float* g2, float* part, double* gsum,
                               float* d_params, hipStream_t st) {
  constexpr int N3 = 1 * SN_C * 9 + 1, N2 = SN_C * SN_C * 9 + SN_C, N1 = SN_C * 3 * 9 + SN_C;
  if (ntiles == 0) {  // no coarse grid: the reductions over zero tiles write zero gradients
    sn_reduce(part, gsum, 0, SN_NP, d_params, st);
    return;
  }
  const int fill = (int)std::min<int64_t>((Pc + 255) / 256, 4096);
  hipLaunchKernelGGL(k_sn_gz, dim3(std::max(1, fill)), dim3(256), 0, st, Pc, d_symbol, symbol, gz);
  // layer 3: weights W3, b3 and the gradient at layer 2's pre-activation
  hipLaunchKernelGGL((k_sn_backward<SN_C, 1, false, true>), dim3(ntiles), dim3(SN_T * SN_T), 0, st, p, g, tiles, Pc,
                     params, SN_W3, a2, (const float*)gz, g2, part);
  sn_reduce(part, gsum, ntiles, N3, d_params + SN_W3, st);
  hipLaunchKernelGGL((k_sn_backward<SN_C, SN_C, false, true>), dim3(ntiles), dim3(SN_T * SN_T), 0, st, p, g, tiles,
                     Pc, params, SN_W2, a1, (const float*)g2, g1, part);
  sn_reduce(part, gsum, ntiles, N2, d_params + SN_W2, st);
  hipLaunchKernelGGL((k_sn_backward<3, SN_C, true, false>), dim3(ntiles), dim3(SN_T * SN_T), 0, st, p, g, tiles, Pc,
                     params, SN_W1, (const float*)nullptr, (const float*)g1, (float*)nullptr, part);
  sn_reduce(part, gsum, ntiles, N1, d_params + SN_W1, st);
}

}  // namespace rmk
