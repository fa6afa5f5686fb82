// Batched restarted flexible GMRES (arXiv 2412.08076 §3.2: FGMRES with restart 20,
// preconditioned by a neural multilevel solver whose action may change per iteration).
//
// Every instance of a plan runs its own FGMRES; the kernels below take one Arnoldi
// step for all active instances at once.  The basis V is FP64, the preconditioned
// directions Z are FP32 (the preconditioner's own output).  Orthogonalisation is
// classical Gram-Schmidt applied twice: one kernel forms, per tile, the dots of w with
// every basis vector (w read once into registers), a second sums them per instance in
// tile order (deterministic), a third subtracts.  The small per-instance algebra
// (Givens rotations, residual estimate, back substitution) runs one thread per instance.
#include "rm_device.h"

#pragma clang fp contract(off)

namespace rmk {

namespace {

constexpr int NW = WG / 64;
constexpr int RPT = TY / NW;  // rows per thread of a 64 x 32 tile

// partial[i * nslot + slot] = sum over the tile of w * V_i, i < nvec (V_i = V + i * stride).
__global__ __launch_bounds__(WG) void k_mdot(PlanDev p, const double* __restrict__ V, int64_t stride, int nvec,
                                             const double* __restrict__ w, const int* __restrict__ active,
                                             double* __restrict__ partial, int nslot) {
  __shared__ double sh[NW];
  const Tile tl = p.tiles[xcd_remap(blockIdx.x, gridDim.x)];
  if (tl.inst < 0) return;
  if (active[tl.inst] == 0) return;
  const Inst in = p.inst[tl.inst];
  const int n = in.n;
  const int tx = threadIdx.x & 63, ty0 = threadIdx.x >> 6;
  const int gx = tl.x0 + tx;
  double rw[RPT];
  int64_t idx[RPT];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int gy = tl.y0 + ty0 + NW * k;
    const bool ok = gx < n && gy < n;
    idx[k] = ok ? in.off + (int64_t)gy * n + gx : -1;
    rw[k] = ok ? w[idx[k]] : 0.0;
  }
  for (int i = 0; i < nvec; ++i) {
    const double* vi = V + (int64_t)i * stride;
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < RPT; ++k)
      if (idx[k] >= 0) acc = __builtin_fma(rw[k], vi[idx[k]], acc);
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[(int64_t)i * nslot + tl.pad] = t;
  }
}

// out[b * ldo + col0 + i] (+)= sum over the instance's tiles of partial[i * nslot + slot]:
// one wave per (instance, vector), lanes striding over the tiles in order, then a
// fixed shuffle tree (deterministic).
__global__ __launch_bounds__(64) void k_mreduce(PlanDev p, const double* __restrict__ partial, int nvec, int nslot,
                                                const int* __restrict__ active, double* __restrict__ out, int ldo,
                                                int col0, int accumulate) {
  const int t = blockIdx.x;
  const int b = t / nvec, i = t - b * nvec;
  if (active[b] == 0) return;
  const Inst in = p.inst[b];
  double s = 0.0;
  for (int k = in.tile_begin + (int)threadIdx.x; k < in.tile_end; k += 64)
    s += partial[(int64_t)i * nslot + p.tiles[k].pad];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (threadIdx.x == 0) {
    double* o = out + (int64_t)b * ldo + col0 + i;
    *o = accumulate ? *o + s : s;
  }
}

// w -= sum_i h[b * ldh + col0 + i] V_i over the plan's tiles.
__global__ __launch_bounds__(WG) void k_maxpy(PlanDev p, const double* __restrict__ V, int64_t stride, int nvec,
                                              const double* __restrict__ h, int ldh, int col0, double* __restrict__ w,
                                              const int* __restrict__ active) {
  const Tile tl = p.tiles[xcd_remap(blockIdx.x, gridDim.x)];
  if (tl.inst < 0) return;
  if (active[tl.inst] == 0) return;
  const Inst in = p.inst[tl.inst];
  const int n = in.n;
  const int tx = threadIdx.x & 63, ty0 = threadIdx.x >> 6;
  const int gx = tl.x0 + tx;
  if (gx >= n) return;
  const double* hb = h + (int64_t)tl.inst * ldh + col0;
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int gy = tl.y0 + ty0 + NW * k;
    if (gy >= n) break;
    const int64_t idx = in.off + (int64_t)gy * n + gx;
    double acc = w[idx];
    for (int i = 0; i < nvec; ++i) acc = __builtin_fma(-hb[i], V[(int64_t)i * stride + idx], acc);
    w[idx] = acc;
  }
}

// dst = src / sqrt(nrm2[b]) (0 when the norm is 0) for active instances.
__global__ __launch_bounds__(WG) void k_scale(PlanDev p, const double* __restrict__ src, const double* __restrict__ nrm2,
                                              int ldn, double* __restrict__ dst, const int* __restrict__ active) {
  const Tile tl = p.tiles[xcd_remap(blockIdx.x, gridDim.x)];
  if (tl.inst < 0) return;
  if (active[tl.inst] == 0) return;
  const Inst in = p.inst[tl.inst];
  const int n = in.n;
  const double s2 = nrm2[(int64_t)tl.inst * ldn];
  const double inv = s2 > 0.0 ? 1.0 / sqrt(s2) : 0.0;
  const int tx = threadIdx.x & 63, ty0 = threadIdx.x >> 6;
  const int gx = tl.x0 + tx;
  if (gx >= n) return;
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int gy = tl.y0 + ty0 + NW * k;
    if (gy >= n) break;
    const int64_t idx = in.off + (int64_t)gy * n + gx;
    dst[idx] = src[idx] * inv;
  }
}

// dst = fl32(src) on the instances in the current cycle, 0 on the others.
__global__ __launch_bounds__(WG) void k_to_f32_masked(PlanDev p, const double* __restrict__ src,
                                                      float* __restrict__ dst, const int* __restrict__ active) {
  const Tile tl = p.tiles[xcd_remap(blockIdx.x, gridDim.x)];
  if (tl.inst < 0) return;
  const Inst in = p.inst[tl.inst];
  const int n = in.n;
  const bool on = active[tl.inst] != 0;
  const int tx = threadIdx.x & 63, ty0 = threadIdx.x >> 6;
  const int gx = tl.x0 + tx;
  if (gx >= n) return;
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int gy = tl.y0 + ty0 + NW * k;
    if (gy >= n) break;
    const int64_t idx = in.off + (int64_t)gy * n + gx;
    dst[idx] = on ? (float)src[idx] : 0.f;
  }
}

__global__ void k_f32_to_f64(const float* __restrict__ s, double* __restrict__ d, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) d[i] = (double)s[i];
}

// Start of a cycle: for every instance still running, the true residual's ||r||^2 and
// ||b||^2 decide whether it has finished (converged, diverged or out of iterations);
// the others join the cycle with g = (beta, 0, ..).  jdone = 0 for all.
__global__ void k_fgm_start(int B, const double* __restrict__ r2b2, double tol, int max_iter,
                            const int* __restrict__ iters, int* __restrict__ running, int* __restrict__ active,
                            int* __restrict__ status, double* __restrict__ relres, double* __restrict__ g, int ldg,
                            int* __restrict__ jdone) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  jdone[b] = 0;
  active[b] = 0;
  if (running[b] == 0) return;
  const double r2 = r2b2[2 * b], b2 = r2b2[2 * b + 1];
  const double rel = b2 > 0.0 ? sqrt(r2 / b2) : 0.0;
  relres[b] = rel;
  if (!(rel == rel) || rel > 1e300) {
    running[b] = 0;
    status[b] = 5;  // RM_EDIVERGED
    return;
  }
  if (rel <= tol) {
    running[b] = 0;
    status[b] = 0;
    return;
  }
  if (iters[b] >= max_iter) {
    running[b] = 0;
    status[b] = 4;  // RM_ENOTCONV
    return;
  }
  active[b] = 1;
  double* gb = g + (int64_t)b * ldg;
  gb[0] = sqrt(r2);
  for (int k = 1; k < ldg; ++k) gb[k] = 0.0;
}

// After Arnoldi step j: column j of H (rows 0..j from the dots, row j + 1 = ||w||),
// previous rotations applied, a new one formed, g rotated; the residual estimate
// |g_{j+1}| / ||b|| decides whether the instance stops in this cycle.
__global__ void k_fgm_givens(int B, int j, int restart, double* __restrict__ H, const double* __restrict__ hn2,
                             double* __restrict__ cs, double* __restrict__ sn, double* __restrict__ g,
                             const double* __restrict__ r2b2, double tol, int max_iter, int* __restrict__ iters,
                             int* __restrict__ jdone, int* __restrict__ active, double* __restrict__ est) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  if (active[b] == 0) return;
  const int ldh = restart + 1;
  double* h = H + ((int64_t)b * restart + j) * ldh;  // column j of instance b
  double* c = cs + (int64_t)b * restart;
  double* s = sn + (int64_t)b * restart;
  double* gb = g + (int64_t)b * (restart + 1);
  h[j + 1] = sqrt(hn2[b]);
  for (int i = 0; i < j; ++i) {
    const double t = c[i] * h[i] + s[i] * h[i + 1];
    h[i + 1] = -s[i] * h[i] + c[i] * h[i + 1];
    h[i] = t;
  }
  const double rr = hypot(h[j], h[j + 1]);
  const double cj = rr > 0.0 ? h[j] / rr : 1.0;
  const double sj = rr > 0.0 ? h[j + 1] / rr : 0.0;
  c[j] = cj;
  s[j] = sj;
  h[j] = rr;
  h[j + 1] = 0.0;
  gb[j + 1] = -sj * gb[j];
  gb[j] = cj * gb[j];
  jdone[b] = j + 1;
  iters[b] += 1;
  const double bn = sqrt(r2b2[2 * b + 1]);
  const double e = bn > 0.0 ? fabs(gb[j + 1]) / bn : 0.0;
  est[b] = e;
  if (e <= tol || iters[b] >= max_iter || hn2[b] == 0.0 || !(e == e) || j + 1 == restart) active[b] = 0;
}

// y = R^{-1} g over the first jdone[b] columns (R the rotated H), one thread per instance.
__global__ void k_fgm_backsolve(int B, int restart, const double* __restrict__ H, const double* __restrict__ g,
                                const int* __restrict__ jdone, double* __restrict__ y) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const int J = jdone[b];
  const int ldh = restart + 1;
  const double* Hb = H + (int64_t)b * restart * ldh;
  const double* gb = g + (int64_t)b * (restart + 1);
  double* yb = y + (int64_t)b * restart;
  for (int k = J - 1; k >= 0; --k) {
    double s = gb[k];
    for (int q = k + 1; q < J; ++q) s -= Hb[(int64_t)q * ldh + k] * yb[q];
    yb[k] = s / Hb[(int64_t)k * ldh + k];
  }
}

// x += sum_{k < jdone[b]} y[b][k] Z_k (Z FP32).
__global__ __launch_bounds__(WG) void k_fgm_xupdate(PlanDev p, const float* __restrict__ Z, int64_t stride,
                                                    const double* __restrict__ y, int restart,
                                                    const int* __restrict__ jdone, double* __restrict__ x) {
  const Tile tl = p.tiles[xcd_remap(blockIdx.x, gridDim.x)];
  if (tl.inst < 0) return;
  const int J = jdone[tl.inst];
  if (J == 0) return;
  const Inst in = p.inst[tl.inst];
  const int n = in.n;
  const int tx = threadIdx.x & 63, ty0 = threadIdx.x >> 6;
  const int gx = tl.x0 + tx;
  if (gx >= n) return;
  const double* yb = y + (int64_t)tl.inst * restart;
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int gy = tl.y0 + ty0 + NW * k;
    if (gy >= n) break;
    const int64_t idx = in.off + (int64_t)gy * n + gx;
    double acc = x[idx];
    for (int q = 0; q < J; ++q) acc = __builtin_fma(yb[q], (double)Z[(int64_t)q * stride + idx], acc);
    x[idx] = acc;
  }
}

}  // namespace

void launch_mdot(const PlanDev& p, const double* V, int64_t stride, int nvec, const double* w, const int* active,
                 double* partial, int nslot, hipStream_t st) {
  hipLaunchKernelGGL(k_mdot, dim3(p.ntiles), dim3(WG), 0, st, p, V, stride, nvec, w, active, partial, nslot);
}
void launch_mreduce(const PlanDev& p, const double* partial, int nvec, int nslot, const int* active, double* out,
                    int ldo, int col0, bool accumulate, hipStream_t st) {
  hipLaunchKernelGGL(k_mreduce, dim3(p.B * nvec), dim3(64), 0, st, p, partial, nvec, nslot, active, out, ldo, col0,
                     accumulate ? 1 : 0);
}
void launch_maxpy(const PlanDev& p, const double* V, int64_t stride, int nvec, const double* h, int ldh, int col0,
                  double* w, const int* active, hipStream_t st) {
  hipLaunchKernelGGL(k_maxpy, dim3(p.ntiles), dim3(WG), 0, st, p, V, stride, nvec, h, ldh, col0, w, active);
}
void launch_scale(const PlanDev& p, const double* src, const double* nrm2, int ldn, double* dst, const int* active,
                  hipStream_t st) {
  hipLaunchKernelGGL(k_scale, dim3(p.ntiles), dim3(WG), 0, st, p, src, nrm2, ldn, dst, active);
}
void launch_to_f32_masked(const PlanDev& p, const double* src, float* dst, const int* active, hipStream_t st) {
  hipLaunchKernelGGL(k_to_f32_masked, dim3(p.ntiles), dim3(WG), 0, st, p, src, dst, active);
}
void launch_f32_to_f64(const float* s, double* d, int64_t count, hipStream_t st) {
  hipLaunchKernelGGL(k_f32_to_f64, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, s, d, count);
}
void launch_fgm_start(int B, const double* r2b2, double tol, int max_iter, const int* iters, int* running,
                      int* active, int* status, double* relres, double* g, int ldg, int* jdone, hipStream_t st) {
  hipLaunchKernelGGL(k_fgm_start, dim3((B + 63) / 64), dim3(64), 0, st, B, r2b2, tol, max_iter, iters, running,
                     active, status, relres, g, ldg, jdone);
}
void launch_fgm_givens(int B, int j, int restart, double* H, const double* hn2, double* cs, double* sn, double* g,
                       const double* r2b2, double tol, int max_iter, int* iters, int* jdone, int* active, double* est,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_fgm_givens, dim3((B + 63) / 64), dim3(64), 0, st, B, j, restart, H, hn2, cs, sn, g, r2b2, tol,
                     max_iter, iters, jdone, active, est);
}
void launch_fgm_backsolve(int B, int restart, const double* H, const double* g, const int* jdone, double* y,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_fgm_backsolve, dim3((B + 63) / 64), dim3(64), 0, st, B, restart, H, g, jdone, y);
}
void launch_fgm_xupdate(const PlanDev& p, const float* Z, int64_t stride, const double* y, int restart,
                        const int* jdone, double* x, hipStream_t st) {
  hipLaunchKernelGGL(k_fgm_xupdate, dim3(p.ntiles), dim3(WG), 0, st, p, Z, stride, y, restart, jdone, x);
}

}  // namespace rmk
