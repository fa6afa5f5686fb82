// Temporal-blocked fused steps for gfx950 (overlapped tiling).
//
// A workgroup of 8 CW threads owns an extended tile of CW x 8R points: thread t
// holds u, v and f of a vertical strip of R points of column t mod CW in
// registers (consecutive threads take consecutive columns, so every global
// access of a wave is a contiguous row segment).  The workgroup runs T
// consecutive inner steps of a Table-1 scheme (Richardson(m), MOM-, NAG- or
// NAGex-Richardson(m), optionally with weighted-Jacobi preconditioning) on the
// whole extended tile without touching HBM in between:
//   per step: u~ = u + at_i v  ->  LDS
//             v' = a_i v + w_i (f - A u~) from LDS,  u' = u + v'.
// The LDS tile has a zero border.  Where a tile edge lies on or beyond the
// domain boundary that border (and the zeros published by points outside the
// n x n interior) is exactly the homogeneous Dirichlet condition, so nothing
// goes stale there.  Across an interior edge the values outside the tile are
// missing and the outermost ring goes wrong by one point per step; tiles
// therefore overlap by a halo of h >= T points at interior edges and each tile
// stores only its owned rectangle (given per tile).  With a residual requested
// (h >= T + 1), ||f - A u||^2 of the final u is accumulated over the owned
// points as well.  An instance that fits in one tile needs no halo at all and
// can run any number of steps per launch.
//
// One LDS buffer holds the published field; each step has two barriers (after
// publishing, and before the next step overwrites it), which keeps the LDS and
// register footprint small enough for two or three workgroups per CU, so that
// one workgroup's loads and stores overlap another's arithmetic.
//
// The update is evaluated with the same fused multiply-add sequence as the
// one-step kernel, so a launch of T steps reproduces T one-step launches bit
// for bit.
#include "rm_device.h"

#pragma clang fp contract(off)

namespace rmk {

namespace {

// Walk down this thread's strip with a three-row window over the LDS tile B (row
// stride LW, zero border; strip row k sits at LDS row lr0 + k + 1, column lc + 1)
// and hand f(k, C, W, E, S, N, SW, NE, SE, NW) the nine inputs of every point.
template <int R, int LW, typename F>
__device__ __forceinline__ void strip_walk(const float* B, int lc, int lr0, F&& f) {
  const float* q = B + lr0 * LW + lc;
  float Lm = q[0], Cm = q[1], Rm = q[2];
  float L0 = q[LW], C0 = q[LW + 1], R0 = q[LW + 2];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const float* qn = q + (k + 2) * LW;
    const float Lp = qn[0], Cp = qn[1], Rp = qn[2];
    f(k, C0, L0, R0, Cm, Cp, Lm, Rp, Rm, Lp);
    Lm = L0; Cm = C0; Rm = R0;
    L0 = Lp; C0 = Cp; R0 = Rp;
  }
}

// Thread t of a workgroup of 8 CW threads takes column t mod CW and the strip of
// R rows starting at R (t / CW): the extended tile is CW x 8R points.  CW is a
// run-time multiple of 8 (CW + 2 <= LW); T >= 0 is a run-time step count (T = 0
// copies the owned points and can still form the residual).
// With STORE, the owned (u, v) after every step but the last are also written to
// states + t * state_stride (u) and + state_stride / 2 (v) for t = 0 .. T - 2 (the
// adjoint's forward recompute keeps every intermediate state).
template <int R, int LW, int WPE, int METHOD, bool STORE>
__global__ __attribute__((amdgpu_flat_work_group_size(64, 8 * (LW - 2)), amdgpu_waves_per_eu(WPE))) void k_block(
    PlanDev p, const BTile* __restrict__ tiles, int ntiles, int T, int CW, const float* __restrict__ omega,
    const float* __restrict__ alpha, int m, int s0, const float* __restrict__ f, const float* __restrict__ u,
    const float* __restrict__ v, float* __restrict__ u_out, float* __restrict__ v_out,
    const int* __restrict__ active, double* __restrict__ partial2, float* __restrict__ states,
    int64_t state_stride) {
  constexpr int NS = 8;
  constexpr int EH = R * NS;
  constexpr int LH = EH + 2;
  __shared__ float B[LH * LW];
  __shared__ double sh[16];
  const int NT = CW * NS;
  const int per = ntiles >> 3;
  const BTile tl = tiles[(blockIdx.x & 7) * per + (blockIdx.x >> 3)];
  if (tl.inst < 0) return;
  if (active != nullptr && active[tl.inst] == 0) return;
  const Inst in = p.inst[tl.inst];
  const int n = in.n;
  float c[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) c[k] = p.coef32[tl.inst * 8 + k];
  const int lc = (int)threadIdx.x % CW;
  const int lr0 = ((int)threadIdx.x / CW) * R;
  const int gx = tl.x0 + lc;
  const bool colin = gx >= 0 && gx < n;
  const int gy0 = tl.y0 + lr0;
  const float* ui = u + in.off;
  const float* vi = v + in.off;
  const float* fi = f + in.off;
  float ru[R], rv[R], rf[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int gy = gy0 + k;
    const bool ok = colin && gy >= 0 && gy < n;
    const int idx = gy * n + gx;
    ru[k] = ok ? ui[idx] : 0.0f;
    rv[k] = (uses_momentum(METHOD) && ok) ? vi[idx] : 0.0f;
    rf[k] = ok ? fi[idx] : 0.0f;
  }
  // zero border ring for the CW + 2 columns in use
  const int LWc = CW + 2;
  for (int e = threadIdx.x; e < 2 * LWc + 2 * EH; e += NT) {
    int idx;
    if (e < LWc) idx = e;
    else if (e < 2 * LWc) idx = (LH - 1) * LW + (e - LWc);
    else if (e < 2 * LWc + EH) idx = (1 + e - 2 * LWc) * LW;
    else idx = (1 + e - 2 * LWc - EH) * LW + CW + 1;
    B[idx] = 0.0f;
  }
  float* mine = B + (lr0 + 1) * LW + lc + 1;
#pragma unroll 1
  for (int t = 0; t < T; ++t) {
    const int i = (s0 + t) % m;
    float w, a, at;
    step_factors<float, METHOD>(p, omega, alpha, m, tl.inst, i, w, a, at);
    if (t > 0) __syncthreads();  // every read of the previous step is done
#pragma unroll
    for (int k = 0; k < R; ++k) {
      // points outside the n x n interior publish 0 (Dirichlet); their
      // registers are never stored
      const int gy = gy0 + k;
      const bool ok = colin && gy >= 0 && gy < n;
      const float x = uses_lookahead(METHOD) ? fmadd(at, rv[k], ru[k]) : ru[k];
      mine[k * LW] = ok ? x : 0.0f;
    }
    __syncthreads();
    strip_walk<R, LW>(B, lc, lr0, [&](int k, float C, float W, float E, float S, float N, float SW, float NE,
                                      float SE, float NW) {
      const float vn = step_vf(c, w, a, rf[k], rv[k], C, W, E, S, N, SW, NE, SE, NW);
      ru[k] = ru[k] + vn;
      rv[k] = vn;
    });
    if (STORE && t + 1 < T && gx >= tl.ox0 && gx < tl.ox1) {
      float* su = states + (int64_t)t * state_stride + in.off;
      float* sv = su + state_stride / 2;
#pragma unroll
      for (int k = 0; k < R; ++k) {
        const int gy = gy0 + k;
        if (gy >= tl.oy0 && gy < tl.oy1) {
          su[gy * n + gx] = ru[k];
          if (uses_momentum(METHOD)) sv[gy * n + gx] = rv[k];
        }
      }
    }
  }
  const bool colown = gx >= tl.ox0 && gx < tl.ox1;
  double r2 = 0.0;
  if (partial2 != nullptr) {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int gy = gy0 + k;
      const bool ok = colin && gy >= 0 && gy < n;
      mine[k * LW] = ok ? ru[k] : 0.0f;
    }
    __syncthreads();
    strip_walk<R, LW>(B, lc, lr0, [&](int k, float C, float W, float E, float S, float N, float SW, float NE,
                                      float SE, float NW) {
      const int gy = gy0 + k;
      if (colown && gy >= tl.oy0 && gy < tl.oy1) {
        const float r = residual9<float>(c, rf[k], C, W, E, S, N, SW, NE, SE, NW);
        r2 += (double)r * (double)r;
      }
    });
  }
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int gy = gy0 + k;
    if (colown && gy >= tl.oy0 && gy < tl.oy1) {
      const int64_t idx = in.off + (int64_t)gy * n + gx;
      u_out[idx] = ru[k];
      if (uses_momentum(METHOD)) v_out[idx] = rv[k];
    }
  }
  if (partial2 != nullptr) {
    // fixed-order workgroup sum over NT / 64 waves
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) r2 += __shfl_xor(r2, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = r2;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int k = 0; k < NT / 64; ++k) s += sh[k];
      partial2[2 * tl.slot] = s;
      partial2[2 * tl.slot + 1] = 0.0;
    }
  }
}

template <int R, int LW, int WPE>
void launch_variant(int T, int cw, int method, const PlanDev& p, const BTile* tiles, int ntiles, const float* omega,
                    const float* alpha, int m, int s0, const float* f, const float* u, const float* v, float* u_out,
                    float* v_out, const int* active, double* partial2, float* states, int64_t state_stride,
                    hipStream_t st) {
  const dim3 grid(ntiles), block(8 * cw);
#define RM_LAUNCH(MM, SS)                                                                                          \
  hipLaunchKernelGGL((k_block<R, LW, WPE, MM, SS>), grid, block, 0, st, p, tiles, ntiles, T, cw, omega, alpha, m, \
                     s0, f, u, v, u_out, v_out, active, partial2, states, state_stride)
  const bool store = states != nullptr;
  switch (method) {
    case M_NAG: if (store) RM_LAUNCH(M_NAG, true); else RM_LAUNCH(M_NAG, false); break;
    case M_MOM: if (store) RM_LAUNCH(M_MOM, true); else RM_LAUNCH(M_MOM, false); break;
    case M_NAGEX: if (store) RM_LAUNCH(M_NAGEX, true); else RM_LAUNCH(M_NAGEX, false); break;
    default: if (store) RM_LAUNCH(M_RICH, true); else RM_LAUNCH(M_RICH, false); break;
  }
#undef RM_LAUNCH
}

}  // namespace


bool launch_block(int variant, int T, int cw, int method, const PlanDev& p, const BTile* tiles, int ntiles,
                  const float* omega, const float* alpha, int m, int s0, const float* f, const float* u,
                  const float* v, float* u_out, float* v_out, const int* active, double* partial2,
                  hipStream_t st, float* states, int64_t state_stride) {
  if (variant < 0 || variant >= kNumBlockVariants || T < 0) return false;
  if (cw < 8 || cw % 8 != 0 || cw + 2 > kBlockVariants[variant].lw) return false;
#define RM_VARIANT_CASE(V, R, LW, WPE)                                                                        \
  case V:                                                                                                     \
    launch_variant<R, LW, WPE>(T, cw, method, p, tiles, ntiles, omega, alpha, m, s0, f, u, v, u_out, v_out, \
                               active, partial2, states, state_stride, st);                                   \
    return true;
  // register caps (waves per SIMD) chosen so that two or three workgroups fit on a CU;
  // the 32-row strips need 168 registers and run one workgroup per CU
  switch (variant) {
    RM_VARIANT_CASE(0, 8, 66, 8)
    RM_VARIANT_CASE(1, 16, 66, 4)
    RM_VARIANT_CASE(2, 8, 130, 7)
    RM_VARIANT_CASE(3, 13, 66, 6)
    RM_VARIANT_CASE(4, 16, 130, 4)
    RM_VARIANT_CASE(5, 12, 98, 6)
    RM_VARIANT_CASE(6, 13, 106, 6)
    RM_VARIANT_CASE(7, 32, 66, 3)
    RM_VARIANT_CASE(8, 32, 98, 3)
    default:
      return false;
  }
#undef RM_VARIANT_CASE
}

}  // namespace rmk
