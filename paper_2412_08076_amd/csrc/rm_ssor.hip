// SSOR-preconditioned inner steps of the Table-1 schemes (arXiv 2412.08076 §2.1:
// the SSOR entry of the stationary preconditioners, B^{-1} = a (2 - a) (D - aU)^{-1}
// D (D - aL)^{-1} with A = D - L - U and relaxation factor a).
//
// Ordering.  The split of A into L and U follows the four-colour ordering
// colour(i, j) = (i mod 2) + 2 (j mod 2): no two points of one colour are coupled by
// the 9-point (or 5-point) stencil, so each triangular solve is four fully parallel
// colour passes.  Relative to a point of colour c, its x-neighbours have colour c^1,
// its y-neighbours c^2 and its diagonal neighbours c^3; a neighbour is "lower" when its
// colour is smaller.
//   forward  (c = 0, 1, 2, 3):  y_p = (r_p - a sum_{lower q} A_pq y_q) / D
//   backward (c = 2, 1, 0):     w_p = y_p - (a / D) sum_{upper q} A_pq w_q   (colour 3: w = y)
//   B^{-1} r = a (2 - a) w.
//
// One inner step per launch.  A workgroup owns a 64 x 32 tile; the six passes that
// read neighbours each invalidate one more ring at the edge of the LDS region, so the
// region carries a halo of 6 (7 for the look-ahead field the residual needs) and is
// swept in place.  Points outside the domain hold 0 and are never updated (Dirichlet).
// Temporal blocking would need a halo of 7 per step, so none is attempted.
#include "rm_device.h"

#pragma clang fp contract(off)

namespace rmk {

namespace {

constexpr int HR = 6;               // halo of the swept region
constexpr int HU = HR + 1;          // halo of the field the residual is formed from
constexpr int RW = TX + 2 * HR;     // swept region 76 x 44
constexpr int RH = TY + 2 * HR;
constexpr int PW = RW + 2;          // plus a zero ring, so every neighbour read is in bounds
constexpr int PH = RH + 2;
constexpr int UW = TX + 2 * HU;     // 78 x 46 (= PW x PH)
constexpr int UH = TY + 2 * HU;
constexpr int NW = WG / 64;
static_assert(UW == PW && UH == PH, "the padded region and the residual input coincide");

// In-place SSOR sweeps on a padded LDS field s: a W x H region (W, H even) at offset
// (1, 1) of a (W + 2)-wide array whose outer ring is 0; region origin (ox, oy) in
// instance coordinates.  On entry the region holds r (0 outside the domain), on exit
// w with B^{-1} r = a (2 - a) w.  Colours are taken from instance coordinates.
template <typename T, int W, int H>
__device__ __forceinline__ void ssor_lds(T* s, int ox, int oy, int n, const T c[5], T relax, T dinv) {
  constexpr int S = W + 2, AW = W / 2, AH = H / 2;
  for (int col = 0; col < 4; ++col) {
    const int lx0 = (col & 1) ^ (ox & 1), ly0 = (col >> 1) ^ (oy & 1);
    for (int k = threadIdx.x; k < AW * AH; k += WG) {
      const int b = k / AW, a = k - b * AW;
      const int lx = 2 * a + lx0, ly = 2 * b + ly0;
      const int gx = ox + lx, gy = oy + ly;
      if (gx < 0 || gx >= n || gy < 0 || gy >= n) continue;
      T* q = s + (ly + 1) * S + (lx + 1);
      T acc = T(0);
      if (col & 1) acc = fmadd(c[1], q[-1] + q[1], acc);      // x-neighbours, colour col - 1
      if (col >= 2) {
        acc = fmadd(c[2], q[-S] + q[S], acc);                 // y-neighbours, colour col - 2
        acc = fmadd(c[3], q[-S - 1] + q[S + 1], acc);         // diagonals, colour col ^ 3
        acc = fmadd(c[4], q[-S + 1] + q[S - 1], acc);
      }
      q[0] = (q[0] - relax * acc) * dinv;
    }
    __syncthreads();
  }
  for (int col = 2; col >= 0; --col) {
    const int lx0 = (col & 1) ^ (ox & 1), ly0 = (col >> 1) ^ (oy & 1);
    for (int k = threadIdx.x; k < AW * AH; k += WG) {
      const int b = k / AW, a = k - b * AW;
      const int lx = 2 * a + lx0, ly = 2 * b + ly0;
      const int gx = ox + lx, gy = oy + ly;
      if (gx < 0 || gx >= n || gy < 0 || gy >= n) continue;
      T* q = s + (ly + 1) * S + (lx + 1);
      T acc = T(0);
      if (!(col & 1)) acc = fmadd(c[1], q[-1] + q[1], acc);   // x-neighbours, colour col + 1
      if (col < 2) {
        acc = fmadd(c[2], q[-S] + q[S], acc);                 // y-neighbours, colour col + 2
        acc = fmadd(c[3], q[-S - 1] + q[S + 1], acc);         // diagonals, colour col ^ 3
        acc = fmadd(c[4], q[-S + 1] + q[S - 1], acc);
      }
      q[0] = fmadd(-(relax * dinv), acc, q[0]);
    }
    __syncthreads();
  }
}

// 9-point stencil at padded position q (row stride W), fixed order.
template <typename T>
__device__ __forceinline__ T stencil_at(const T* q, int W, const T c[5]) {
  T acc = c[0] * q[0];
  acc = fmadd(c[1], q[-1] + q[1], acc);
  acc = fmadd(c[2], q[-W] + q[W], acc);
  acc = fmadd(c[3], q[-W - 1] + q[W + 1], acc);
  acc = fmadd(c[4], q[-W + 1] + q[W - 1], acc);
  return acc;
}

// One SSOR-preconditioned inner step (NAGex form):
//   u~ = u + at v;  r = f - A u~;  v' = a v + w B^{-1} r;  u' = u + v'.
template <typename T, int METHOD>
__global__ __launch_bounds__(WG) void k_ssor_step(PlanDev p, const Tile* __restrict__ tiles,
                                                  const float* __restrict__ omega, const float* __restrict__ alpha,
                                                  int m, int i, T relax, const T* __restrict__ f,
                                                  const T* __restrict__ u, const T* __restrict__ v,
                                                  T* __restrict__ u_out, T* __restrict__ v_out,
                                                  const int* __restrict__ active) {
  __shared__ T su[UH * UW];
  __shared__ T sr[PH * PW];
  const Tile tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
  if (tl.inst < 0) return;
  if (active != nullptr && active[tl.inst] == 0) return;
  const int bi = tl.inst;
  const Inst in = p.inst[bi];
  const int n = in.n;
  T c[5];
  load_coef<T>(p, bi, c);
  const T dinv = sizeof(T) == 4 ? (T)p.coef32[bi * 8 + 5] : (T)p.coef64[bi * 8 + 5];
  T w, a, at;
  step_factors<T, METHOD>(p, omega, alpha, m, bi, i, w, a, at);
  const T* ui = u + in.off;
  const T* vi = v + in.off;
  const T* fi = f + in.off;
  for (int k = threadIdx.x; k < UH * UW; k += WG) {
    const int ly = k / UW, lx = k - ly * UW;
    const int gx = tl.x0 - HU + lx, gy = tl.y0 - HU + ly;
    T val = T(0);
    if (gx >= 0 && gx < n && gy >= 0 && gy < n) {
      const int64_t idx = (int64_t)gy * n + gx;
      val = uses_lookahead(METHOD) ? fmadd(at, vi[idx], ui[idx]) : ui[idx];
    }
    su[k] = val;
  }
  __syncthreads();
  // residual on the swept region (its padded ring and the outside of the domain stay 0)
  for (int k = threadIdx.x; k < PH * PW; k += WG) {
    const int py = k / PW, px = k - py * PW;
    const int gx = tl.x0 - HR - 1 + px, gy = tl.y0 - HR - 1 + py;
    T r = T(0);
    const bool ring = px == 0 || py == 0 || px == PW - 1 || py == PH - 1;
    if (!ring && gx >= 0 && gx < n && gy >= 0 && gy < n)
      r = fi[(int64_t)gy * n + gx] - stencil_at(su + k, UW, c);
    sr[k] = r;
  }
  __syncthreads();
  ssor_lds<T, RW, RH>(sr, tl.x0 - HR, tl.y0 - HR, n, c, relax, dinv);
  const T s2 = relax * (T(2) - relax);
  const int tx = threadIdx.x & 63, ty0 = threadIdx.x >> 6;
  const int gx = tl.x0 + tx;
  if (gx >= n) return;
  for (int k = 0; k < TY / NW; ++k) {
    const int ly = ty0 + NW * k, gy = tl.y0 + ly;
    if (gy >= n) break;
    const int64_t idx = in.off + (int64_t)gy * n + gx;
    const T z = s2 * sr[(ly + HR + 1) * PW + (tx + HR + 1)];
    const T vv = uses_momentum(METHOD) ? v[idx] : T(0);
    const T vn = uses_momentum(METHOD) ? fmadd(a, vv, w * z) : w * z;
    v_out[idx] = vn;
    u_out[idx] = u[idx] + vn;
  }
}

// Reverse of one SSOR-preconditioned step (B^{-1} is symmetric):
//   g = vb + ub;  r = f - A u~;  z = B^{-1} r;  rb = w B^{-1} g;  fb += rb;
//   ut_bar = -A rb;  ub' = ub + ut_bar;  vb' = a g + at ut_bar (NAG: a (g + ut_bar)).
// Per tile: <g, z>, <g, v>, <ut_bar, v>.  rb is needed on the tile and a one-point
// ring, so g is staged with a halo of HR + 1.
template <int METHOD>
__global__ __launch_bounds__(WG) void k_adj_ssor_step(PlanDev p, const float* __restrict__ omega,
                                                      const float* __restrict__ alpha, int m, int i, float relax,
                                                      const float* __restrict__ f, const float* __restrict__ u,
                                                      const float* __restrict__ v, const float* __restrict__ ub,
                                                      const float* __restrict__ vb, float* __restrict__ ub_out,
                                                      float* __restrict__ vb_out, float* __restrict__ fb,
                                                      double* __restrict__ partial4) {
  constexpr int GW = TX + 2 * (HR + 1), GH = TY + 2 * (HR + 1);  // g region (halo 7)
  constexpr int GPW = GW + 2, GPH = GH + 2;
  __shared__ float su[UH * UW];
  __shared__ float sr[PH * PW];
  __shared__ float sg[GPH * GPW];
  __shared__ double sh[NW];
  const Tile tl = p.tiles[xcd_remap(blockIdx.x, gridDim.x)];
  if (tl.inst < 0) return;
  const int bi = tl.inst;
  const Inst in = p.inst[bi];
  const int n = in.n;
  float c[5];
  load_coef<float>(p, bi, c);
  const float dinv = p.coef32[bi * 8 + 5];
  float w, a, at;
  step_factors<float, METHOD>(p, omega, alpha, m, bi, i, w, a, at);
  const float* ui = u + in.off;
  const float* vi = v + in.off;
  const float* ubi = ub + in.off;
  const float* vbi = vb + in.off;
  const float* fi = f + in.off;
  for (int k = threadIdx.x; k < UH * UW; k += WG) {
    const int ly = k / UW, lx = k - ly * UW;
    const int gx = tl.x0 - HU + lx, gy = tl.y0 - HU + ly;
    float val = 0.f;
    if (gx >= 0 && gx < n && gy >= 0 && gy < n) {
      const int64_t idx = (int64_t)gy * n + gx;
      val = uses_lookahead(METHOD) ? fmadd(at, vi[idx], ui[idx]) : ui[idx];
    }
    su[k] = val;
  }
  for (int k = threadIdx.x; k < GPH * GPW; k += WG) {
    const int py = k / GPW, px = k - py * GPW;
    const int gx = tl.x0 - HR - 2 + px, gy = tl.y0 - HR - 2 + py;
    float val = 0.f;
    const bool ring = px == 0 || py == 0 || px == GPW - 1 || py == GPH - 1;
    if (!ring && gx >= 0 && gx < n && gy >= 0 && gy < n) {
      const int64_t idx = (int64_t)gy * n + gx;
      val = uses_momentum(METHOD) ? vbi[idx] + ubi[idx] : ubi[idx];
    }
    sg[k] = val;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < PH * PW; k += WG) {
    const int py = k / PW, px = k - py * PW;
    const int gx = tl.x0 - HR - 1 + px, gy = tl.y0 - HR - 1 + py;
    float r = 0.f;
    const bool ring = px == 0 || py == 0 || px == PW - 1 || py == PH - 1;
    if (!ring && gx >= 0 && gx < n && gy >= 0 && gy < n)
      r = fi[(int64_t)gy * n + gx] - stencil_at(su + k, UW, c);
    sr[k] = r;
  }
  __syncthreads();
  ssor_lds<float, RW, RH>(sr, tl.x0 - HR, tl.y0 - HR, n, c, relax, dinv);
  ssor_lds<float, GW, GH>(sg, tl.x0 - HR - 1, tl.y0 - HR - 1, n, c, relax, dinv);
  const float s2 = relax * (2.f - relax);
  double pw = 0.0, pg = 0.0, pl = 0.0;
  const int tx = threadIdx.x & 63, ty0 = threadIdx.x >> 6;
  const int gx = tl.x0 + tx;
  if (gx < n) {
    for (int k = 0; k < TY / NW; ++k) {
      const int ly = ty0 + NW * k, gy = tl.y0 + ly;
      if (gy >= n) break;
      const int64_t idx = in.off + (int64_t)gy * n + gx;
      const float z = s2 * sr[(ly + HR + 1) * PW + (tx + HR + 1)];
      const float* qg = sg + (ly + HR + 2) * GPW + (tx + HR + 2);  // w_g at this point
      // rb = w s2 w_g at the point and its ring; ut_bar = -A rb
      const float wsc = w * s2;
      float acc = c[0] * (wsc * qg[0]);
      acc = fmadd(c[1], wsc * qg[-1] + wsc * qg[1], acc);
      acc = fmadd(c[2], wsc * qg[-GPW] + wsc * qg[GPW], acc);
      acc = fmadd(c[3], wsc * qg[-GPW - 1] + wsc * qg[GPW + 1], acc);
      acc = fmadd(c[4], wsc * qg[-GPW + 1] + wsc * qg[GPW - 1], acc);
      const float utb = -acc;
      const float ubv = ubi[idx - in.off];
      const float vv = uses_momentum(METHOD) ? vi[idx - in.off] : 0.f;
      const float g = uses_momentum(METHOD) ? vbi[idx - in.off] + ubv : ubv;
      pw += (double)g * (double)z;
      pg += (double)g * (double)vv;
      pl += (double)utb * (double)vv;
      ub_out[idx] = ubv + utb;
      if (METHOD == M_NAG) vb_out[idx] = a * (g + utb);
      if (METHOD == M_MOM) vb_out[idx] = a * g;
      if (METHOD == M_NAGEX) vb_out[idx] = fmadd(at, utb, a * g);
      if (fb != nullptr) fb[idx] += wsc * qg[0];
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

}  // namespace

template <typename T>
void launch_ssor_step(int method, const PlanDev& p, const Tile* tiles, int ntiles, const float* omega,
                      const float* alpha, int m, int i, double relax, const T* f, const T* u, const T* v, T* u_out,
                      T* v_out, const int* active, hipStream_t st) {
  const T a = (T)relax;
  switch (method) {
    case M_RICH:
      hipLaunchKernelGGL((k_ssor_step<T, M_RICH>), dim3(ntiles), dim3(WG), 0, st, p, tiles, omega, alpha, m, i, a, f,
                         u, v, u_out, v_out, active);
      break;
    case M_NAG:
      hipLaunchKernelGGL((k_ssor_step<T, M_NAG>), dim3(ntiles), dim3(WG), 0, st, p, tiles, omega, alpha, m, i, a, f,
                         u, v, u_out, v_out, active);
      break;
    case M_MOM:
      hipLaunchKernelGGL((k_ssor_step<T, M_MOM>), dim3(ntiles), dim3(WG), 0, st, p, tiles, omega, alpha, m, i, a, f,
                         u, v, u_out, v_out, active);
      break;
    default:
      hipLaunchKernelGGL((k_ssor_step<T, M_NAGEX>), dim3(ntiles), dim3(WG), 0, st, p, tiles, omega, alpha, m, i, a,
                         f, u, v, u_out, v_out, active);
      break;
  }
}

template void launch_ssor_step<float>(int, const PlanDev&, const Tile*, int, const float*, const float*, int, int,
                                      double, const float*, const float*, const float*, float*, float*, const int*,
                                      hipStream_t);
template void launch_ssor_step<double>(int, const PlanDev&, const Tile*, int, const float*, const float*, int, int,
                                       double, const double*, const double*, const double*, double*, double*,
                                       const int*, hipStream_t);

void launch_adj_ssor_step(int method, const PlanDev& p, const float* omega, const float* alpha, int m, int i,
                          double relax, const float* f, const float* u, const float* v, const float* ub,
                          const float* vb, float* ub_out, float* vb_out, float* fb, double* partial4,
                          hipStream_t st) {
  const float a = (float)relax;
  switch (method) {
    case M_RICH:
      hipLaunchKernelGGL((k_adj_ssor_step<M_RICH>), dim3(p.ntiles), dim3(WG), 0, st, p, omega, alpha, m, i, a, f, u,
                         v, ub, vb, ub_out, vb_out, fb, partial4);
      break;
    case M_NAG:
      hipLaunchKernelGGL((k_adj_ssor_step<M_NAG>), dim3(p.ntiles), dim3(WG), 0, st, p, omega, alpha, m, i, a, f, u, v,
                         ub, vb, ub_out, vb_out, fb, partial4);
      break;
    case M_MOM:
      hipLaunchKernelGGL((k_adj_ssor_step<M_MOM>), dim3(p.ntiles), dim3(WG), 0, st, p, omega, alpha, m, i, a, f, u, v,
                         ub, vb, ub_out, vb_out, fb, partial4);
      break;
    default:
      hipLaunchKernelGGL((k_adj_ssor_step<M_NAGEX>), dim3(p.ntiles), dim3(WG), 0, st, p, omega, alpha, m, i, a, f, u,
                         v, ub, vb, ub_out, vb_out, fb, partial4);
      break;
  }
}

}  // namespace rmk
