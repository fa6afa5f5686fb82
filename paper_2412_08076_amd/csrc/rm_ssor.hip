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
// One inner step per launch.  A workgroup owns a 64 x 32 tile.  Each of the six passes
// that read neighbours needs its inputs one ring further out than its own output, so the
// passes run on the tile plus a ring that shrinks from 6 (first pass) to 0 (last), and
// the residual is formed on a halo of 6 from a look-ahead field with a halo of 7.
// Points outside the domain hold 0 and are never updated (Dirichlet).  Temporal
// blocking would need a halo of 7 per step, so none is attempted.
//
// LDS layout.  The swept field is held as four colour planes: padded point (x, y) lives
// in plane (x mod 2, y mod 2) at index (y / 2) * QW + x / 2.  In a colour pass every
// neighbour of a point then sits at a fixed offset in one other plane, so consecutive
// lanes read and write consecutive words.  The look-ahead field and the residual share
// one buffer: the residual is held in registers across a barrier and then scattered
// into the planes, which keeps one workgroup at 14 KB of LDS in FP32.
#include "rm_device.h"

#pragma clang fp contract(off)

namespace rmk {

namespace {

constexpr int HR = 6;               // halo of the residual and of the first colour pass
constexpr int HU = HR + 1;          // halo of the field the residual is formed from
constexpr int RW = TX + 2 * HR;     // residual region 76 x 44
constexpr int RH = TY + 2 * HR;
constexpr int PW = RW + 2;          // plus one ring: 78 x 46, the look-ahead region
constexpr int PH = RH + 2;
constexpr int UW = TX + 2 * HU;
constexpr int UH = TY + 2 * HU;
constexpr int NW = WG / 64;
static_assert(UW == PW && UH == PH, "the padded region and the look-ahead region coincide");
static_assert(TX % 2 == 0 && TY % 2 == 0, "tile origins are even: the colour of a padded point is fixed");

// Colour planes of a padded (W + 2) x (H + 2) region (W, H even).
template <int W, int H>
struct Planes {
  static constexpr int QW = W / 2 + 1, QH = H / 2 + 1, QS = QW * QH, SIZE = 4 * QS;
  static __device__ __forceinline__ int at(int x, int y) {
    return ((y & 1) * 2 + (x & 1)) * QS + (y >> 1) * QW + (x >> 1);
  }
};

// One colour pass of the SSOR sweeps (FWD: the forward solve with D - aL, else the
// backward solve with D - aU) over the points of colour COL within h of the tile.  s
// holds the colour planes Q of a region whose padded point (x, y) is instance point
// (px0 + x, py0 + y), with px0 and py0 of parity OP (tile origins are even, so the
// parity is fixed per field and every plane offset below is a constant); the tile
// starts at padded (G, G).
template <typename T, typename Q, int G, int h, bool FWD, int COL, int OP>
__device__ __forceinline__ void ssor_pass(T* s, int px0, int py0, int n, const T c[5], T relax, T dinv) {
  constexpr int NX = TX / 2 + h, NY = TY / 2 + h;   // points of one colour per row, rows
  static_assert(G - h >= 1 && G + TX + h <= 2 * Q::QW - 1 && G + TY + h <= 2 * Q::QH - 1,
                "a pass and its neighbour reads stay inside the padded region");
  constexpr int a = (COL ^ OP) & 1, b = ((COL >> 1) ^ OP) & 1;   // plane of colour COL
  constexpr int lo = G - h;
  constexpr int i0 = (lo + ((lo ^ a) & 1)) >> 1, j0 = (lo + ((lo ^ b) & 1)) >> 1;
  constexpr int xm = a - 1, xp = a;                         // plane offsets of x - 1, x + 1
  constexpr int ym = (b - 1) * Q::QW, yp = b * Q::QW;       // and of y - 1, y + 1
  constexpr bool xn = FWD ? (COL & 1) != 0 : (COL & 1) == 0;
  constexpr bool yn = FWD ? COL >= 2 : COL < 2;
  T* q0 = s + (2 * b + a) * Q::QS;
  const T* qx = s + (2 * b + (a ^ 1)) * Q::QS;          // x-neighbours
  const T* qy = s + (2 * (b ^ 1) + a) * Q::QS;          // y-neighbours
  const T* qd = s + (2 * (b ^ 1) + (a ^ 1)) * Q::QS;    // diagonal neighbours
  for (int k = threadIdx.x; k < NX * NY; k += WG) {
    const int jj = k / NX, ii = k - jj * NX;
    const int i = i0 + ii, j = j0 + jj;
    const int gx = px0 + 2 * i + a, gy = py0 + 2 * j + b;
    if ((unsigned)gx >= (unsigned)n || (unsigned)gy >= (unsigned)n) continue;
    const int e = j * Q::QW + i;
    T acc = T(0);
    if (xn) acc = fmadd(c[1], qx[e + xm] + qx[e + xp], acc);
    if (yn) {
      acc = fmadd(c[2], qy[e + ym] + qy[e + yp], acc);
      acc = fmadd(c[3], qd[e + ym + xm] + qd[e + yp + xp], acc);   // (-1, -1) and (+1, +1)
      acc = fmadd(c[4], qd[e + ym + xp] + qd[e + yp + xm], acc);   // (+1, -1) and (-1, +1)
    }
    if (FWD)
      q0[e] = (q0[e] - relax * acc) * dinv;
    else
      q0[e] = fmadd(-(relax * dinv), acc, q0[e]);
  }
}

// The seven colour passes: forward colours 0..3, backward colours 2..0.  On entry s
// holds r on the tile plus a ring of h0 + 6; on exit it holds w (B^{-1} r = a (2 - a) w)
// on the tile plus a ring of h0.
template <typename T, typename Q, int G, int h0, int OP>
__device__ __forceinline__ void ssor_sweeps(T* s, int px0, int py0, int n, const T c[5], T relax, T dinv) {
  ssor_pass<T, Q, G, h0 + 6, true, 0, OP>(s, px0, py0, n, c, relax, dinv);
  __syncthreads();
  ssor_pass<T, Q, G, h0 + 5, true, 1, OP>(s, px0, py0, n, c, relax, dinv);
  __syncthreads();
  ssor_pass<T, Q, G, h0 + 4, true, 2, OP>(s, px0, py0, n, c, relax, dinv);
  __syncthreads();
  ssor_pass<T, Q, G, h0 + 3, true, 3, OP>(s, px0, py0, n, c, relax, dinv);
  __syncthreads();
  ssor_pass<T, Q, G, h0 + 2, false, 2, OP>(s, px0, py0, n, c, relax, dinv);
  __syncthreads();
  ssor_pass<T, Q, G, h0 + 1, false, 1, OP>(s, px0, py0, n, c, relax, dinv);
  __syncthreads();
  ssor_pass<T, Q, G, h0, false, 0, OP>(s, px0, py0, n, c, relax, dinv);
  __syncthreads();
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

// Residual r = f - A u~ on the padded region (0 on its outer ring and outside the
// domain), read from the look-ahead field s (row-major, UW wide), then written over s
// as colour planes Q.  Plane by plane (the plane's parities are constants), thread t
// forms the residual of plane elements e = t + j WG, so the write after the barrier goes
// to s[plane * QS + e] with no index arithmetic, and an element's padded point needs one
// division by the plane width.  Ends with a barrier.
template <typename T, typename Q>
__device__ __forceinline__ void residual_to_planes(T* s, const Field<T>& fi, int ox, int oy, int n, const T c[5]) {
  static_assert(Q::SIZE == PH * PW && 2 * Q::QW == PW && 2 * Q::QH == PH, "one plane element per padded point");
  constexpr int NE = (Q::QS + WG - 1) / WG;  // elements per thread and plane
  T rr[4][NE];
  const int t0 = opaque_tid();
#pragma unroll
  for (int pl = 0; pl < 4; ++pl) {
    const int a = pl & 1, b = pl >> 1;  // x and y parity of the plane's padded points
    T fv[NE];
    int kk[NE];  // row-major index of the element's point, or -1 where the residual is 0
#pragma unroll
    for (int j = 0; j < NE; ++j) {  // points not formed read f at 0
      const int e = t0 + j * WG;
      const int jj = e / Q::QW, i = e - jj * Q::QW;
      const int px = 2 * i + a, py = 2 * jj + b;
      const int gx = ox + px, gy = oy + py;
      // the outer ring: x = 0 (i = 0 of an even plane) or PW - 1 (the last i of an odd
      // one), likewise in y; and elements past the plane
      const bool ring = e >= Q::QS || i == (a ? Q::QW - 1 : 0) || jj == (b ? Q::QH - 1 : 0);
      const bool ok = !ring && (unsigned)gx < (unsigned)n && (unsigned)gy < (unsigned)n;
      kk[j] = ok ? py * PW + px : -1;
      fv[j] = fi[ok ? (unsigned)(gy * n + gx) : 0u];
    }
#pragma unroll
    for (int j = 0; j < NE; ++j) {
      // points not formed read the stencil at an interior point
      T st = stencil_at(s + (kk[j] >= 0 ? kk[j] : PW + 1), UW, c);
      // the stencil is complete before the next one's LDS reads are issued, so the
      // reads of one stencil at a time occupy registers
      asm volatile("" : "+v"(st)::"memory");
      rr[pl][j] = kk[j] >= 0 ? fv[j] - st : T(0);
    }
  }
  __syncthreads();
  const int t1 = opaque_tid();
#pragma unroll
  for (int pl = 0; pl < 4; ++pl)
#pragma unroll
    for (int j = 0; j < NE; ++j) {
      const int e = t1 + j * WG;
      if (e < Q::QS) s[pl * Q::QS + e] = rr[pl][j];
    }
  __syncthreads();
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
  using Q = Planes<RW, RH>;
  static_assert(Q::SIZE == UH * UW, "the planes and the look-ahead field share one buffer");
  __shared__ T s[UH * UW];
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
  const int nn = n * n;
  const Field<T> uf(u + in.off, nn), vf(v + in.off, nn), fi(f + in.off, nn);
  const int ox = tl.x0 - HU, oy = tl.y0 - HU;   // instance point of padded (0, 0)
  stage<T, UW, UH, false>(
      ox, oy, n,
      [&](unsigned idx) { return uses_lookahead(METHOD) ? fmadd(at, vf[idx], uf[idx]) : uf[idx]; },
      [&](int k, int, int, T val) { s[k] = val; });
  __syncthreads();
  residual_to_planes<T, Q>(s, fi, ox, oy, n, c);
  ssor_sweeps<T, Q, HU, 0, HU & 1>(s, ox, oy, n, c, relax, dinv);
  const T s2 = relax * (T(2) - relax);
  const int tx = threadIdx.x & 63, ty0 = threadIdx.x >> 6;
  const int gx = tl.x0 + tx;
  if (gx >= n) return;
  constexpr int NY = TY / NW;
  T uu[NY], vv[NY];
#pragma unroll
  for (int k = 0; k < NY; ++k) {   // rows below the domain load its last row
    const unsigned idx = (unsigned)(min(tl.y0 + ty0 + NW * k, n - 1) * n + gx);
    uu[k] = uf[idx];
    vv[k] = uses_momentum(METHOD) ? vf[idx] : T(0);
  }
  const Field<T> uo(u_out + in.off, nn), vo(v_out + in.off, nn);
#pragma unroll
  for (int k = 0; k < NY; ++k) {   // rows below the domain are dropped by the stores
    const int ly = ty0 + NW * k;
    const unsigned idx = (unsigned)((tl.y0 + ly) * n + gx);
    const T z = s2 * s[Q::at(tx + HU, ly + HU)];
    const T vn = uses_momentum(METHOD) ? fmadd(a, vv[k], w * z) : w * z;
    vo.store(idx, vn);
    uo.store(idx, uu[k] + vn);
  }
}

// Reverse of one SSOR-preconditioned step (B^{-1} is symmetric):
//   g = vb + ub;  r = f - A u~;  z = B^{-1} r;  rb = w B^{-1} g;  fb += rb;
//   ut_bar = -A rb;  ub' = ub + ut_bar;  vb' = a g + at ut_bar (NAG: a (g + ut_bar)).
// Per tile: <g, z>, <g, v>, <ut_bar, v>.  rb is needed on the tile and a one-point
// ring, so g is staged with a halo of HR + 1 and its sweeps end on a ring of 1.  The
// passes of the two SSOR applications share their barriers.
template <int METHOD>
__global__ __launch_bounds__(WG) void k_adj_ssor_step(PlanDev p, const float* __restrict__ omega,
                                                      const float* __restrict__ alpha, int m, int i, float relax,
                                                      const float* __restrict__ f, const float* __restrict__ u,
                                                      const float* __restrict__ v, const float* __restrict__ ub,
                                                      const float* __restrict__ vb, float* __restrict__ ub_out,
                                                      float* __restrict__ vb_out, float* __restrict__ fb,
                                                      double* __restrict__ partial4) {
  using Q = Planes<RW, RH>;
  using QG = Planes<TX + 2 * (HR + 1), TY + 2 * (HR + 1)>;   // g region (halo 7) and its ring
  constexpr int GPW = 2 * QG::QW, GPH = 2 * QG::QH;
  constexpr int GG = HR + 2;                                  // tile origin in the padded g region
  __shared__ float s[UH * UW];
  __shared__ float sg[QG::SIZE];
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
  const int nn = n * n;
  const Field<float> uf(u + in.off, nn), vf(v + in.off, nn), ubf(ub + in.off, nn), vbf(vb + in.off, nn);
  const Field<float> fi(f + in.off, nn), fbf(fb != nullptr ? fb + in.off : ub + in.off, nn);
  const int ox = tl.x0 - HU, oy = tl.y0 - HU;
  const int gox = tl.x0 - GG, goy = tl.y0 - GG;
  stage<float, UW, UH, false>(
      ox, oy, n,
      [&](unsigned idx) { return uses_lookahead(METHOD) ? fmadd(at, vf[idx], uf[idx]) : uf[idx]; },
      [&](int k, int, int, float val) { s[k] = val; });
  stage<float, GPW, GPH, true>(
      gox, goy, n, [&](unsigned idx) { return uses_momentum(METHOD) ? vbf[idx] + ubf[idx] : ubf[idx]; },
      [&](int, int x, int y, float val) { sg[QG::at(x, y)] = val; });
  __syncthreads();
  residual_to_planes<float, Q>(s, fi, ox, oy, n, c);
  ssor_pass<float, Q, HU, 6, true, 0, HU & 1>(s, ox, oy, n, c, relax, dinv);
  ssor_pass<float, QG, GG, 7, true, 0, GG & 1>(sg, gox, goy, n, c, relax, dinv);
  __syncthreads();
  ssor_pass<float, Q, HU, 5, true, 1, HU & 1>(s, ox, oy, n, c, relax, dinv);
  ssor_pass<float, QG, GG, 6, true, 1, GG & 1>(sg, gox, goy, n, c, relax, dinv);
  __syncthreads();
  ssor_pass<float, Q, HU, 4, true, 2, HU & 1>(s, ox, oy, n, c, relax, dinv);
  ssor_pass<float, QG, GG, 5, true, 2, GG & 1>(sg, gox, goy, n, c, relax, dinv);
  __syncthreads();
  ssor_pass<float, Q, HU, 3, true, 3, HU & 1>(s, ox, oy, n, c, relax, dinv);
  ssor_pass<float, QG, GG, 4, true, 3, GG & 1>(sg, gox, goy, n, c, relax, dinv);
  __syncthreads();
  ssor_pass<float, Q, HU, 2, false, 2, HU & 1>(s, ox, oy, n, c, relax, dinv);
  ssor_pass<float, QG, GG, 3, false, 2, GG & 1>(sg, gox, goy, n, c, relax, dinv);
  __syncthreads();
  ssor_pass<float, Q, HU, 1, false, 1, HU & 1>(s, ox, oy, n, c, relax, dinv);
  ssor_pass<float, QG, GG, 2, false, 1, GG & 1>(sg, gox, goy, n, c, relax, dinv);
  __syncthreads();
  ssor_pass<float, Q, HU, 0, false, 0, HU & 1>(s, ox, oy, n, c, relax, dinv);
  ssor_pass<float, QG, GG, 1, false, 0, GG & 1>(sg, gox, goy, n, c, relax, dinv);
  __syncthreads();
  const float s2 = relax * (2.f - relax);
  double pw = 0.0, pg = 0.0, pl = 0.0;
  const int tx = threadIdx.x & 63, ty0 = threadIdx.x >> 6;
  const int gx = tl.x0 + tx;
  if (gx < n) {
    constexpr int NY = TY / NW;
    float ubr[NY], vr[NY], vbr[NY], fbr[NY];
#pragma unroll
    for (int k = 0; k < NY; ++k) {   // rows below the domain load its last row
      const unsigned idx = (unsigned)(min(tl.y0 + ty0 + NW * k, n - 1) * n + gx);
      ubr[k] = ubf[idx];
      vr[k] = uses_momentum(METHOD) ? vf[idx] : 0.f;
      vbr[k] = uses_momentum(METHOD) ? vbf[idx] : 0.f;
      fbr[k] = fb != nullptr ? fbf[idx] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < NY; ++k) {
      const int ly = ty0 + NW * k, gy = tl.y0 + ly;
      if (gy >= n) break;
      const int64_t idx = in.off + (int64_t)gy * n + gx;
      const float z = s2 * s[Q::at(tx + HU, ly + HU)];
      const int x = tx + GG, y = ly + GG;   // w_g at this point and its ring
      // rb = w s2 w_g at the point and its ring; ut_bar = -A rb
      const float wsc = w * s2;
      const float g0 = sg[QG::at(x, y)];
      float acc = c[0] * (wsc * g0);
      acc = fmadd(c[1], wsc * sg[QG::at(x - 1, y)] + wsc * sg[QG::at(x + 1, y)], acc);
      acc = fmadd(c[2], wsc * sg[QG::at(x, y - 1)] + wsc * sg[QG::at(x, y + 1)], acc);
      acc = fmadd(c[3], wsc * sg[QG::at(x - 1, y - 1)] + wsc * sg[QG::at(x + 1, y + 1)], acc);
      acc = fmadd(c[4], wsc * sg[QG::at(x + 1, y - 1)] + wsc * sg[QG::at(x - 1, y + 1)], acc);
      const float utb = -acc;
      const float ubv = ubr[k];
      const float vv = vr[k];
      const float g = uses_momentum(METHOD) ? vbr[k] + ubv : ubv;
      pw += (double)g * (double)z;
      pg += (double)g * (double)vv;
      pl += (double)utb * (double)vv;
      ub_out[idx] = ubv + utb;
      if (METHOD == M_NAG) vb_out[idx] = a * (g + utb);
      if (METHOD == M_MOM) vb_out[idx] = a * g;
      if (METHOD == M_NAGEX) vb_out[idx] = fmadd(at, utb, a * g);
      if (fb != nullptr) fb[idx] = fbr[k] + wsc * g0;
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
