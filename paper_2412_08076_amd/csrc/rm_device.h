// Device helpers shared by the kernel files (internal).  Every kernel that evaluates
// the stencil uses stencil9's fixed order of operations, so different kernels that
// apply the same update produce the same bits.
#pragma once

#include "rm_internal.h"

namespace rmk {
namespace {

__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Tile tables are padded to a multiple of 8 entries; hardware dispatches workgroups
// round robin over the 8 XCDs, so XCD k (blocks bid = k mod 8) takes the contiguous
// range [k * nb / 8, (k + 1) * nb / 8) and neighbouring tiles share one L2.
__device__ __forceinline__ int xcd_remap(int bid, int nb) {
  const int per = nb >> 3;
  return (bid & 7) * per + (bid >> 3);
}

// Weighted 9-point sum in a fixed order: C centre, W/E = x -+ 1, S/N = y -+ 1, then
// the diagonal pairs (1,1)/(-1,-1) and (-1,1)/(1,-1).
template <typename T>
__device__ __forceinline__ T stencil9(const T c[5], T C, T W, T E, T S, T N, T SW, T NE, T SE, T NW) {
#pragma clang fp contract(off)
  T acc = c[0] * C;
  acc = fmadd(c[1], W + E, acc);
  acc = fmadd(c[2], S + N, acc);
  acc = fmadd(c[3], SW + NE, acc);
  acc = fmadd(c[4], SE + NW, acc);
  return acc;
}

// f - sum_j c_j s_j, the residual of a 9-point stencil, in the one order every FP32
// sweep kernel and the residual kernels use: starting from f, subtract the south row
// (S, SW, SE), then the centre row (C, then the pair W + E), then the north row (N, NE,
// NW) -- the order in which a row pipeline receives the rows -- each as a fused
// multiply-add.  Coefficients as in stencil9: c2 for S and N, c3 for SW and NE, c4 for
// SE and NW.  Kernels that form the same residual in this order agree bit for bit.
template <typename T>
__device__ __forceinline__ T residual9(const T c[5], T f, T C, T W, T E, T S, T N, T SW, T NE, T SE, T NW) {
#pragma clang fp contract(off)
  T acc = fmadd(-c[2], S, f);
  acc = fmadd(-c[3], SW, acc);
  acc = fmadd(-c[4], SE, acc);
  acc = fmadd(-c[0], C, acc);
  acc = fmadd(-c[1], W + E, acc);
  acc = fmadd(-c[2], N, acc);
  acc = fmadd(-c[3], NE, acc);
  return fmadd(-c[4], NW, acc);
}

// New momentum of a Table-1 step, v' = a v + w (f - A s) with the residual of
// residual9; c, w and a are the same for every point of a workgroup, so they stay in
// scalar registers.
__device__ __forceinline__ float step_vf(const float c[5], float w, float a, float f, float v, float C, float W,
                                         float E, float S, float N, float SW, float NE, float SE, float NW) {
#pragma clang fp contract(off)
  return fmadd(a, v, w * residual9<float>(c, f, C, W, E, S, N, SW, NE, SE, NW));
}

// A value the whole workgroup shares, moved to a scalar register (for values formed by
// vector arithmetic on scalar inputs, which would otherwise occupy a vector register).
__device__ __forceinline__ float uniform_f32(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

// The five stencil coefficients of instance b in the precision of T.
template <typename T>
__device__ __forceinline__ void load_coef(const PlanDev& p, int b, T c[5]);
template <>
__device__ __forceinline__ void load_coef<float>(const PlanDev& p, int b, float c[5]) {
#pragma unroll
  for (int k = 0; k < 5; ++k) c[k] = p.coef32[b * 8 + k];
}
template <>
__device__ __forceinline__ void load_coef<double>(const PlanDev& p, int b, double c[5]) {
#pragma unroll
  for (int k = 0; k < 5; ++k) c[k] = p.coef64[b * 8 + k];
}

// Sum over a workgroup of WG threads in a fixed order (shuffle tree per wave, then the
// waves in order); the result is valid in thread 0.  Safe to call repeatedly.
__device__ __forceinline__ double block_sum(double x, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = x;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < WG / 64; ++k) r += sh[k];
  }
  return r;
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// An instance field read through a buffer resource: a 32-bit offset from a uniform
// base, so an address costs one register.  The byte size (at most 2^31 for an FP64
// field of the largest instance) is formed unsigned; the hardware reads the record
// count and the offsets as unsigned 32-bit values.
template <typename T>
struct Field {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ Field(const T* base, int count)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), (short)0,
                                            (int)((unsigned)count * (unsigned)sizeof(T)), 0x00020000)) {}
  __device__ __forceinline__ T operator[](unsigned idx) const {
    if constexpr (sizeof(T) == 4) {
      return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)(idx * 4u), 0, 0));
    } else {
      const auto w = __builtin_amdgcn_raw_buffer_load_b64(r, (int)(idx * 8u), 0, 0);
      return __hiloint2double((int)w[1], (int)w[0]);
    }
  }
  // A store at idx >= count is dropped by the hardware.
  __device__ __forceinline__ void store(unsigned idx, T x) const {
    if constexpr (sizeof(T) == 4) {
      __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), r, (int)(idx * 4u), 0, 0);
    } else {
      typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
      const long long b = __double_as_longlong(x);
      const u32x2 w = {(unsigned)b, (unsigned)(b >> 32)};
      __builtin_amdgcn_raw_buffer_store_b64(w, r, (int)(idx * 8u), 0, 0);
    }
  }
};

// Global loads a thread keeps in flight while staging.
constexpr int kLoadBatch = 8;

// The thread index through an opaque copy: index arithmetic derived from it is not
// merged with the same arithmetic of an earlier phase, whose results would otherwise
// stay live (in registers) from one phase to the next.
__device__ __forceinline__ int opaque_tid() {
  int t;
  asm volatile("v_mov_b32 %0, %1" : "=v"(t) : "v"((int)threadIdx.x));
  return t;
}

// Stages a W x H region whose point (x, y) is point (ox + x, oy + y) of an n x n field
// into LDS (a workgroup of WG threads): put(k, x, y, load(idx)) at flat position
// k = y W + x, with the value 0 outside the field (and, with RING, on the region's
// outer ring).  Every global load takes an in-bounds index (0 stands in for points
// that are not loaded) and sits behind no branch, so the loads of a batch are all in
// flight before the first is used.
template <typename T, int W, int H, bool RING, typename Load, typename Put>
__device__ __forceinline__ void stage(int ox, int oy, int n, Load load, Put put) {
  constexpr int NK = W * H, NU = (NK + WG - 1) / WG;
#pragma unroll
  for (int j0 = 0; j0 < NU; j0 += kLoadBatch) {
    T val[kLoadBatch];
    const int t0 = opaque_tid();
#pragma unroll
    for (int j = 0; j < kLoadBatch && j0 + j < NU; ++j) {
      const int k = t0 + (j0 + j) * WG;
      const int y = k / W, x = k - y * W;
      const int gx = ox + x, gy = oy + y;
      bool ok = (unsigned)gx < (unsigned)n && (unsigned)gy < (unsigned)n;
      if (RING) ok = ok && x > 0 && y > 0 && x < W - 1 && y < H - 1;
      const T t = load(ok ? (unsigned)(gy * n + gx) : 0u);
      val[j] = ok ? t : T(0);
    }
    const int t1 = opaque_tid();
#pragma unroll
    for (int j = 0; j < kLoadBatch && j0 + j < NU; ++j) {
      const int k = t1 + (j0 + j) * WG;
      const int y = k / W, x = k - y * W;
      if (k < NK) put(k, x, y, val[j]);
    }
  }
}

}  // namespace
}  // namespace rmk
