// devutil.h - small wavefront (64-lane) helpers for the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace allegro {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// Butterfly sum over all 64 lanes; every lane receives the same total.
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) v += __shfl_xor(v, off, kWave);
  return v;
}
__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) v += __shfl_xor(v, off, kWave);
  return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) v += __shfl_xor(v, off, kWave);
  return v;
}
// Inclusive prefix sum over the 64 lanes.
__device__ __forceinline__ int wave_incl_scan(int v) {
  const int l = lane_id();
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    int t = __shfl_up(v, off, kWave);
    if (l >= off) v += t;
  }
  return v;
}

// Sum over lanes that share (lane / width) groups: reduces across the
// kWave/width groups with the same lane % width, butterfly style.
__device__ __forceinline__ float group_cross_sum(float v, int width) {
  for (int off = width; off < kWave; off <<= 1) v += __shfl_xor(v, off, kWave);
  return v;
}
// Sum within aligned groups of `width` lanes (width a power of two <= 64).
__device__ __forceinline__ float group_inner_sum(float v, int width) {
  for (int off = 1; off < width; off <<= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Sums over aligned lane groups with DPP moves (no LDS traffic, fixed order).
// dpp_add<CTRL, ROWS>: v + (v moved by the DPP pattern CTRL) in the rows
// selected by ROWS, v elsewhere.
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ float dpp_add(float v) {
  const int t = __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xf, false);
  return v + __int_as_float(t);
}
constexpr int kDppXor1 = 0xB1;         // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;         // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;  // lane i <- 7 - i within 8
constexpr int kDppMirror = 0x140;      // lane i <- 15 - i within 16
constexpr int kDppBcast15 = 0x142;     // lane 15 of each row into the next row
constexpr int kDppBcast31 = 0x143;     // lane 31 into rows 2 and 3

// Sum over each group of N lanes (N = 8, 16, 32 or 64).  For N <= 16 every
// lane of the group holds the sum; for N = 32 / 64 the last lane of the group
// does.
template <int N>
__device__ __forceinline__ float group_sum_dpp(float v) {
  static_assert(N == 8 || N == 16 || N == 32 || N == 64, "group of 8, 16, 32 or 64 lanes");
  v = dpp_add<kDppXor1>(v);
  v = dpp_add<kDppXor2>(v);
  v = dpp_add<kDppHalfMirror>(v);
  if constexpr (N >= 16) v = dpp_add<kDppMirror>(v);
  if constexpr (N >= 32) v = dpp_add<kDppBcast15, 0xa>(v);
  if constexpr (N >= 64) v = dpp_add<kDppBcast31, 0xc>(v);
  return v;
}

// SiLU and its derivative with the hardware reciprocal (1 ulp) instead of an
// IEEE division.
__device__ __forceinline__ float sigmoid(float x) { return __builtin_amdgcn_rcpf(1.0f + __expf(-x)); }
__device__ __forceinline__ float silu(float x) { return x * sigmoid(x); }
__device__ __forceinline__ float silu_grad(float x) {
  const float s = sigmoid(x);
  return s * (1.0f + x * (1.0f - s));
}

}  // namespace allegro
