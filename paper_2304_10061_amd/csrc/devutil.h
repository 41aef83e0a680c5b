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

// SiLU and its derivative with the hardware reciprocal (1 ulp) instead of an
// IEEE division.
__device__ __forceinline__ float sigmoid(float x) { return __builtin_amdgcn_rcpf(1.0f + __expf(-x)); }
__device__ __forceinline__ float silu(float x) { return x * sigmoid(x); }
__device__ __forceinline__ float silu_grad(float x) {
  const float s = sigmoid(x);
  return s * (1.0f + x * (1.0f - s));
}

}  // namespace allegro
