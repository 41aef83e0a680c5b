// tensor.hip - the tensor track: environment sums, the Clebsch-Gordan tensor
// product with its pre-fused coupling table, linear channel mixing, and their
// adjoints.  All FP32.
//
// Eq. tp (section "Allegro: Scalable Equivariant Deep Learning"): the features
// of pair (i, j) are coupled with a weighted sum over the neighbours k of the
// same centre i; bilinearity lets the sum over k be taken first, once per
// centre:
//   Gamma_i[b][u] = c sum_{k in N(i)} w^{ik}[l(b)][u] Y^{ik}[b]        (env kernel)
//   T[e][c][u]    = sum_{a,b} W[a][b][c] V[e][a][u] Gamma_{i(e)}[b][u]   (tensor product)
// W is the path-weighted sum of the real Gaunt tables (section "Optimized
// tensor product": one contraction over the strided components instead of one
// per path); its sparsity pattern is a compile-time constant, so each (edge,
// channel) pair executes only the non-zero multiply-adds.
// Linear channel mixing: V^L[e][c][v] = sum_u M_{l(c)}[v][u] T[e][c][u] / sqrt(n),
// a dense contraction over channels run on FP32 MFMA.
//
// Work mapping.  Per-centre kernels (environment sums and the tensor-product
// adjoint, which both reduce over a centre's edges) give one wavefront to one
// centre: lane = channel u (+ edge sub-group when n < 64), so every reduction
// over the segment stays in registers and is deterministic.  Edge-tile
// kernels (tensor product + mixing) stage a tile of T in LDS and feed MFMA.
#include <utility>

#include "coupling.h"
#include "devutil.h"
#include "internal.h"

namespace allegro {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int lof(int c) { return c == 0 ? 0 : (c < 4 ? 1 : 2); }

template <int LMAX>
__device__ __forceinline__ void load_v(const VSrc& v, const float* eb_e, int64_t e, int u, int n,
                                       float* V) {
  constexpr int DIM = (LMAX + 1) * (LMAX + 1);
  const float* p = v.p + (size_t)e * v.ld + u;
  if (v.from_a0) {
    float a0[LMAX + 1];
#pragma unroll
    for (int l = 0; l <= LMAX; ++l) a0[l] = p[l * n];
#pragma unroll
    for (int c = 0; c < DIM; ++c) V[c] = a0[lof(c)] * eb_e[c];
  } else {
#pragma unroll
    for (int c = 0; c < DIM; ++c) V[c] = p[c * n];
  }
}

// ---------------------------------------------------------------------------
// Environment sums: one wavefront per centre.
template <int LMAX>
__global__ __launch_bounds__(256) void k_env(TensorArgs a) {
  constexpr int DIM = (LMAX + 1) * (LMAX + 1);
  const int lane = lane_id();
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= a.n_centres) return;
  const int n = a.n, G = kWave / n, u = lane & (n - 1), g = lane / n;
  float acc[DIM];
#pragma unroll
  for (int b = 0; b < DIM; ++b) acc[b] = 0.0f;
  for (int e = a.row_ptr[c] + g; e < a.row_ptr[c + 1]; e += G) {
    const float* w = a.w_env + (size_t)e * a.ld_w + u;
    const float* Y = a.eb + (size_t)e * kEB;
    float wl[LMAX + 1];
#pragma unroll
    for (int l = 0; l <= LMAX; ++l) wl[l] = w[l * n];
#pragma unroll
    for (int b = 0; b < DIM; ++b) acc[b] = fmaf(wl[lof(b)], Y[b], acc[b]);
  }
#pragma unroll
  for (int b = 0; b < DIM; ++b) acc[b] = group_cross_sum(acc[b], n);
  if (g == 0) {
    float* out = a.gam + (size_t)c * DIM * n + u;
#pragma unroll
    for (int b = 0; b < DIM; ++b) out[b * n] = acc[b] * a.c_norm;
  }
}

// ---------------------------------------------------------------------------
// Edge-tile kernels staging a [DIM][TT][n] block in LDS, then mixing channels
// on MFMA.  B operands are the packed mixing matrices (one per l).
constexpr int TT = 32;

__device__ __forceinline__ f32x4 mma8(const float* a, const float* b, f32x4 c) {
  // the K = 32 block as eight K = 4 steps (lane group g holds k = 8 g + s)
#pragma unroll
  for (int s = 0; s < 8; ++s) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], b[s], c, 0, 0, 0);
  return c;
}

// out[e][c][v] = scale * sum_k S[c][e][k] B_{l(c)}[k][v]   for the tile rows
template <int DIM>
__device__ void mix_tile(const float* S, int lds_ld, const float* Bbase, int b_stride, int n, int Kp,
                         int Np, float scale, float* out, int64_t e0, int E) {
  const int wave = threadIdx.x >> 6, lane = lane_id();
  const int nct = Np >> 4, nkb = Kp >> 5;
  const int items = DIM * nct;
  for (int it = wave; it < items; it += 4) {
    const int c = it / nct, nt = it - c * nct;
    const float* B = Bbase + (size_t)lof(c) * b_stride;
    f32x4 acc[2] = {f32x4{0, 0, 0, 0}, f32x4{0, 0, 0, 0}};
    for (int kb = 0; kb < nkb; ++kb) {
      float bf[8], af0[8], af1[8];
      const float* bp = B + ((size_t)(nt * nkb + kb) * 64 + lane) * 8;
#pragma unroll
      for (int s = 0; s < 8; ++s) bf[s] = bp[s];
      const float* ap = S + (size_t)c * TT * lds_ld + (lane & 15) * lds_ld + kb * 32 + 8 * (lane >> 4);
#pragma unroll
      for (int s = 0; s < 8; ++s) { af0[s] = ap[s]; af1[s] = ap[16 * lds_ld + s]; }
      acc[0] = mma8(af0, bf, acc[0]);
      acc[1] = mma8(af1, bf, acc[1]);
    }
    const int col = nt * 16 + (lane & 15);
    if (col < n) {
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = rt * 16 + 4 * (lane >> 4) + i;
          if (e0 + r < E) out[((size_t)(e0 + r) * DIM + c) * n + col] = acc[rt][i] * scale;
        }
    }
  }
}

// Tensor product (non-final layers) + channel mixing -> V^L.
template <int LMAX>
__global__ __launch_bounds__(256) void k_tp_mix(TensorArgs a, int lds_ld, int Kp, int Np) {
  using Pat = TpPattern<LMAX, false>;
  constexpr int DIM = Pat::DIM;
  extern __shared__ __align__(16) float S[];   // [DIM][TT][lds_ld]
  const int64_t e0 = (int64_t)blockIdx.x * TT;
  const int n = a.n;
  float w[Pat::NNZ];
#pragma unroll
  for (int k = 0; k < Pat::NNZ; ++k) w[k] = a.tpw[k];
  for (int p = threadIdx.x; p < TT * Kp; p += 256) {
    const int r = p / Kp, u = p - r * Kp;
    const int64_t e = e0 + r;
    float T[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) T[c] = 0.0f;
    if (e < a.E && u < n) {
      const float* Y = a.eb + (size_t)e * kEB;
      float V[DIM], G[DIM];
      load_v<LMAX>(a.v, Y, e, u, n, V);
      const float* gp = a.gam + (size_t)(a.ei[e] - a.centre_base) * DIM * n + u;
#pragma unroll
      for (int b = 0; b < DIM; ++b) G[b] = gp[b * n];
      tp_forward<Pat>(V, G, T, w, std::make_index_sequence<Pat::NNZ>{});
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) S[((size_t)c * TT + r) * lds_ld + u] = T[c];
  }
  __syncthreads();
  if (a.channel_mix) {
    mix_tile<DIM>(S, lds_ld, (const float*)a.mixB, a.mix_stride, n, Kp, Np, a.mix_scale, a.v_out, e0, a.E);
  } else {
    for (int p = threadIdx.x; p < TT * DIM * n; p += 256) {
      const int r = p / (DIM * n), rem = p - r * DIM * n, c = rem / n, u = rem - c * n;
      if (e0 + r < a.E) a.v_out[((size_t)(e0 + r) * DIM + c) * n + u] = S[((size_t)c * TT + r) * lds_ld + u];
    }
  }
}

// Adjoint of channel mixing for a non-final layer.  dE/dV^L is rebuilt from
// the final layer: dE/dV[a][u] = w_a Gamma'[a][u] dE/dT'[u] (+ dE/ds at a = 0).
template <int LMAX>
__global__ __launch_bounds__(256) void k_mix_adjoint(TensorArgs a, int lds_ld, int Kp, int Np) {
  constexpr int DIM = (LMAX + 1) * (LMAX + 1);
  extern __shared__ __align__(16) float S[];
  const int64_t e0 = (int64_t)blockIdx.x * TT;
  const int n = a.n;
  for (int p = threadIdx.x; p < TT * Kp; p += 256) {
    const int r = p / Kp, u = p - r * Kp;
    const int64_t e = e0 + r;
    float gV[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) gV[c] = 0.0f;
    if (e < a.E && u < n) {
      const float gt = a.g_tnext[(size_t)e * n + u];
      const float* gp = a.gam_next + (size_t)(a.ei[e] - a.centre_base) * DIM * n + u;
#pragma unroll
      for (int c = 0; c < DIM; ++c) gV[c] = a.tp_wnext[c] * gp[c * n] * gt;
      gV[0] += a.g_s[(size_t)e * n + u];
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) S[((size_t)c * TT + r) * lds_ld + u] = gV[c];
  }
  __syncthreads();
  if (a.channel_mix) {
    mix_tile<DIM>(S, lds_ld, (const float*)a.mixB, a.mix_stride, n, Kp, Np, a.mix_scale, a.g_tout, e0, a.E);
  } else {
    for (int p = threadIdx.x; p < TT * DIM * n; p += 256) {
      const int r = p / (DIM * n), rem = p - r * DIM * n, c = rem / n, u = rem - c * n;
      if (e0 + r < a.E) a.g_tout[((size_t)(e0 + r) * DIM + c) * n + u] = S[((size_t)c * TT + r) * lds_ld + u];
    }
  }
}

// ---------------------------------------------------------------------------
// Adjoint of the tensor product and the environment sum: one wavefront per
// centre.  Pass 1 accumulates dE/dGamma over the centre's edges (and, when V
// is built from a0 Y, emits dE/da0 and that part of dE/dY).  Pass 2 emits
// dE/dw and the environment part of dE/dY.
template <int LMAX, bool FINAL>
__global__ __launch_bounds__(256) void k_tp_env_adjoint(TensorArgs a) {
  using Pat = TpPattern<LMAX, FINAL>;
  constexpr int DIM = Pat::DIM, DOUT = Pat::DOUT;
  const int lane = lane_id();
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= a.n_centres) return;
  const int n = a.n, G = kWave / n, u = lane & (n - 1), g = lane / n;
  float w[Pat::NNZ];
#pragma unroll
  for (int k = 0; k < Pat::NNZ; ++k) w[k] = a.tpw[k];
  float Gm[DIM], gG[DIM];
  {
    const float* gp = a.gam + (size_t)c * DIM * n + u;
#pragma unroll
    for (int b = 0; b < DIM; ++b) { Gm[b] = gp[b * n]; gG[b] = 0.0f; }
  }
  const int eb0 = a.row_ptr[c], eb1 = a.row_ptr[c + 1];
  const int ntrip = (eb1 - eb0 + G - 1) / G;   // uniform trip count within the wave
  for (int t = 0; t < ntrip; ++t) {
    const int e = eb0 + g + t * G;
    const bool act = e < eb1;
    const float* Y = a.eb + (size_t)(act ? e : eb0) * kEB;
    float V[DIM], gT[DOUT];
    if (act) {
      load_v<LMAX>(a.v, Y, e, u, n, V);
      const float* gtp = a.g_t + (size_t)e * DOUT * n + u;
#pragma unroll
      for (int k = 0; k < DOUT; ++k) gT[k] = gtp[k * n];
    } else {
#pragma unroll
      for (int k = 0; k < DIM; ++k) V[k] = 0.0f;
#pragma unroll
      for (int k = 0; k < DOUT; ++k) gT[k] = 0.0f;
    }
    tp_adjoint_g<Pat>(V, gT, gG, w, std::make_index_sequence<Pat::NNZ>{});
    if (a.v.from_a0) {
      float gV[DIM];
#pragma unroll
      for (int k = 0; k < DIM; ++k) gV[k] = 0.0f;
      tp_adjoint_v<Pat>(Gm, gT, gV, w, std::make_index_sequence<Pat::NNZ>{});
      const float* a0 = a.v.p + (size_t)(act ? e : eb0) * a.v.ld + u;
      float ga[LMAX + 1];
#pragma unroll
      for (int l = 0; l <= LMAX; ++l) ga[l] = 0.0f;
      float gy[DIM];
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        ga[lof(k)] = fmaf(gV[k], Y[k], ga[lof(k)]);
        gy[k] = group_inner_sum(act ? gV[k] * a0[lof(k) * n] : 0.0f, n);
      }
      if (act) {
#pragma unroll
        for (int l = 0; l <= LMAX; ++l) a.g_a0[(size_t)e * a.ld_gw + l * n + u] = ga[l];
        if (u == 0) {
          float* o = a.g_Y + (size_t)e * 9;
#pragma unroll
          for (int k = 0; k < DIM; ++k) o[k] = (a.gy_accum ? o[k] : 0.0f) + gy[k];
        }
      }
    }
  }
#pragma unroll
  for (int b = 0; b < DIM; ++b) gG[b] = group_cross_sum(gG[b], n);
  const bool keep_gy = a.gy_accum || a.v.from_a0;
  for (int t = 0; t < ntrip; ++t) {
    const int e = eb0 + g + t * G;
    const bool act = e < eb1;
    const int ee = act ? e : eb0;
    const float* Y = a.eb + (size_t)ee * kEB;
    const float* wv = a.w_env + (size_t)ee * a.ld_w + u;
    float gw[LMAX + 1];
#pragma unroll
    for (int l = 0; l <= LMAX; ++l) gw[l] = 0.0f;
    float gy[DIM];
#pragma unroll
    for (int b = 0; b < DIM; ++b) {
      gw[lof(b)] = fmaf(gG[b], Y[b], gw[lof(b)]);
      gy[b] = group_inner_sum(act ? gG[b] * wv[lof(b) * n] : 0.0f, n);
    }
    if (act) {
#pragma unroll
      for (int l = 0; l <= LMAX; ++l) a.g_w[(size_t)e * a.ld_gw + l * n + u] = gw[l] * a.c_norm;
      if (u == 0) {
        float* o = a.g_Y + (size_t)e * 9;
#pragma unroll
        for (int b = 0; b < DIM; ++b) o[b] = (keep_gy ? o[b] : 0.0f) + gy[b] * a.c_norm;
#pragma unroll
        for (int b = DIM; b < 9; ++b) o[b] = 0.0f;
      }
    }
  }
}

inline unsigned blocks(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

void mix_dims(int n, int dim, int* lds_ld, int* Kp, int* Np, size_t* bytes) {
  *Kp = ((n + 31) / 32) * 32;
  *Np = ((n + 31) / 32) * 32;
  *lds_ld = *Kp + 4;
  *bytes = (size_t)dim * TT * (*lds_ld) * sizeof(float);
}

template <class K>
hipError_t launch_lds(K kern, unsigned grid, size_t bytes, hipStream_t s, const TensorArgs& a, int ld, int Kp,
                      int Np) {
  hipError_t st = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (st != hipSuccess) return st;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(256), bytes, s, a, ld, Kp, Np);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_env(const TensorArgs& a, hipStream_t s) {
  if (a.n_centres <= 0) return hipSuccess;
  if (a.l_max == 1) hipLaunchKernelGGL(k_env<1>, dim3(blocks(a.n_centres, 4)), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_env<2>, dim3(blocks(a.n_centres, 4)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_tp_mix(const TensorArgs& a, bool final_layer, hipStream_t s) {
  if (final_layer) return hipErrorInvalidValue;   // the final layer is fused into the last MLP
  if (a.E <= 0) return hipSuccess;
  const int dim = (a.l_max + 1) * (a.l_max + 1);
  int ld, Kp, Np;
  size_t bytes;
  mix_dims(a.n, dim, &ld, &Kp, &Np, &bytes);
  if (a.l_max == 1) return launch_lds(k_tp_mix<1>, blocks(a.E, TT), bytes, s, a, ld, Kp, Np);
  return launch_lds(k_tp_mix<2>, blocks(a.E, TT), bytes, s, a, ld, Kp, Np);
}

hipError_t launch_mix_adjoint(const TensorArgs& a, hipStream_t s) {
  if (a.E <= 0) return hipSuccess;
  const int dim = (a.l_max + 1) * (a.l_max + 1);
  int ld, Kp, Np;
  size_t bytes;
  mix_dims(a.n, dim, &ld, &Kp, &Np, &bytes);
  if (a.l_max == 1) return launch_lds(k_mix_adjoint<1>, blocks(a.E, TT), bytes, s, a, ld, Kp, Np);
  return launch_lds(k_mix_adjoint<2>, blocks(a.E, TT), bytes, s, a, ld, Kp, Np);
}

hipError_t launch_tp_env_adjoint(const TensorArgs& a, bool final_layer, hipStream_t s) {
  if (a.n_centres <= 0) return hipSuccess;
  const dim3 grid(blocks(a.n_centres, 4)), block(256);
  if (a.l_max == 1) {
    if (final_layer) hipLaunchKernelGGL((k_tp_env_adjoint<1, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_tp_env_adjoint<1, false>), grid, block, 0, s, a);
  } else {
    if (final_layer) hipLaunchKernelGGL((k_tp_env_adjoint<2, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_tp_env_adjoint<2, false>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace allegro
