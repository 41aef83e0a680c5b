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

__device__ __forceinline__ f32x4 mma8(const float* a, const float* b, f32x4 c) {
  // the K = 32 block as eight K = 4 steps (lane group g holds k = 8 g + s)
#pragma unroll
  for (int s = 0; s < 8; ++s) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], b[s], c, 0, 0, 0);
  return c;
}

// out[e][c][v] = scale * sum_k S[c][e][k] B_{l(c)}[k][v]   for the tile rows.
// Work items (c, column tile) are dealt to the four waves; the B fragments of
// the next item are loaded while the current one runs on the matrix cores.
template <int DIM, int TT>
__device__ void mix_tile(const float* S, int lds_ld, const float* Bbase, int b_stride, int n, int Kp,
                         int Np, float scale, float* out, int64_t e0, int E) {
  constexpr int RT = TT / 16;
  constexpr int MAXKB = 2;   // K = n <= 64
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = lane_id();
  const int nct = Np >> 4, nkb = Kp >> 5;
  const int items = DIM * nct;
  float bc[MAXKB][8], bn[MAXKB][8];
  auto load_b = [&](int it, float (&dst)[MAXKB][8]) {
    const int c = it / nct, nt = it - c * nct;
    const float* B = Bbase + (size_t)lof(c) * b_stride;
#pragma unroll
    for (int kb = 0; kb < MAXKB; ++kb)
      if (kb < nkb) {
        const float* bp = B + ((size_t)(nt * nkb + kb) * 64 + lane) * 8;
#pragma unroll
        for (int s = 0; s < 8; ++s) dst[kb][s] = bp[s];
      }
  };
  if (wave < items) load_b(wave, bc);
  for (int it = wave; it < items; it += 4) {
    if (it + 4 < items) load_b(it + 4, bn);
    const int c = it / nct, nt = it - c * nct;
    f32x4 acc[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) acc[rt] = f32x4{0, 0, 0, 0};
#pragma unroll
    for (int kb = 0; kb < MAXKB; ++kb) {
      if (kb < nkb) {
        const float* ap = S + (size_t)c * TT * lds_ld + (lane & 15) * lds_ld + kb * 32 + 8 * (lane >> 4);
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
          // two 16-byte LDS reads (row stride = 4 mod 64 banks: conflict-free)
          const float4 lo = *(const float4*)(ap + rt * 16 * lds_ld);
          const float4 hi = *(const float4*)(ap + rt * 16 * lds_ld + 4);
          const float af[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
          acc[rt] = mma8(af, bc[kb], acc[rt]);
        }
      }
    }
    const int col = nt * 16 + (lane & 15);
    if (col < n) {
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = rt * 16 + 4 * (lane >> 4) + i;
          if (e0 + r < E) out[((size_t)(e0 + r) * DIM + c) * n + col] = acc[rt][i] * scale;
        }
    }
#pragma unroll
    for (int kb = 0; kb < MAXKB; ++kb)
#pragma unroll
      for (int s = 0; s < 8; ++s) bc[kb][s] = bn[kb][s];
  }
}

// Tensor product (non-final layers) + channel mixing -> V^L.
template <int LMAX, int TT>
__global__ __launch_bounds__(256) void k_tp_mix(TensorArgs a, int lds_ld, int Kp, int Np) {
  using Pat = TpPattern<LMAX, false>;
  constexpr int DIM = Pat::DIM;
  extern __shared__ __align__(16) float S[];   // [DIM][TT][lds_ld]
  const int64_t e0 = (int64_t)blockIdx.x * TT;
  const int n = a.n;
  const float* w = a.tpw_v;   // kernel-argument array: uniform, read with scalar loads
  // TT * Kp is a multiple of 512: two (edge, channel) items per thread per step,
  // loads of both issued before either is used
  for (int p0 = threadIdx.x; p0 < TT * Kp; p0 += 512) {
    float V[2][DIM], G[2][DIM];
    bool ok[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int p = p0 + 256 * h;
      const int r = p / Kp, u = p - r * Kp;
      const int64_t e = e0 + r;
      ok[h] = e < a.E && u < n;
      const int64_t ee = ok[h] ? e : 0;
      const int uu = ok[h] ? u : 0;
      load_v<LMAX>(a.v, a.eb + (size_t)ee * kEB, ee, uu, n, V[h]);
      const float* gp = a.gam + (size_t)(a.ei[ee] - a.centre_base) * DIM * n + uu;
#pragma unroll
      for (int b = 0; b < DIM; ++b) G[h][b] = gp[b * n];
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int p = p0 + 256 * h;
      const int r = p / Kp, u = p - r * Kp;
      float T[DIM];
#pragma unroll
      for (int c = 0; c < DIM; ++c) T[c] = 0.0f;
      if (ok[h]) tp_forward<Pat>(V[h], G[h], T, w, std::make_index_sequence<Pat::NNZ>{});
#pragma unroll
      for (int c = 0; c < DIM; ++c) S[((size_t)c * TT + r) * lds_ld + u] = T[c];
    }
  }
  __syncthreads();
  if (a.channel_mix) {
    mix_tile<DIM, TT>(S, lds_ld, (const float*)a.mixB, a.mix_stride, n, Kp, Np, a.mix_scale, a.v_out, e0, a.E);
  } else {
    for (int p = threadIdx.x; p < TT * DIM * n; p += 256) {
      const int r = p / (DIM * n), rem = p - r * DIM * n, c = rem / n, u = rem - c * n;
      if (e0 + r < a.E) a.v_out[((size_t)(e0 + r) * DIM + c) * n + u] = S[((size_t)c * TT + r) * lds_ld + u];
    }
  }
}

// Adjoint of channel mixing for a non-final layer.  dE/dV^L is rebuilt from
// the final layer: dE/dV[a][u] = w_a Gamma'[a][u] dE/dT'[u] (+ dE/ds at a = 0).
template <int LMAX, int TT>
__global__ __launch_bounds__(256) void k_mix_adjoint(TensorArgs a, int lds_ld, int Kp, int Np) {
  constexpr int DIM = (LMAX + 1) * (LMAX + 1);
  extern __shared__ __align__(16) float S[];
  const int64_t e0 = (int64_t)blockIdx.x * TT;
  const int n = a.n;
  for (int p0 = threadIdx.x; p0 < TT * Kp; p0 += 512) {
    float gam[2][DIM], gt[2], gs[2];
    bool ok[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int p = p0 + 256 * h;
      const int r = p / Kp, u = p - r * Kp;
      const int64_t e = e0 + r;
      ok[h] = e < a.E && u < n;
      const int64_t ee = ok[h] ? e : 0;
      const int uu = ok[h] ? u : 0;
      gt[h] = a.g_tnext[(size_t)ee * n + uu];
      gs[h] = a.g_s[(size_t)ee * n + uu];
      const float* gp = a.gam_next + (size_t)(a.ei[ee] - a.centre_base) * DIM * n + uu;
#pragma unroll
      for (int c = 0; c < DIM; ++c) gam[h][c] = gp[c * n];
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int p = p0 + 256 * h;
      const int r = p / Kp, u = p - r * Kp;
#pragma unroll
      for (int c = 0; c < DIM; ++c) {
        float gV = ok[h] ? a.tp_wnext[c] * gam[h][c] * gt[h] : 0.0f;
        if (c == 0 && ok[h]) gV += gs[h];
        S[((size_t)c * TT + r) * lds_ld + u] = gV;
      }
    }
  }
  __syncthreads();
  if (a.channel_mix) {
    mix_tile<DIM, TT>(S, lds_ld, (const float*)a.mixB, a.mix_stride, n, Kp, Np, a.mix_scale, a.g_tout, e0, a.E);
  } else {
    for (int p = threadIdx.x; p < TT * DIM * n; p += 256) {
      const int r = p / (DIM * n), rem = p - r * DIM * n, c = rem / n, u = rem - c * n;
      if (e0 + r < a.E) a.g_tout[((size_t)(e0 + r) * DIM + c) * n + u] = S[((size_t)c * TT + r) * lds_ld + u];
    }
  }
}

// ---------------------------------------------------------------------------
// Adjoint of the tensor product and the environment sum: one wavefront per
// centre, lane = channel (with n < 64, 64/n groups of lanes take interleaved
// edges).  Pass 1 accumulates dE/dGamma over the centre's edges (and, when V
// is built from a0 Y, emits dE/da0 and that part of dE/dY).  Pass 2 emits
// dE/dw and the environment part of dE/dY.  Edges are processed in batches of
// kBatch per group so that their loads are in flight together; the per-edge
// sums over channels needed for dE/dY go through a padded LDS transpose
// (one lane per (edge, component) row) instead of cross-lane shuffles.
constexpr int kBatch = 4;
constexpr int kRedPerWave = 2600;   // >= kBatch * 9 * (64 + 64/n) for n in {8,...,64}

template <int DIM>
__device__ __forceinline__ void reduce_rows(const float* red, int rows, int n, int eb0, int eb1, int G,
                                            int t, float* gY, bool keep, float scale, int lane) {
  for (int idx = lane; idx < rows; idx += kWave) {
    const int slot = idx / DIM, b = idx - slot * DIM;
    const int j = slot / G, g = slot - j * G;
    const int e = eb0 + g + G * (t * kBatch + j);
    float sum = 0.0f;
    const float* r = red + idx * (n + 1);
    for (int u = 0; u < n; ++u) sum += r[u];
    if (e < eb1) {
      float* o = gY + (size_t)e * 9 + b;
      *o = (keep ? *o : 0.0f) + sum * scale;
    }
  }
}

template <int LMAX, bool FINAL>
__global__ __launch_bounds__(256) void k_tp_env_adjoint(TensorArgs a) {
  using Pat = TpPattern<LMAX, FINAL>;
  constexpr int DIM = Pat::DIM, DOUT = Pat::DOUT;
  __shared__ float red_all[4][kRedPerWave];
  const int lane = lane_id();
  float* red = red_all[threadIdx.x >> 6];
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= a.n_centres) return;
  const int n = a.n, G = kWave / n, u = lane & (n - 1), g = lane / n;
  const float* w = a.tpw_v;   // kernel-argument array: uniform, read with scalar loads
  float Gm[DIM], gG[DIM];
  {
    const float* gp = a.gam + (size_t)c * DIM * n + u;
#pragma unroll
    for (int b = 0; b < DIM; ++b) { Gm[b] = gp[b * n]; gG[b] = 0.0f; }
  }
  const int eb0 = a.row_ptr[c], eb1 = a.row_ptr[c + 1];
  const int nbatch = (eb1 - eb0 + G * kBatch - 1) / (G * kBatch);   // uniform within the wave
  const int rows = kBatch * G * DIM;
  const bool from_a0 = a.v.from_a0 != 0;
  // ---- pass 1
  for (int t = 0; t < nbatch; ++t) {
    float V[kBatch][DIM], gT[kBatch][DOUT], a0v[kBatch][LMAX + 1], Yv[kBatch][DIM];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int e = eb0 + g + G * (t * kBatch + j);
      const bool act = e < eb1;
      const int ee = act ? e : eb0;
      const float* Y = a.eb + (size_t)ee * kEB;
      const float* vp = a.v.p + (size_t)ee * a.v.ld + u;
      const float* gtp = a.g_t + (size_t)ee * DOUT * n + u;
#pragma unroll
      for (int k = 0; k < DIM; ++k) Yv[j][k] = Y[k];
      if (from_a0) {
#pragma unroll
        for (int l = 0; l <= LMAX; ++l) a0v[j][l] = act ? vp[l * n] : 0.0f;
#pragma unroll
        for (int k = 0; k < DIM; ++k) V[j][k] = a0v[j][lof(k)] * Yv[j][k];
      } else {
#pragma unroll
        for (int k = 0; k < DIM; ++k) V[j][k] = act ? vp[k * n] : 0.0f;
      }
#pragma unroll
      for (int k = 0; k < DOUT; ++k) gT[j][k] = act ? gtp[k * n] : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < kBatch; ++j) tp_adjoint_g<Pat>(V[j], gT[j], gG, w, std::make_index_sequence<Pat::NNZ>{});
    if (from_a0) {
#pragma unroll
      for (int j = 0; j < kBatch; ++j) {
        const int e = eb0 + g + G * (t * kBatch + j);
        const bool act = e < eb1;
        float gV[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) gV[k] = 0.0f;
        tp_adjoint_v<Pat>(Gm, gT[j], gV, w, std::make_index_sequence<Pat::NNZ>{});
        float ga[LMAX + 1];
#pragma unroll
        for (int l = 0; l <= LMAX; ++l) ga[l] = 0.0f;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
          ga[lof(k)] = fmaf(gV[k], Yv[j][k], ga[lof(k)]);
          red[((j * G + g) * DIM + k) * (n + 1) + u] = gV[k] * a0v[j][lof(k)];
        }
        if (act) {
#pragma unroll
          for (int l = 0; l <= LMAX; ++l) a.g_a0[(size_t)e * a.ld_gw + l * n + u] = ga[l];
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      reduce_rows<DIM>(red, rows, n, eb0, eb1, G, t, a.g_Y, a.gy_accum != 0, 1.0f, lane);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
#pragma unroll
  for (int b = 0; b < DIM; ++b) gG[b] = group_cross_sum(gG[b], n);
  // ---- pass 2
  const bool keep_gy = a.gy_accum || from_a0;
  for (int t = 0; t < nbatch; ++t) {
    float Yv[kBatch][DIM], wv[kBatch][LMAX + 1];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int e = eb0 + g + G * (t * kBatch + j);
      const bool act = e < eb1;
      const int ee = act ? e : eb0;
      const float* Y = a.eb + (size_t)ee * kEB;
      const float* wp = a.w_env + (size_t)ee * a.ld_w + u;
#pragma unroll
      for (int k = 0; k < DIM; ++k) Yv[j][k] = Y[k];
#pragma unroll
      for (int l = 0; l <= LMAX; ++l) wv[j][l] = act ? wp[l * n] : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int e = eb0 + g + G * (t * kBatch + j);
      float gw[LMAX + 1];
#pragma unroll
      for (int l = 0; l <= LMAX; ++l) gw[l] = 0.0f;
#pragma unroll
      for (int b = 0; b < DIM; ++b) {
        gw[lof(b)] = fmaf(gG[b], Yv[j][b], gw[lof(b)]);
        red[((j * G + g) * DIM + b) * (n + 1) + u] = gG[b] * wv[j][lof(b)];
      }
      if (e < eb1) {
#pragma unroll
        for (int l = 0; l <= LMAX; ++l) a.g_w[(size_t)e * a.ld_gw + l * n + u] = gw[l] * a.c_norm;
        if (u == 0) {
#pragma unroll
          for (int b = DIM; b < 9; ++b) a.g_Y[(size_t)e * 9 + b] = 0.0f;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    reduce_rows<DIM>(red, rows, n, eb0, eb1, G, t, a.g_Y, keep_gy, a.c_norm, lane);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

inline unsigned blocks(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

void mix_dims(int n, int dim, int tt, int* lds_ld, int* Kp, int* Np, size_t* bytes) {
  *Kp = ((n + 31) / 32) * 32;
  *Np = ((n + 31) / 32) * 32;
  *lds_ld = *Kp + 4;
  *bytes = (size_t)dim * tt * (*lds_ld) * sizeof(float);
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

template <int TT>
hipError_t launch_tp_mix_tt(const TensorArgs& a, hipStream_t s) {
  const int dim = (a.l_max + 1) * (a.l_max + 1);
  int ld, Kp, Np;
  size_t bytes;
  mix_dims(a.n, dim, TT, &ld, &Kp, &Np, &bytes);
  if (a.l_max == 1) return launch_lds(k_tp_mix<1, TT>, blocks(a.E, TT), bytes, s, a, ld, Kp, Np);
  return launch_lds(k_tp_mix<2, TT>, blocks(a.E, TT), bytes, s, a, ld, Kp, Np);
}

template <int TT>
hipError_t launch_mix_adjoint_tt(const TensorArgs& a, hipStream_t s) {
  const int dim = (a.l_max + 1) * (a.l_max + 1);
  int ld, Kp, Np;
  size_t bytes;
  mix_dims(a.n, dim, TT, &ld, &Kp, &Np, &bytes);
  if (a.l_max == 1) return launch_lds(k_mix_adjoint<1, TT>, blocks(a.E, TT), bytes, s, a, ld, Kp, Np);
  return launch_lds(k_mix_adjoint<2, TT>, blocks(a.E, TT), bytes, s, a, ld, Kp, Np);
}

hipError_t launch_tp_mix(const TensorArgs& a, bool final_layer, hipStream_t s) {
  if (final_layer) return hipErrorInvalidValue;   // the final layer is fused into the last MLP
  if (a.E <= 0) return hipSuccess;
  return a.tile == 16 ? launch_tp_mix_tt<16>(a, s) : launch_tp_mix_tt<32>(a, s);
}

hipError_t launch_mix_adjoint(const TensorArgs& a, hipStream_t s) {
  if (a.E <= 0) return hipSuccess;
  return a.tile == 16 ? launch_mix_adjoint_tt<16>(a, s) : launch_mix_adjoint_tt<32>(a, s);
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
