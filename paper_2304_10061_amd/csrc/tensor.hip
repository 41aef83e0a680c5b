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
#include <algorithm>
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

// Channel mixing out[e][c][v] = scale * sum_k S[c][e][k] B_{l(c)}[k][v] for
// the rows of an edge tile.  Each wave owns one 16-wide column tile of the
// output (with fewer column tiles than waves, the waves also split the
// components); the B fragments of that column tile for every l stay in
// registers for all the tiles a block processes.
constexpr int kMixKB = 2;   // K = n <= 64

template <int LMAX>
struct MixB {
  float b[LMAX + 1][kMixKB][8];
  int nt, csub, wpt;
};

template <int LMAX>
__device__ __forceinline__ void load_mix_b(MixB<LMAX>& m, const float* Bbase, int b_stride, int Kp, int Np) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = lane_id();
  const int nct = Np >> 4, nkb = Kp >> 5;   // nct is 2 or 4 (Np a multiple of 32, n <= 64)
  m.nt = wave % nct;
  m.wpt = nct >= 4 ? 1 : 4 / nct;
  m.csub = nct >= 4 ? 0 : wave / nct;
#pragma unroll
  for (int l = 0; l <= LMAX; ++l)
#pragma unroll
    for (int kb = 0; kb < kMixKB; ++kb) {
      const int kk = kb < nkb ? kb : 0;
      const float* bp = Bbase + (size_t)l * b_stride + ((size_t)(m.nt * nkb + kk) * 64 + lane) * 8;
      const float4 lo = *(const float4*)bp, hi = *(const float4*)(bp + 4);
      m.b[l][kb][0] = lo.x; m.b[l][kb][1] = lo.y; m.b[l][kb][2] = lo.z; m.b[l][kb][3] = lo.w;
      m.b[l][kb][4] = hi.x; m.b[l][kb][5] = hi.y; m.b[l][kb][6] = hi.z; m.b[l][kb][7] = hi.w;
    }
}

template <int LMAX, int TT>
__device__ void mix_tile(const float* S, int lds_ld, const MixB<LMAX>& m, int n, int Kp, float scale, float* out,
                         int64_t e0, int E) {
  constexpr int DIM = (LMAX + 1) * (LMAX + 1);
  constexpr int RT = TT / 16;
  const int lane = lane_id();
  const int nkb = Kp >> 5;
  const int col = m.nt * 16 + (lane & 15);
#pragma unroll
  for (int l = 0; l <= LMAX; ++l) {
#pragma unroll 1
    for (int c = l * l; c < (l + 1) * (l + 1); ++c) {
      if (c % m.wpt != m.csub) continue;
      f32x4 acc[RT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) acc[rt] = f32x4{0, 0, 0, 0};
#pragma unroll
      for (int kb = 0; kb < kMixKB; ++kb) {
        if (kb < nkb) {
          const float* ap = S + (size_t)c * TT * lds_ld + (lane & 15) * lds_ld + kb * 32 + 8 * (lane >> 4);
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) {
            // two 16-byte LDS reads (row stride = 4 mod 64 banks: conflict-free)
            const float4 lo = *(const float4*)(ap + rt * 16 * lds_ld);
            const float4 hi = *(const float4*)(ap + rt * 16 * lds_ld + 4);
            const float af[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
            acc[rt] = mma8(af, m.b[l][kb], acc[rt]);
          }
        }
      }
      if (col < n) {
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int r = rt * 16 + 4 * (lane >> 4) + i;
            if (e0 + r < E) out[((size_t)(e0 + r) * DIM + c) * n + col] = acc[rt][i] * scale;
          }
      }
    }
  }
}

template <int LMAX, int TT>
__device__ void copy_tile(const float* S, int lds_ld, int n, float* out, int64_t e0, int E) {
  constexpr int DIM = (LMAX + 1) * (LMAX + 1);
  for (int p = threadIdx.x; p < TT * DIM * n; p += 256) {
    const int r = p / (DIM * n), rem = p - r * DIM * n, c = rem / n, u = rem - c * n;
    if (e0 + r < E) out[((size_t)(e0 + r) * DIM + c) * n + u] = S[((size_t)c * TT + r) * lds_ld + u];
  }
}

// Tensor product (non-final layers) + channel mixing -> V^L.  Each block
// walks edge tiles blockIdx.x, blockIdx.x + gridDim.x, ... with the mixing
// fragments loaded once.
template <int LMAX, int TT>
__global__ __launch_bounds__(256) void k_tp_mix(TensorArgs a, int lds_ld, int Kp, int Np) {
  using Pat = TpPattern<LMAX, false>;
  constexpr int DIM = Pat::DIM;
  extern __shared__ __align__(16) float S[];   // [DIM][TT][lds_ld]
  const int n = a.n;
  const float* w = a.tpw_v;   // kernel-argument array: uniform, read with scalar loads
  MixB<LMAX> mb;
  if (a.channel_mix) load_mix_b<LMAX>(mb, (const float*)a.mixB, a.mix_stride, Kp, Np);
  const int ntiles = (a.E + TT - 1) / TT;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t e0 = (int64_t)tile * TT;
    // TT * Kp is a multiple of 512: two (edge, channel) items per thread per
    // step, loads of both issued before either is used
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
    if (a.channel_mix) mix_tile<LMAX, TT>(S, lds_ld, mb, n, Kp, a.mix_scale, a.v_out, e0, a.E);
    else copy_tile<LMAX, TT>(S, lds_ld, n, a.v_out, e0, a.E);
    __syncthreads();   // S is rewritten by the next tile
  }
}

// Adjoint of channel mixing for a non-final layer.  dE/dV^L is rebuilt from
// the final layer: dE/dV[a][u] = w_a Gamma'[a][u] dE/dT'[u] (+ dE/ds at a = 0).
template <int LMAX, int TT>
__global__ __launch_bounds__(256) void k_mix_adjoint(TensorArgs a, int lds_ld, int Kp, int Np) {
  constexpr int DIM = (LMAX + 1) * (LMAX + 1);
  extern __shared__ __align__(16) float S[];
  const int n = a.n;
  MixB<LMAX> mb;
  if (a.channel_mix) load_mix_b<LMAX>(mb, (const float*)a.mixB, a.mix_stride, Kp, Np);
  const int ntiles = (a.E + TT - 1) / TT;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t e0 = (int64_t)tile * TT;
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
    if (a.channel_mix) mix_tile<LMAX, TT>(S, lds_ld, mb, n, Kp, a.mix_scale, a.g_tout, e0, a.E);
    else copy_tile<LMAX, TT>(S, lds_ld, n, a.g_tout, e0, a.E);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Adjoint of the tensor product and the environment sum, in two kernels.
//
// k_tp_adjoint_gamma (one wavefront per centre; lane = channel u, and with
// n < 64 the G = 64/n lane groups take interleaved edges) accumulates
//   dE/dGamma_i[b][u] = sum_{e in N(i)} sum_{a,c} W[a][b][c] V_e[a][u] dE/dT_e[c][u]
// in registers and writes it once per centre (without the factor c).
//
// k_tp_adjoint_edges (edge-parallel; G edges per wavefront step, each wave a
// contiguous run of edges) then produces the per-edge gradients:
//   dE/dw_e[l][u] = c sum_{b: l(b)=l} dE/dGamma_i[b][u] Y_e[b]
//   dE/dY_e[b]   += c sum_u dE/dGamma_i[b][u] w_e[l(b)][u]
// and, when V_e = a0_e[l(a)][u] Y_e[a] (first layer),
//   dE/dV_e[a][u] = sum_{b,c} W[a][b][c] Gamma_i[b][u] dE/dT_e[c][u]
//   dE/da0_e[l][u] = sum_{a: l(a)=l} dE/dV_e[a][u] Y_e[a]
//   dE/dY_e[a]   += sum_u dE/dV_e[a][u] a0_e[l(a)][u].
// The sums over channels use DPP lane moves within each group of n lanes, in
// a fixed order: deterministic.
constexpr int kBatch = 4;

template <int LMAX, bool FINAL, int G>
__global__ __launch_bounds__(256) void k_tp_adjoint_gamma(TensorArgs a) {
  using Pat = TpPattern<LMAX, FINAL>;
  constexpr int DIM = Pat::DIM, DOUT = Pat::DOUT;
  constexpr int n = kWave / G;
  const int lane = lane_id();
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= a.n_centres) return;
  const int u = lane & (n - 1), g = lane / n;
  const float* w = a.tpw_v;
  float gG[DIM];
#pragma unroll
  for (int b = 0; b < DIM; ++b) gG[b] = 0.0f;
  const int eb0 = a.row_ptr[c], eb1 = a.row_ptr[c + 1];
  const bool from_a0 = a.v.from_a0 != 0;
  for (int e0 = eb0; e0 < eb1; e0 += G * kBatch) {
    float V[kBatch][DIM], gT[kBatch][DOUT];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int e = e0 + g + G * j;
      const bool act = e < eb1;
      const uint32_t ee = act ? e : eb0;
      const float* vp = a.v.p + ee * (uint32_t)a.v.ld + u;
      const float* gtp = a.g_t + ee * (uint32_t)(DOUT * n) + u;
      if (from_a0) {
        const float* Y = a.eb + ee * kEB;
        float a0v[LMAX + 1];
#pragma unroll
        for (int l = 0; l <= LMAX; ++l) a0v[l] = vp[l * n];
#pragma unroll
        for (int k = 0; k < DIM; ++k) V[j][k] = a0v[lof(k)] * Y[k];
      } else {
#pragma unroll
        for (int k = 0; k < DIM; ++k) V[j][k] = vp[k * n];
      }
#pragma unroll
      for (int k = 0; k < DOUT; ++k) gT[j][k] = act ? gtp[k * n] : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < kBatch; ++j) tp_adjoint_g<Pat>(V[j], gT[j], gG, w, std::make_index_sequence<Pat::NNZ>{});
  }
  if constexpr (G > 1) {
#pragma unroll
    for (int b = 0; b < DIM; ++b) gG[b] = group_cross_sum(gG[b], n);
  }
  if (g == 0) {
    float* out = a.g_gam + (size_t)c * DIM * n + u;
#pragma unroll
    for (int b = 0; b < DIM; ++b) out[b * n] = gG[b];
  }
}

constexpr int kEdgesPerWave = 32;

// A0: the layer's V is the rank-1 first-layer form a0[l(a)][u] Y[a].
template <int LMAX, bool FINAL, int G, bool A0>
__global__ __launch_bounds__(256) void k_tp_adjoint_edges(TensorArgs a) {
  using Pat = TpPattern<LMAX, FINAL>;
  constexpr int DIM = Pat::DIM, DOUT = Pat::DOUT;
  constexpr int n = kWave / G;
  constexpr int KB = A0 ? 2 : 4;   // edges per lane group whose loads are issued together
  const int lane = lane_id();
  const int u = lane & (n - 1), g = lane / n;
  const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t w0 = (int64_t)wave * kEdgesPerWave;
  const float* w = a.tpw_v;
  const bool keep_gy = a.gy_accum != 0;
  const float cn = a.c_norm;
  // centres of the wave's edges: one load per lane, read out per edge.  With
  // one edge per wave step (G = 1) the centre is wave-uniform; without the
  // first-layer rank-1 form its dE/dGamma rows then stay in registers until
  // it changes (CACHE).  The rank-1 form keeps every row load in the batched
  // load phase, where its latency overlaps the batch's other loads.
  constexpr bool CACHE = G == 1 && !A0;
  const int64_t el = w0 + (lane & (kEdgesPerWave - 1));
  const int ci_lane = el < a.E ? a.ei[el] - a.centre_base : 0;
  int cur = -1;
  float cG[CACHE ? DIM : 1];
  for (int j0 = 0; j0 < kEdgesPerWave; j0 += G * KB) {
    float gG[CACHE ? 1 : KB][DIM], Yv[KB][DIM], wv[KB][LMAX + 1];
    float Gm[A0 ? KB : 1][DIM], gT[A0 ? KB : 1][DOUT], a0v[A0 ? KB : 1][LMAX + 1];
    bool act[KB];
    uint32_t eev[KB], civ[KB];
#pragma unroll
    for (int q = 0; q < KB; ++q) {
      const int jj = j0 + g + G * q;
      const int64_t e = w0 + jj;
      act[q] = jj < kEdgesPerWave && e < a.E;
      const uint32_t ee = act[q] ? (uint32_t)e : 0u;
      eev[q] = ee;
      uint32_t ci = (uint32_t)__shfl(ci_lane, jj & (kEdgesPerWave - 1), kWave);
      if constexpr (G == 1) ci = __builtin_amdgcn_readfirstlane(ci);
      civ[q] = ci;
      const float* Y = a.eb + ee * kEB;
      const float* wp = a.w_env + ee * (uint32_t)a.ld_w + u;
#pragma unroll
      for (int b = 0; b < DIM; ++b) Yv[q][b] = Y[b];
#pragma unroll
      for (int l = 0; l <= LMAX; ++l) wv[q][l] = wp[l * n];
      if constexpr (!CACHE) {
        const float* ggp = a.g_gam + ci * (uint32_t)(DIM * n) + u;
#pragma unroll
        for (int b = 0; b < DIM; ++b) gG[q][b] = ggp[b * n];
      }
      if constexpr (A0) {
        const float* gtp = a.g_t + ee * (uint32_t)(DOUT * n) + u;
        const float* vp = a.v.p + ee * (uint32_t)a.v.ld + u;
        const float* gmp = a.gam + ci * (uint32_t)(DIM * n) + u;
#pragma unroll
        for (int b = 0; b < DIM; ++b) Gm[q][b] = gmp[b * n];
#pragma unroll
        for (int k = 0; k < DOUT; ++k) gT[q][k] = gtp[k * n];
#pragma unroll
        for (int l = 0; l <= LMAX; ++l) a0v[q][l] = vp[l * n];
      }
    }
#pragma unroll
    for (int q = 0; q < KB; ++q) {
      const uint32_t ee = eev[q];
      if constexpr (CACHE) {
        if ((int)civ[q] != cur) {   // wave-uniform
          const float* ggp = a.g_gam + civ[q] * (uint32_t)(DIM * n) + u;
#pragma unroll
          for (int b = 0; b < DIM; ++b) cG[b] = ggp[b * n];
          cur = (int)civ[q];
        }
      }
      const float* gGq = CACHE ? cG : gG[CACHE ? 0 : q];
      float r[DIM];
#pragma unroll
      for (int k = 0; k < DIM; ++k) r[k] = 0.0f;
      float gw[LMAX + 1];
#pragma unroll
      for (int l = 0; l <= LMAX; ++l) gw[l] = 0.0f;
#pragma unroll
      for (int b = 0; b < DIM; ++b) {
        gw[lof(b)] = fmaf(gGq[b], Yv[q][b], gw[lof(b)]);
        r[b] = cn * gGq[b] * wv[q][lof(b)];
      }
      if constexpr (A0) {
        float gV[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) gV[k] = 0.0f;
        tp_adjoint_v<Pat>(Gm[q], gT[q], gV, w, std::make_index_sequence<Pat::NNZ>{});
        float ga[LMAX + 1];
#pragma unroll
        for (int l = 0; l <= LMAX; ++l) ga[l] = 0.0f;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
          ga[lof(k)] = fmaf(gV[k], Yv[q][k], ga[lof(k)]);
          r[k] = fmaf(gV[k], a0v[q][lof(k)], r[k]);
        }
        if (act[q]) {
#pragma unroll
          for (int l = 0; l <= LMAX; ++l) a.g_a0[ee * (uint32_t)a.ld_gw + l * n + u] = ga[l];
        }
      }
      if (act[q]) {
#pragma unroll
        for (int l = 0; l <= LMAX; ++l) a.g_w[ee * (uint32_t)a.ld_gw + l * n + u] = gw[l] * cn;
      }
      // sums over the group's channels (DPP; the group's last lane holds them)
#pragma unroll
      for (int k = 0; k < DIM; ++k) r[k] = group_sum_dpp<n>(r[k]);
      if (act[q] && u == n - 1) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          float* o = a.g_Y + ee * 9u + k;
          const float val = k < DIM ? r[k] : 0.0f;
          *o = (keep_gy && k < DIM) ? *o + val : val;
        }
      }
    }
  }
}

inline unsigned blocks(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// Blocks of the edge-tile mixing kernels: a few per compute unit, each
// walking many tiles with its mixing fragments in registers.
constexpr unsigned kMixBlocks = 256 * 8;

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
  // one tile per block: the tensor-product phase's load latency is hidden by
  // many resident blocks rather than by a tile loop
  const unsigned grid = blocks(a.E, TT);
  if (a.l_max == 1) return launch_lds(k_tp_mix<1, TT>, grid, bytes, s, a, ld, Kp, Np);
  return launch_lds(k_tp_mix<2, TT>, grid, bytes, s, a, ld, Kp, Np);
}

template <int TT>
hipError_t launch_mix_adjoint_tt(const TensorArgs& a, hipStream_t s) {
  const int dim = (a.l_max + 1) * (a.l_max + 1);
  int ld, Kp, Np;
  size_t bytes;
  mix_dims(a.n, dim, TT, &ld, &Kp, &Np, &bytes);
  const unsigned grid = std::min<unsigned>(blocks(a.E, TT), kMixBlocks);
  if (a.l_max == 1) return launch_lds(k_mix_adjoint<1, TT>, grid, bytes, s, a, ld, Kp, Np);
  return launch_lds(k_mix_adjoint<2, TT>, grid, bytes, s, a, ld, Kp, Np);
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

template <int LMAX, bool FINAL, int G>
hipError_t launch_adjoint_g(const TensorArgs& a, hipStream_t s) {
  if (a.n_centres > 0)
    hipLaunchKernelGGL((k_tp_adjoint_gamma<LMAX, FINAL, G>), dim3(blocks(a.n_centres, 4)), dim3(256), 0, s, a);
  if (a.E > 0) {
    const dim3 grid(blocks(a.E, 4 * kEdgesPerWave));
    if (a.v.from_a0) hipLaunchKernelGGL((k_tp_adjoint_edges<LMAX, FINAL, G, true>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_tp_adjoint_edges<LMAX, FINAL, G, false>), grid, dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

template <int LMAX, bool FINAL>
hipError_t launch_adjoint_n(const TensorArgs& a, hipStream_t s) {
  switch (a.n) {
    case 64: return launch_adjoint_g<LMAX, FINAL, 1>(a, s);
    case 32: return launch_adjoint_g<LMAX, FINAL, 2>(a, s);
    case 16: return launch_adjoint_g<LMAX, FINAL, 4>(a, s);
    case 8: return launch_adjoint_g<LMAX, FINAL, 8>(a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_tp_env_adjoint(const TensorArgs& a, bool final_layer, hipStream_t s) {
  if (a.l_max == 1) return final_layer ? launch_adjoint_n<1, true>(a, s) : launch_adjoint_n<1, false>(a, s);
  return final_layer ? launch_adjoint_n<2, true>(a, s) : launch_adjoint_n<2, false>(a, s);
}

}  // namespace allegro
