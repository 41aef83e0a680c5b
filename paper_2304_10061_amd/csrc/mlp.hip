// mlp.hip - fused, edge-batched MLP chains on MFMA (the scalar track).
//
// The scalar track carries most of the model's capacity as dense MLPs over
// ordered pairs (section "Allegro: Scalable Equivariant Deep Learning": the two
// tracks; section "Training details": two-body and later latent MLPs with SiLU,
// a linear environment embedding, an edge-energy MLP with no nonlinearity).
// The matrix products are the bulk of the cost (section "Mixed-precision
// calculations"), so each MLP chain runs as one kernel per tile of TM edges:
// activations stay in LDS, weights stream from L2 in a pre-packed MFMA operand
// layout, and the linear map that consumes the MLP output (environment
// embedding of the next layer, or the edge energy) is fused as a "head".
//
// Precision: PREC 1 = BF16 operands (v_mfma_f32_16x16x32_bf16) with FP32
// accumulation, PREC 0 = FP32 (v_mfma_f32_16x16x4_f32).  The residual stream
// and all epilogues are FP32.
//
// Kinds (x_prev, u from the edge record, rs = 1/sqrt(2)):
//   two-body      x0 = u * MLP([onehot(Z_i), onehot(Z_j), R])        head: [a0 | w^1]
//   latent        x^L = rs (x^{L-1} + u * MLP([x^{L-1}, V^L[0]]))     head: w^{L+1}
//   latent-final  same with the final scalar tensor product computed in the
//                 prologue from V^{L-1} and Gamma^L; the edge energy
//                 E_ij = x^L . we (edge MLP folded into one vector) is the head.
// The backward kernel recomputes the chain from its inputs (no stored
// activations), then propagates input gradients only (no weight gradients).
#include "devutil.h"
#include "internal.h"

namespace allegro {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int PREC> struct PT;

template <> struct PT<1> {
  using T = __bf16;
  struct F { bf16x8 v; };
  static __device__ __forceinline__ F load(const T* p) { F f; f.v = *(const bf16x8*)p; return f; }
  static __device__ __forceinline__ f32x4 mma(const F& a, const F& b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b.v, c, 0, 0, 0);
  }
};

// PREC 2: BF16 operands with single-rounded weights (no low-order correction).
template <> struct PT<2> : PT<1> {};

template <> struct PT<0> {
  using T = float;
  struct F { f32x4 lo, hi; };
  static __device__ __forceinline__ F load(const T* p) {
    F f;
    f.lo = *(const f32x4*)p;
    f.hi = *(const f32x4*)(p + 4);
    return f;
  }
  // Eight K=4 steps; step s takes k = 8 (lane/16) + s from each lane group, so
  // the 32-wide K block is covered exactly once with the same fragment layout
  // as the BF16 instruction.
  static __device__ __forceinline__ f32x4 mma(const F& a, const F& b, f32x4 c) {
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.lo[0], b.lo[0], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.lo[1], b.lo[1], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.lo[2], b.lo[2], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.lo[3], b.lo[3], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.hi[0], b.hi[0], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.hi[1], b.hi[1], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.hi[2], b.hi[2], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.hi[3], b.hi[3], c, 0, 0, 0);
    return c;
  }
};

// Column tiles of a GEMM output are dealt to the four waves round-robin; pass
// p covers nt = wave + 4 (p MAXCT + q), q < MAXCT, so wide outputs run in
// several passes with a bounded accumulator set.
template <int MAXCT>
__device__ __forceinline__ int tile_of(int pass, int q, int wave) { return wave + 4 * (pass * MAXCT + q); }

template <int MAXCT>
__device__ __forceinline__ int npasses(int Np) { return (Np / 16 + 4 * MAXCT - 1) / (4 * MAXCT); }

// acc[rt][q] = A[TM x K-range] (LDS) @ B[K-range x tiles of this pass].
// A holds the columns of K blocks [kb0, kb1) starting at its column 0.  The
// loop is branch-free: column tiles beyond the matrix are clamped to its last
// tile (their results are never stored), and the B fragments of the next K
// block are requested before the MFMAs of the current one, so L2 latency
// overlaps matrix-core work.  `wave` must be wave-uniform (readfirstlane).
template <int PREC, int RT, int MAXCT>
__device__ __forceinline__ void gemm_tile(f32x4 (&acc)[RT][MAXCT], const typename PT<PREC>::T* A,
                                          int lda, const GemmB& B, int wave, int lane, int pass,
                                          int kb0 = 0, int kb1 = -1, bool zero = true) {
  using P = PT<PREC>;
  using T = typename P::T;
  using F = typename P::F;
  if (zero) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int q = 0; q < MAXCT; ++q) acc[rt][q] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  }
  const int nkb = B.Kp >> 5, nct = B.Np >> 4;
  if (kb1 < 0) kb1 = nkb;
  // PREC 1 keeps each weight as a pair of BF16 values (hi + lo, lo stored
  // after the hi fragments) and issues two MFMAs per product.
  constexpr bool kSplit = PREC == 1;
  const size_t lo_off = (size_t)B.Kp * B.Np;
  const T* Bl = (const T*)B.p + (size_t)lane * 8;
  const T* Arow = A + (lane & 15) * lda + 8 * (lane >> 4) - kb0 * 32;
  size_t boff[MAXCT];
#pragma unroll
  for (int q = 0; q < MAXCT; ++q) {
    int nt = tile_of<MAXCT>(pass, q, wave);
    nt = nt < nct ? nt : nct - 1;
    boff[q] = (size_t)(nt * nkb) * 512;
  }
  // two register buffers of B fragments, used alternately (no copies)
  F b0[MAXCT], b1[MAXCT], l0[kSplit ? MAXCT : 1], l1[kSplit ? MAXCT : 1];
  auto load_b = [&](F (&bb)[MAXCT], F (&ll)[kSplit ? MAXCT : 1], int kb) {
#pragma unroll
    for (int q = 0; q < MAXCT; ++q) {
      bb[q] = P::load(Bl + boff[q] + (size_t)kb * 512);
      if constexpr (kSplit) ll[q] = P::load(Bl + lo_off + boff[q] + (size_t)kb * 512);
    }
  };
  auto compute = [&](const F (&bb)[MAXCT], const F (&ll)[kSplit ? MAXCT : 1], int kb) {
    F a[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) a[rt] = P::load(Arow + rt * 16 * lda + kb * 32);
    if constexpr (kSplit) {
#pragma unroll
      for (int q = 0; q < MAXCT; ++q)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) acc[rt][q] = P::mma(a[rt], ll[q], acc[rt][q]);
    }
#pragma unroll
    for (int q = 0; q < MAXCT; ++q)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) acc[rt][q] = P::mma(a[rt], bb[q], acc[rt][q]);
  };
  load_b(b0, l0, kb0);
  int kb = kb0;
  for (; kb + 1 < kb1; kb += 2) {
    load_b(b1, l1, kb + 1);
    compute(b0, l0, kb);
    load_b(b0, l0, kb + 2 < kb1 ? kb + 2 : kb + 1);   // the last pass reloads a block it has
    compute(b1, l1, kb + 1);
  }
  if (kb < kb1) compute(b0, l0, kb);
  // tiles clamped onto the last one hold copies: zero them so that register
  // uses of acc (gradients, dot products) see exact zeros there
#pragma unroll
  for (int q = 0; q < MAXCT; ++q)
    if (tile_of<MAXCT>(pass, q, wave) >= nct)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) acc[rt][q] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
}

template <class T> __device__ __forceinline__ T to_t(float v) { return (T)v; }

__device__ __forceinline__ void store4(__bf16* p, float4 v) {
  typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
  bf16x4 b = {(__bf16)v.x, (__bf16)v.y, (__bf16)v.z, (__bf16)v.w};
  *(bf16x4*)p = b;
}
__device__ __forceinline__ void store4(float* p, float4 v) { *(float4*)p = v; }

// Four consecutive input columns c..c+3 (c a multiple of 4) of edge e.
__device__ __forceinline__ float4 input4(const MlpArgs& a, int e, int c) {
  float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if (e >= a.E) return v;
  if (a.kind == kTwoBody) {
    const int S = a.n_species, zi = a.species[a.ei[e]], zj = a.species[a.ej[e]];
    float t[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int cc = c + k;
      float x = 0.0f;
      if (cc < S) x = zi == cc ? 1.0f : 0.0f;
      else if (cc < 2 * S) x = zj == cc - S ? 1.0f : 0.0f;
      else if (cc < 2 * S + a.n_bessel) x = a.eb[(size_t)e * kEB + kEB_R + (cc - 2 * S)];
      t[k] = x;
    }
    return make_float4(t[0], t[1], t[2], t[3]);
  }
  if (c < a.d) return *(const float4*)(a.x_prev + (size_t)e * a.d + c);
  if (c >= a.d + a.n) return v;
  const int u = c - a.d;
  if (a.kind == kLatent) return *(const float4*)(a.s_in + (size_t)e * a.s_ld + u);
  // final-layer scalar tensor product: T[u] = sum_c w_c V[c][u] Gamma[c][u]
  const int dim = (a.l_max + 1) * (a.l_max + 1);
  const float* gam = a.tp_gam + (size_t)(a.ei[e] - a.centre_base) * dim * a.n + u;
  const float* vp = a.tp_v.p + (size_t)e * a.tp_v.ld + u;
  const float* Y = a.eb + (size_t)e * kEB;
  for (int cc = 0; cc < dim; ++cc) {
    const int l = cc == 0 ? 0 : (cc < 4 ? 1 : 2);
    float4 vv = a.tp_v.from_a0 ? *(const float4*)(vp + l * a.n) : *(const float4*)(vp + cc * a.n);
    const float y = a.tp_v.from_a0 ? Y[cc] : 1.0f;
    const float4 g = *(const float4*)(gam + cc * a.n);
    const float w = a.tp_w[cc] * y;
    v.x = fmaf(w * vv.x, g.x, v.x);
    v.y = fmaf(w * vv.y, g.y, v.y);
    v.z = fmaf(w * vv.z, g.z, v.z);
    v.w = fmaf(w * vv.w, g.w, v.w);
  }
  return v;
}

// Input rows of the chain for edges e0 .. e0+TM-1, zero padded to Kp.  Each
// wave fills TM/4 rows; a lane gathers 16-byte chunks of four rows before
// storing them, so several global loads are in flight per lane.
template <int PREC, int TM>
__device__ void build_input(const MlpArgs& a, typename PT<PREC>::T* X, int ldx, int e0, int Kp) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  constexpr int RPW = TM / 4;
  const int nq = Kp >> 2;
  for (int q0 = 0; q0 < nq; q0 += 64) {
    const int q = q0 + lane;
    for (int r0 = 0; r0 < RPW; r0 += 4) {
      float4 v[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int r = wave * RPW + r0 + k;
        v[k] = q < nq ? input4(a, e0 + r, 4 * q) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      }
      if (q < nq) {
#pragma unroll
        for (int k = 0; k < 4; ++k) store4(X + (wave * RPW + r0 + k) * ldx + 4 * q, v[k]);
      }
    }
  }
}

// Rows of a row-major FP32 matrix (row stride ld) into X, columns [c0, c0+w).
template <int PREC, int TM>
__device__ void stage_rows(const float* src, int ld, int ncols, int E, typename PT<PREC>::T* X, int ldx,
                           int e0, int c0, int w) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  constexpr int RPW = TM / 4;
  const int nq = w >> 2;
  for (int q0 = 0; q0 < nq; q0 += 64) {
    const int q = q0 + lane;
    for (int r0 = 0; r0 < RPW; r0 += 4) {
      float4 v[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int e = e0 + wave * RPW + r0 + k;
        const int c = c0 + 4 * q;
        v[k] = (q < nq && e < E && c < ncols) ? *(const float4*)(src + (size_t)e * ld + c)
                                              : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      }
      if (q < nq) {
#pragma unroll
        for (int k = 0; k < 4; ++k) store4(X + (wave * RPW + r0 + k) * ldx + 4 * q, v[k]);
      }
    }
  }
}

// Writes f(acc) of pass `pass` into an LDS tile (row-major, T) for columns < Np.
template <int PREC, int RT, int MAXCT, class Fn>
__device__ __forceinline__ void store_tile(const f32x4 (&acc)[RT][MAXCT], typename PT<PREC>::T* out,
                                           int ldo, int Np, int wave, int lane, int pass, Fn fn) {
  using T = typename PT<PREC>::T;
#pragma unroll
  for (int q = 0; q < MAXCT; ++q) {
    const int nt = tile_of<MAXCT>(pass, q, wave);
    if (nt * 16 >= Np) continue;
    const int col = nt * 16 + (lane & 15);
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = rt * 16 + 4 * (lane >> 4) + i;
        out[row * ldo + col] = to_t<T>(fn(acc[rt][q][i], row, col));
      }
  }
}

// Hidden layers of the chain: `in` -> SiLU -> alternate buffer, optionally
// keeping the pre-activations.  Returns the buffer holding the last hidden
// activation (the input of the last layer).
template <int PREC, int TM, int MAXCT>
__device__ __forceinline__ const typename PT<PREC>::T* hidden_layers(
    const MlpArgs& a, typename PT<PREC>::T* X, int ldx, typename PT<PREC>::T* H, int ldh,
    typename PT<PREC>::T* Pb, int ldp, int* ldin, int wave, int lane) {
  using T = typename PT<PREC>::T;
  constexpr int RT = TM / 16;
  const T* in = X;
  *ldin = ldx;
  f32x4 acc[RT][MAXCT];
  for (int l = 0; l + 1 < a.w.nl; ++l) {
    T* out = (in == X) ? H : X;
    const int ldo = (in == X) ? ldh : ldx;
    const GemmB& B = a.w.fwd[l];
    for (int p = 0; p < npasses<MAXCT>(B.Np); ++p) {
      gemm_tile<PREC, RT, MAXCT>(acc, in, *ldin, B, wave, lane, p);
      if (Pb) store_tile<PREC, RT, MAXCT>(acc, Pb + l * TM * ldp, ldp, B.Np, wave, lane, p,
                                          [](float v, int, int) { return v; });
      store_tile<PREC, RT, MAXCT>(acc, out, ldo, B.Np, wave, lane, p, [](float v, int, int) { return silu(v); });
    }
    __syncthreads();
    in = out;
    *ldin = ldo;
  }
  return in;
}

template <int PREC, int TM, int MAXCT>
__global__ __launch_bounds__(256, 1) void k_mlp_fwd(MlpArgs a, int ldx, int ldh) {
  using P = PT<PREC>;
  using T = typename P::T;
  constexpr int RT = TM / 16;
  extern __shared__ __align__(16) char smem[];
  T* X = (T*)smem;
  T* H = X + TM * ldx;
  __shared__ float red[4][TM];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int e0 = blockIdx.x * TM;

  build_input<PREC, TM>(a, X, ldx, e0, a.w.fwd[0].Kp);
  __syncthreads();
  int ldin;
  const T* in = hidden_layers<PREC, TM, MAXCT>(a, X, ldx, H, ldh, nullptr, 0, &ldin, wave, lane);
  const int nl = a.w.nl;
  f32x4 acc[RT][MAXCT];
  gemm_tile<PREC, RT, MAXCT>(acc, in, ldin, a.w.fwd[nl - 1], wave, lane, 0);   // N = d: one pass
  // epilogue: x = u h (two-body) or rs (x_prev + u h) (latent), kept in acc
  const int d = a.d;
#pragma unroll
  for (int q = 0; q < MAXCT; ++q) {
    const int col = tile_of<MAXCT>(0, q, wave) * 16 + (lane & 15);
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int e = e0 + rt * 16 + 4 * (lane >> 4) + i;
        float v = 0.0f;
        if (e < a.E && col < d) {
          const float u = a.eb[(size_t)e * kEB + kEB_U];
          if (a.kind == kTwoBody) v = u * acc[rt][q][i];
          else v = a.res_scale * (a.x_prev[(size_t)e * d + col] + u * acc[rt][q][i]);
          if (a.x_out) a.x_out[(size_t)e * d + col] = v;
        }
        acc[rt][q][i] = v;
      }
  }
  if (a.kind == kLatentFinal) {
    // E_ij = x . we : per-lane partial over its columns, then across lanes and waves
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float sum = 0.0f;
#pragma unroll
        for (int q = 0; q < MAXCT; ++q) {
          const int col = tile_of<MAXCT>(0, q, wave) * 16 + (lane & 15);
          if (col < d) sum = fmaf(acc[rt][q][i], a.we[col], sum);
        }
        sum = group_inner_sum(sum, 16);
        if ((lane & 15) == 0) red[wave][rt * 16 + 4 * (lane >> 4) + i] = sum;
      }
    __syncthreads();
    if ((int)threadIdx.x < TM) {
      const int e = e0 + threadIdx.x;
      if (e < a.E)
        a.eij[e] = ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
    }
    return;
  }
  if (a.head.p == nullptr) return;
  // head GEMM on x, staged in the buffer the last layer did not read
  T* xb = (in == X) ? H : X;
  const int ldxb = (in == X) ? ldh : ldx;
  store_tile<PREC, RT, MAXCT>(acc, xb, ldxb, a.w.fwd[nl - 1].Np, wave, lane, 0, [](float v, int, int) { return v; });
  __syncthreads();
  const int Nh = a.head.N;
  for (int p = 0; p < npasses<MAXCT>(a.head.Np); ++p) {
    gemm_tile<PREC, RT, MAXCT>(acc, xb, ldxb, a.head, wave, lane, p);
#pragma unroll
    for (int q = 0; q < MAXCT; ++q) {
      const int col = tile_of<MAXCT>(p, q, wave) * 16 + (lane & 15);
      if (col >= Nh) continue;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int e = e0 + rt * 16 + 4 * (lane >> 4) + i;
          if (e < a.E) a.head_out[(size_t)e * Nh + col] = acc[rt][q][i];
        }
    }
  }
}

template <int PREC, int TM, int MAXCT>
__global__ __launch_bounds__(256, 1) void k_mlp_bwd(MlpArgs a, int ldx, int ldh) {
  using P = PT<PREC>;
  using T = typename P::T;
  constexpr int RT = TM / 16;
  extern __shared__ __align__(16) char smem[];
  T* X = (T*)smem;
  T* H = X + TM * ldx;
  T* Pb = H + TM * ldh;                 // nl-1 pre-activation buffers [TM][ldh]
  __shared__ float red[4][TM];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int e0 = blockIdx.x * TM;
  const int d = a.d;
  const int nl = a.w.nl;

  // 1. G = dE/dx_out (columns < d all lie in pass 0)
  f32x4 G[RT][MAXCT];
#pragma unroll
  for (int q = 0; q < MAXCT; ++q) {
    const int col = tile_of<MAXCT>(0, q, wave) * 16 + (lane & 15);
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int e = e0 + rt * 16 + 4 * (lane >> 4) + i;
        float v = 0.0f;
        if (e < a.E && col < d) {
          if (a.kind == kLatentFinal) v = a.g_const[(size_t)a.species[a.ei[e]] * d + col];
          else if (a.g_x) v = a.g_x[(size_t)e * d + col];
        }
        G[rt][q][i] = v;
      }
  }
  f32x4 acc[RT][MAXCT];
  if (a.kind != kLatentFinal && a.head_bwd.p != nullptr) {
    // G += g_head @ W_head^T, K staged through X in chunks of its width
    const int Kh = a.head_bwd.K, nkb = a.head_bwd.Kp >> 5, chunk = ldx >> 5;
    for (int kb0 = 0; kb0 < nkb; kb0 += chunk) {
      const int kb1 = kb0 + chunk < nkb ? kb0 + chunk : nkb;
      const int w = (kb1 - kb0) * 32;
      stage_rows<PREC, TM>(a.g_head, Kh, Kh, a.E, X, ldx, e0, kb0 * 32, w);
      __syncthreads();
      gemm_tile<PREC, RT, MAXCT>(acc, X, ldx, a.head_bwd, wave, lane, 0, kb0, kb1, true);
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int q = 0; q < MAXCT; ++q) G[rt][q] += acc[rt][q];
      __syncthreads();
    }
  }

  // 2. recompute the chain, keeping hidden pre-activations
  build_input<PREC, TM>(a, X, ldx, e0, a.w.fwd[0].Kp);
  __syncthreads();
  int ldin;
  const T* in = hidden_layers<PREC, TM, MAXCT>(a, X, ldx, H, ldh, Pb, ldh, &ldin, wave, lane);
  gemm_tile<PREC, RT, MAXCT>(acc, in, ldin, a.w.fwd[nl - 1], wave, lane, 0);   // acc = h
  const float rs = (a.kind == kTwoBody) ? 1.0f : a.res_scale;
  // dE/du = rs sum_c G h
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float sum = 0.0f;
#pragma unroll
      for (int q = 0; q < MAXCT; ++q) sum = fmaf(G[rt][q][i], acc[rt][q][i], sum);
      sum = group_inner_sum(sum, 16);
      if ((lane & 15) == 0) red[wave][rt * 16 + 4 * (lane >> 4) + i] = sum;
    }
  __syncthreads();   // also: every wave is done reading `in`
  if ((int)threadIdx.x < TM) {
    const int e = e0 + threadIdx.x;
    if (e < a.E) {
      const float gu = rs * (((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) +
                             red[3][threadIdx.x]);
      a.g_u[e] = a.gu_accum ? a.g_u[e] + gu : gu;
    }
  }
  // dE/dh = rs u G into the buffer the last layer did not read
  T* cur = (in == X) ? H : X;
  int ldc = (in == X) ? ldh : ldx;
  store_tile<PREC, RT, MAXCT>(G, cur, ldc, a.w.fwd[nl - 1].Np, wave, lane, 0, [&](float v, int row, int) {
    const int e = e0 + row;
    return e < a.E ? rs * a.eb[(size_t)e * kEB + kEB_U] * v : 0.0f;
  });
  __syncthreads();
  // 3. back through the hidden layers (ping-pong between X and H)
  for (int l = nl - 1; l > 0; --l) {
    T* nxt = (cur == X) ? H : X;
    const int ldn = (cur == X) ? ldh : ldx;
    const T* Pl = Pb + (l - 1) * TM * ldh;
    const GemmB& B = a.w.bwd[l];
    for (int p = 0; p < npasses<MAXCT>(B.Np); ++p) {
      gemm_tile<PREC, RT, MAXCT>(acc, cur, ldc, B, wave, lane, p);
      store_tile<PREC, RT, MAXCT>(acc, nxt, ldn, B.Np, wave, lane, p, [&](float v, int row, int col) {
        return v * silu_grad((float)Pl[row * ldh + col]);
      });
    }
    __syncthreads();
    cur = nxt;
    ldc = ldn;
  }
  // 4. dE/dz, written straight to the outputs
  const int S = a.n_species;
  const GemmB& B0 = a.w.bwd[0];
  for (int p = 0; p < npasses<MAXCT>(B0.Np); ++p) {
    gemm_tile<PREC, RT, MAXCT>(acc, cur, ldc, B0, wave, lane, p);
#pragma unroll
    for (int q = 0; q < MAXCT; ++q) {
      const int col = tile_of<MAXCT>(p, q, wave) * 16 + (lane & 15);
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int e = e0 + rt * 16 + 4 * (lane >> 4) + i;
          if (e >= a.E) continue;
          const float g = acc[rt][q][i];
          if (a.kind == kTwoBody) {
            if (col >= 2 * S && col < 2 * S + a.n_bessel) a.g_R[(size_t)e * a.n_bessel + col - 2 * S] = g;
          } else if (col < d) {
            a.g_xprev[(size_t)e * d + col] = rs * G[rt][q][i] + g;   // p == 0 here
          } else if (col < d + a.n) {
            a.g_s[(size_t)e * a.n + col - d] = g;
          }
        }
    }
  }
}

// LDS layout: X [TM][ldx] and H [TM][ldh] (+ nl-1 pre-activation buffers of
// [TM][ldh] in the backward kernel).
template <int PREC>
void lds_dims(const MlpArgs& a, int TM, bool bwd, int* ldx, int* ldh, size_t* bytes) {
  int kh = 32;                       // widths of hidden layers and of the output d
  for (int l = 0; l < a.w.nl; ++l) kh = kh > a.w.fwd[l].Np ? kh : a.w.fwd[l].Np;
  int kx = kh > a.w.fwd[0].Kp ? kh : a.w.fwd[0].Kp;
  const int pad = PREC ? 8 : 4;
  *ldx = kx + pad;
  *ldh = kh + pad;
  const int nbuf_h = bwd ? a.w.nl : 1;
  *bytes = (size_t)TM * ((size_t)*ldx + (size_t)nbuf_h * *ldh) * (PREC ? 2 : 4);
}

// Accumulator tiles per wave: the latent width d must fit one pass.
int max_ct(const MlpArgs& a) {
  const int dt = (a.d + 15) / 16;
  return (dt + 3) / 4;
}

constexpr size_t kLdsLimit = 160 * 1024 - 4096;

template <int PREC, int TM, int MAXCT>
hipError_t launch_one(const MlpArgs& a, bool bwd, hipStream_t s) {
  int ldx, ldh;
  size_t bytes;
  lds_dims<PREC>(a, TM, bwd, &ldx, &ldh, &bytes);
  const dim3 grid((a.E + TM - 1) / TM), block(256);
  if (bwd) {
    auto k = k_mlp_bwd<PREC, TM, MAXCT>;
    hipError_t st = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (st != hipSuccess) return st;
    hipLaunchKernelGGL(k, grid, block, bytes, s, a, ldx, ldh);
  } else {
    auto k = k_mlp_fwd<PREC, TM, MAXCT>;
    hipError_t st = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (st != hipSuccess) return st;
    hipLaunchKernelGGL(k, grid, block, bytes, s, a, ldx, ldh);
  }
  return hipGetLastError();
}

template <int PREC, int TM>
hipError_t dispatch_ct(const MlpArgs& a, bool bwd, hipStream_t s) {
  const int ct = max_ct(a);
  if (ct <= 1) return launch_one<PREC, TM, 1>(a, bwd, s);
  if (ct <= 2) return launch_one<PREC, TM, 2>(a, bwd, s);
  if (ct <= 4) return launch_one<PREC, TM, 4>(a, bwd, s);
  return hipErrorInvalidValue;
}

template <int PREC>
int pick_tm(const MlpArgs& a, bool bwd) {
  const int cands[2] = {PREC ? 64 : 32, PREC ? 32 : 16};
  for (int t : cands) {
    int ldx, ldh;
    size_t bytes;
    lds_dims<PREC>(a, t, bwd, &ldx, &ldh, &bytes);
    if (bytes <= kLdsLimit) return t;
  }
  return 0;
}

template <int PREC>
bool fits(const MlpArgs& a, bool bwd, int tm) {
  int ldx, ldh;
  size_t bytes;
  lds_dims<PREC>(a, tm, bwd, &ldx, &ldh, &bytes);
  return bytes <= kLdsLimit;
}

hipError_t launch(const MlpArgs& a, int prec, bool bwd, hipStream_t s) {
  if (a.E <= 0) return hipSuccess;
  if (prec == 1 || prec == 2) {
    const int tm = (a.tm == 64 || a.tm == 32) && fits<1>(a, bwd, a.tm) ? a.tm : pick_tm<1>(a, bwd);
    if (prec == 1) {
      if (tm == 64) return dispatch_ct<1, 64>(a, bwd, s);
      if (tm == 32) return dispatch_ct<1, 32>(a, bwd, s);
    } else {
      if (tm == 64) return dispatch_ct<2, 64>(a, bwd, s);
      if (tm == 32) return dispatch_ct<2, 32>(a, bwd, s);
    }
  } else {
    const int tm = (a.tm == 32 || a.tm == 16) && fits<0>(a, bwd, a.tm) ? a.tm : pick_tm<0>(a, bwd);
    if (tm == 32) return dispatch_ct<0, 32>(a, bwd, s);
    if (tm == 16) return dispatch_ct<0, 16>(a, bwd, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

size_t mlp_lds_bytes(const MlpArgs& a, int prec, bool bwd) {
  int ldx, ldh;
  size_t bytes;
  const int tm = prec ? pick_tm<1>(a, bwd) : pick_tm<0>(a, bwd);
  if (tm == 0 || max_ct(a) > 4) return (size_t)-1;
  if (prec) lds_dims<1>(a, tm, bwd, &ldx, &ldh, &bytes);
  else lds_dims<0>(a, tm, bwd, &ldx, &ldh, &bytes);
  return bytes;
}

bool mlp_tile_fits(const MlpArgs& a, int prec, bool bwd, int tm) {
  if (prec) return (tm == 64 || tm == 32) && fits<1>(a, bwd, tm);
  return (tm == 32 || tm == 16) && fits<0>(a, bwd, tm);
}

hipError_t launch_mlp_fwd(const MlpArgs& a, int prec, hipStream_t s) { return launch(a, prec, false, s); }
hipError_t launch_mlp_bwd(const MlpArgs& a, int prec, hipStream_t s) { return launch(a, prec, true, s); }

}  // namespace allegro
