// mlp_kernels.h - fused, edge-batched MLP chains on MFMA (the scalar track).
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
//
// The kernel templates are instantiated per precision in mlp_fp32.hip,
// mlp_bf16.hip and mlp_bf16s.hip (compiled in parallel); mlp.hip holds the
// host-side tile selection.
#pragma once

#include "devutil.h"
#include "internal.h"

namespace allegro {
namespace mlpk {


typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int PREC> struct PT;

// Buffer resource of a read-only array of `bytes` bytes (raw buffer, gfx9
// descriptor word 3); out-of-range reads return zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t ro_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

template <> struct PT<1> {
  using T = __bf16;
  struct F { bf16x8 v; };
  static __device__ __forceinline__ F load(const T* p) { F f; f.v = *(const bf16x8*)p; return f; }
  // 16 bytes at voff + soff (soff wave-uniform)
  static __device__ __forceinline__ F load_buf(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    F f;
    f.v = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
    return f;
  }
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
  static __device__ __forceinline__ F load_buf(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    F f;
    f.lo = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
    f.hi = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, voff + 16, soff, 0));
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

// Waves per block.  Eight waves (two per SIMD) give each SIMD a second
// instruction stream to issue from while one waits on memory or a barrier.
constexpr int kNW = 8;
constexpr int kThreads = 64 * kNW;

// Column tiles of a GEMM output are dealt to the waves round-robin; pass p
// covers nt = wave + kNW (p MAXCT + q), q < MAXCT, so wide outputs run in
// several passes with a bounded accumulator set.
template <int MAXCT>
__device__ __forceinline__ int tile_of(int pass, int q, int wave) { return wave + kNW * (pass * MAXCT + q); }

template <int MAXCT>
__host__ __device__ __forceinline__ int npasses(int Np) { return (Np / 16 + kNW * MAXCT - 1) / (kNW * MAXCT); }

// Sum of the per-wave partials of row r, in wave order.
template <int TM>
__device__ __forceinline__ float wave_partials_sum(const float (&red)[kNW][TM], int r) {
  float s = red[0][r];
#pragma unroll
  for (int w = 1; w < kNW; ++w) s += red[w][r];
  return s;
}

// acc[rt][q] = A[TM x K-range] (LDS) @ B[K-range x tiles of this pass].
// A holds the columns of K blocks [kb0, kb1) starting at its column 0.  The
// loop is branch-free: column tiles beyond the matrix are clamped to its last
// tile (their results are never stored), and the B fragments of the next K
// block are requested before the MFMAs of the current one, so L2 latency
// overlaps matrix-core work.  `wave` must be wave-uniform (readfirstlane).
//
// PREF_A: the A fragments of the next K block are also requested ahead (two
// register sets); without it (tall tiles, RT = 8) each row tile's A fragment
// is read from LDS just before its MFMAs.
template <int PREC, int RT, int MAXCT, bool PREF_A, bool kSplit>
__device__ __forceinline__ void gemm_tile_k(f32x4 (&acc)[RT][MAXCT], const typename PT<PREC>::T* A,
                                            int lda, const GemmB& B, int wave, int lane, int pass,
                                            int kb0, int kb1, bool zero) {
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
  // kSplit: each weight is a pair of BF16 values (hi + lo, lo stored after
  // the hi fragments), two MFMAs per product.
  constexpr int NA = PREF_A ? RT : 1;
  const T* Arow = A + (lane & 15) * lda + 8 * (lane >> 4) - kb0 * 32;
  // B fragments through a buffer resource: the lane's slot is a fixed vector
  // offset, the column tile and K block a wave-uniform scalar offset, so the
  // loads need no per-lane address arithmetic
  const uint32_t lo_bytes = (uint32_t)(B.Kp * B.Np * sizeof(T));
  const __amdgpu_buffer_rsrc_t rb = ro_rsrc(B.p, lo_bytes * (kSplit ? 2 : 1));
  const uint32_t loff = (uint32_t)lane * 8 * sizeof(T);
  uint32_t bq[MAXCT];
#pragma unroll
  for (int q = 0; q < MAXCT; ++q) {
    int nt = tile_of<MAXCT>(pass, q, wave);
    nt = nt < nct ? nt : nct - 1;
    bq[q] = (uint32_t)(nt * nkb) * 512 * sizeof(T);
  }
  // Two register sets of B (and A) fragments, used in turn: the fragments of
  // K block kb + 1 are requested before the MFMAs of block kb.
  // Scheduling barriers keep the compiler from sinking those loads next to
  // their first use.
  F a0[NA], a1[NA], b0[MAXCT], b1[MAXCT], l0[kSplit ? MAXCT : 1], l1[kSplit ? MAXCT : 1];
  auto load = [&](F (&aa)[NA], F (&bb)[MAXCT], F (&ll)[kSplit ? MAXCT : 1], int kb) {
#pragma unroll
    for (int q = 0; q < MAXCT; ++q) {
      const uint32_t so = bq[q] + (uint32_t)kb * 512 * sizeof(T);
      bb[q] = P::load_buf(rb, loff, so);
      if constexpr (kSplit) ll[q] = P::load_buf(rb, loff, so + lo_bytes);
    }
    if constexpr (PREF_A) {
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) aa[rt] = P::load(Arow + rt * 16 * lda + kb * 32);
    }
    __builtin_amdgcn_sched_barrier(0);
  };
  auto clampk = [&](int k) { return k < kb1 ? k : kb1 - 1; };   // tail re-requests a loaded block
  // without PREF_A: the A fragment of the next (row tile, K block) step is
  // read from LDS before the MFMAs of the current one
  F anext;
  if constexpr (!PREF_A) anext = P::load(Arow + kb0 * 32);
  auto compute = [&](const F (&aa)[NA], const F (&bb)[MAXCT], const F (&ll)[kSplit ? MAXCT : 1], int kb) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      F a;
      if constexpr (PREF_A) {
        a = aa[PREF_A ? rt : 0];
      } else {
        a = anext;
        anext = rt + 1 < RT ? P::load(Arow + (rt + 1) * 16 * lda + kb * 32)
                            : P::load(Arow + clampk(kb + 1) * 32);
        __builtin_amdgcn_sched_barrier(0);
      }
      if constexpr (kSplit) {
#pragma unroll
        for (int q = 0; q < MAXCT; ++q) acc[rt][q] = P::mma(a, ll[q], acc[rt][q]);
      }
#pragma unroll
      for (int q = 0; q < MAXCT; ++q) acc[rt][q] = P::mma(a, bb[q], acc[rt][q]);
    }
    __builtin_amdgcn_sched_barrier(0);
  };
  load(a0, b0, l0, kb0);
  int kb = kb0;
  for (; kb + 1 < kb1; kb += 2) {
    load(a1, b1, l1, kb + 1);
    compute(a0, b0, l0, kb);
    load(a0, b0, l0, clampk(kb + 2));
    compute(a1, b1, l1, kb + 1);
  }
  if (kb < kb1) compute(a0, b0, l0, kb);
  // tiles clamped onto the last one hold copies: zero them so that register
  // uses of acc (gradients, dot products) see exact zeros there
#pragma unroll
  for (int q = 0; q < MAXCT; ++q)
    if (tile_of<MAXCT>(pass, q, wave) >= nct)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) acc[rt][q] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
}

// PREC 1 kernels take BF16 matrices with or without lo fragments (B.split,
// wave-uniform), so that a chain can mix paired and single-rounded layers.
template <int PREC, int RT, int MAXCT, bool PREF_A = true>
__device__ __forceinline__ void gemm_tile(f32x4 (&acc)[RT][MAXCT], const typename PT<PREC>::T* A,
                                          int lda, const GemmB& B, int wave, int lane, int pass,
                                          int kb0 = 0, int kb1 = -1, bool zero = true) {
  if constexpr (PREC == 1) {
    if (B.split)
      gemm_tile_k<PREC, RT, MAXCT, PREF_A, true>(acc, A, lda, B, wave, lane, pass, kb0, kb1, zero);
    else
      gemm_tile_k<PREC, RT, MAXCT, PREF_A, false>(acc, A, lda, B, wave, lane, pass, kb0, kb1, zero);
  } else {
    gemm_tile_k<PREC, RT, MAXCT, PREF_A, false>(acc, A, lda, B, wave, lane, pass, kb0, kb1, zero);
  }
}

template <class T> __device__ __forceinline__ T to_t(float v) { return (T)v; }

__device__ __forceinline__ void store4(__bf16* p, float4 v) {
  typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
  bf16x4 b = {(__bf16)v.x, (__bf16)v.y, (__bf16)v.z, (__bf16)v.w};
  *(bf16x4*)p = b;
}
__device__ __forceinline__ void store4(float* p, float4 v) { *(float4*)p = v; }

// 32-bit element offsets: one launch never addresses more than 2^31 floats
// of any edge-major array (the host splits larger edge sets into chunks).
__device__ __forceinline__ float4 ld4(const float* base, uint32_t off) { return *(const float4*)(base + off); }

// Copies float4 chunks of edge rows into X: for each row r of this wave's
// TM/kNW rows and chunk q < w4, X[r][c0 + 4q ..] = *src(e, c0 + 4q) for
// edges e0 + r < E (zero otherwise).  The (row, chunk) items are spread over
// the lanes and processed NB at a time with every load issued before the
// first store: a bulk gather costs one memory round trip per NB items per
// lane (one in all, for rows of up to 320 floats), the round trips being
// what these latency-bound kernels wait on.  `src` must return an in-range
// value for any e < E and column of the range.
template <int PREC, int TM, class Src>
__device__ __forceinline__ void gather_rows(typename PT<PREC>::T* X, int ldx, int e0, int E, int c0, int w4,
                                            Src src) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  constexpr int RPW = TM / kNW;
  constexpr int NB = TM >= 64 ? 12 : 8;
  const int total = RPW * w4;
  for (int t0 = 0; t0 < total; t0 += 64 * NB) {
    float4 v[NB];
    int off[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int t = t0 + lane + 64 * j;
      const int r = t / w4, q = t - r * w4;
      const int row = wave * RPW + (r < RPW ? r : RPW - 1);
      const int e = e0 + row;
      const bool ok = t < total && e < E;
      v[j] = src(ok ? e : E - 1, c0 + 4 * q);
      if (!ok) v[j] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      off[j] = t < total ? row * ldx + c0 + 4 * q : -1;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j)
      if (off[j] >= 0) store4(X + off[j], v[j]);
  }
}

// Zero columns [c0, c0 + 4 w4) of this wave's rows.
template <int PREC, int TM>
__device__ __forceinline__ void zero_cols(typename PT<PREC>::T* X, int ldx, int c0, int w4) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  constexpr int RPW = TM / kNW;
  for (int t = lane; t < RPW * w4; t += 64) {
    const int r = t / w4, q = t - r * w4;
    store4(X + (wave * RPW + r) * ldx + c0 + 4 * q, make_float4(0.0f, 0.0f, 0.0f, 0.0f));
  }
}

// Final-layer scalar tensor product for channels u..u+3 of edge e:
// T[u] = sum_c w_c V[c][u] Gamma[c][u] (V either stored or the rank-1
// first-layer form a0[l(c)][u] Y_c), over components C0 .. C0+NC-1 (those at
// or beyond dim weigh zero).
template <int C0, int NC>
__device__ __forceinline__ void final_tp_part(const MlpArgs& a, int e, int dim, uint32_t gbase, uint32_t vbase,
                                              float4& v) {
  float4 g[NC], vv[NC];
  float wy[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const int c = C0 + k;
    const bool on = c < dim;
    const int cc = on ? c : 0;
    const int l = c == 0 ? 0 : (c < 4 ? 1 : (c < 9 ? 2 : 3));
    g[k] = ld4(a.tp_gam, gbase + cc * a.n);
    vv[k] = ld4(a.tp_v.p, vbase + (a.tp_v.from_a0 ? (on ? l : 0) : cc) * a.n);
    wy[k] = on ? a.tp_w[c] * (a.tp_v.from_a0 ? a.eb[(uint32_t)e * kEB + eb_y(cc)] : 1.0f) : 0.0f;
  }
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const float w = wy[k];
    v.x = fmaf(w * vv[k].x, g[k].x, v.x);
    v.y = fmaf(w * vv[k].y, g[k].y, v.y);
    v.z = fmaf(w * vv[k].z, g[k].z, v.z);
    v.w = fmaf(w * vv[k].w, g[k].w, v.w);
  }
}

__device__ __forceinline__ float4 final_tp4(const MlpArgs& a, int e, int centre, int u) {
  const int dim = (a.l_max + 1) * (a.l_max + 1);
  const uint32_t gbase = (uint32_t)(centre - a.centre_base) * dim * a.n + u;
  const uint32_t vbase = (uint32_t)e * a.tp_v.ld + u;
  float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  final_tp_part<0, 9>(a, e, dim, gbase, vbase, v);
  if (dim > 9) final_tp_part<9, 7>(a, e, dim, gbase, vbase, v);   // l = 3
  return v;
}

// Input rows of the chain for edges e0 .. e0+TM-1, zero padded to Kp.
//   two-body: [onehot(Z_i), onehot(Z_j), R_0..R_{nb-1}]
//   latent:   [x^{L-1}, V^L[0] (or the final scalar tensor product)]
// STORED: the final layer's scalars are read from s_in (backward kernels;
// the host guarantees s_in), never recomputed.
template <int PREC, int KIND, int TM, bool STORED = false>
__device__ void build_input(const MlpArgs& a, typename PT<PREC>::T* X, int ldx, int e0, int Kp, int E) {
  using T = typename PT<PREC>::T;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  constexpr int RPW = TM / kNW;
  if constexpr (KIND == kTwoBody) {
    // one row per lane pass: the row's species pair, then its columns
    const int S = a.n_species, nb = a.n_bessel;
    for (int t = lane; t < RPW * (Kp >> 2); t += 64) {
      const int r = t / (Kp >> 2), q = t - r * (Kp >> 2);
      const int row = wave * RPW + r, e = e0 + row;
      const bool ok = e < E;
      const int ec = ok ? e : E - 1;
      const float* rec = a.eb + (uint32_t)ec * kEB;
      const int zi = (int)rec[kEB_ZI], zj = (int)rec[kEB_ZJ];
      float x[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int c = 4 * q + k;
        const int rc = c - 2 * S;
        const float rv = a.eb[(uint32_t)ec * kEB + kEB_R + (rc >= 0 && rc < nb ? rc : 0)];
        float v = c < S ? (zi == c ? 1.0f : 0.0f)
                        : c < 2 * S ? (zj == c - S ? 1.0f : 0.0f) : (rc < nb ? rv : 0.0f);
        x[k] = ok ? v : 0.0f;
      }
      store4(X + row * ldx + 4 * q, make_float4(x[0], x[1], x[2], x[3]));
    }
  } else {
  const int d = a.d, n = a.n;
  if (KIND == kLatent || STORED || a.s_in != nullptr) {
    // [x_prev | s] in one gather: s is V^L[0] (latent) or, for the final
    // layer, the tensor-product scalars its forward pass stored
    gather_rows<PREC, TM>(X, ldx, e0, E, 0, (d + n) >> 2, [&](int e, int c) {
      const float* p = c < d ? a.x_prev + (uint32_t)e * d + c : a.s_in + (uint32_t)e * a.s_ld + (c - d);
      return *(const float4*)p;
    });
  } else if constexpr (!STORED) {
    // final layer: the scalar tensor product of each (row, 4 channels) item,
    // NI items per lane at a time (a tile has at most TM/32 per lane).  The
    // centres of the first NI are requested before the x_prev gather so that
    // their latency overlaps it.
    constexpr int NI = TM >= 64 ? 2 : 1;
    const int w4 = n >> 2, total = RPW * w4;
    auto item_edge = [&](int t, int* row, int* q) {
      const int r = t / w4;
      *q = t - r * w4;
      *row = wave * RPW + r;
      return e0 + *row;
    };
    int cen[NI];
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      int row, q;
      const int e = item_edge(lane + 64 * j, &row, &q);
      cen[j] = a.ei[e < E ? e : E - 1];
    }
    gather_rows<PREC, TM>(X, ldx, e0, E, 0, d >> 2,
                          [&](int e, int c) { return ld4(a.x_prev, (uint32_t)e * d + c); });
    for (int t0 = 0; t0 < total; t0 += 64 * NI) {
      if (t0 > 0) {
#pragma unroll
        for (int j = 0; j < NI; ++j) {
          int row, q;
          const int e = item_edge(t0 + lane + 64 * j, &row, &q);
          cen[j] = a.ei[e < E ? e : E - 1];
        }
      }
      float4 v[NI];
#pragma unroll
      for (int j = 0; j < NI; ++j) {
        int row, q;
        const int e = item_edge(t0 + lane + 64 * j, &row, &q);
        v[j] = final_tp4(a, e < E ? e : E - 1, cen[j], 4 * q);
      }
#pragma unroll
      for (int j = 0; j < NI; ++j) {
        const int t = t0 + lane + 64 * j;
        int row, q;
        const int e = item_edge(t, &row, &q);
        if (t >= total) continue;
        float4 vv = v[j];
        if (e >= E) vv = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        else if (a.tp_out) *(float4*)(a.tp_out + (uint32_t)e * n + 4 * q) = vv;
        store4(X + row * ldx + d + 4 * q, vv);
      }
    }
  }
  if (Kp > d + n) zero_cols<PREC, TM>(X, ldx, d + n, (Kp - d - n) >> 2);
  }
}

// Rows of a row-major FP32 matrix (row stride ld, ncols columns, a multiple
// of 4) into X, columns [c0, c0+w) (zero beyond ncols).
template <int PREC, int TM>
__device__ void stage_rows(const float* src, int ld, int ncols, int E, typename PT<PREC>::T* X, int ldx,
                           int e0, int c0, int w) {
  gather_rows<PREC, TM>(X, ldx, e0, E, 0, w >> 2, [&](int e, int c) {
    const int cc = c0 + c;
    float4 v = ld4(src, (uint32_t)e * ld + (cc < ncols ? cc : ncols - 4));
    if (cc >= ncols) v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    return v;
  });
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

// Short tiles (32 BF16 / 16 FP32 rows) are compiled for four waves per SIMD
// (<= 128 VGPRs) so that two blocks share a CU: one block's gathers and
// barriers then overlap the other's MFMAs.
template <int PREC, int TM>
constexpr int kWavesPerEu = TM * (PREC ? 1 : 2) <= 32 ? 4 : 1;

template <int PREC, int KIND, int TM, int MAXCT>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kWavesPerEu<PREC, TM>, 8)))
void k_mlp_fwd(MlpArgs a, int ldx, int ldh) {
  const int E = live_edges(a);
  if ((int)blockIdx.x * TM >= E) return;   // tiles beyond the live edges (capacity launches)
  using P = PT<PREC>;
  using T = typename P::T;
  constexpr int RT = TM / 16;
  extern __shared__ __align__(16) char smem[];
  T* X = (T*)smem;
  T* H = X + TM * ldx;
  __shared__ float red[kNW][TM];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int e0 = blockIdx.x * TM;

  // The epilogue's per-row inputs (u, and the residual x_prev in this lane's
  // fragment layout) are requested together with the input gather, so that
  // their latency overlaps it instead of following the last GEMM -- except in
  // the final layer's 32-row kernel, whose input build (the tensor-product
  // scalars) leaves no registers for them under the two-blocks-per-CU limit.
  constexpr bool kEarly = KIND == kLatent || TM >= 64;
  const int d = a.d;
  float ur[RT][4];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int e = e0 + rt * 16 + 4 * (lane >> 4) + i;
      ur[rt][i] = e < E ? a.eb[(uint32_t)e * kEB + kEB_U] : 0.0f;
    }
  float xp[RT][MAXCT][4];
  auto load_xp = [&] {
#pragma unroll
    for (int q = 0; q < MAXCT; ++q) {
      int col = tile_of<MAXCT>(0, q, wave) * 16 + (lane & 15);
      col = col < d ? col : d - 1;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          int e = e0 + rt * 16 + 4 * (lane >> 4) + i;
          e = e < E ? e : E - 1;
          xp[rt][q][i] = a.x_prev[(uint32_t)e * d + col];
        }
    }
  };
  if constexpr (KIND != kTwoBody && kEarly) load_xp();
  build_input<PREC, KIND, TM>(a, X, ldx, e0, a.w.fwd[0].Kp, E);
  __syncthreads();
  int ldin;
  const T* in = hidden_layers<PREC, TM, MAXCT>(a, X, ldx, H, ldh, nullptr, 0, &ldin, wave, lane);
  const int nl = a.w.nl;
  f32x4 acc[RT][MAXCT];
  gemm_tile<PREC, RT, MAXCT>(acc, in, ldin, a.w.fwd[nl - 1], wave, lane, 0);   // N = d: one pass
  // epilogue: x = u h (two-body) or rs (x_prev + u h) (latent), kept in acc
  if constexpr (KIND != kTwoBody) {
    if constexpr (!kEarly) load_xp();
#pragma unroll
    for (int q = 0; q < MAXCT; ++q)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[rt][q][i] = a.res_scale * (xp[rt][q][i] + ur[rt][i] * acc[rt][q][i]);
  } else {
#pragma unroll
    for (int q = 0; q < MAXCT; ++q)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[rt][q][i] = ur[rt][i] * acc[rt][q][i];
  }
  // rows beyond E and clamped column tiles hold zeros
#pragma unroll
  for (int q = 0; q < MAXCT; ++q) {
    const int col = tile_of<MAXCT>(0, q, wave) * 16 + (lane & 15);
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int e = e0 + rt * 16 + 4 * (lane >> 4) + i;
        const bool ok = e < E && col < d;
        if (!ok) acc[rt][q][i] = 0.0f;
        if (ok && a.x_out) a.x_out[(uint32_t)e * d + col] = acc[rt][q][i];
      }
  }
  if constexpr (KIND == kLatentFinal) {
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
        sum = group_sum_dpp<16>(sum);
        if ((lane & 15) == 0) red[wave][rt * 16 + 4 * (lane >> 4) + i] = sum;
      }
    __syncthreads();
    if ((int)threadIdx.x < TM) {
      const int e = e0 + threadIdx.x;
      if (e < E)
        a.eij[e] = wave_partials_sum(red, threadIdx.x);
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
          if (e < E) a.head_out[(size_t)e * Nh + col] = acc[rt][q][i];
        }
    }
  }
}

template <int PREC, int KIND, int TM, int MAXCT>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kWavesPerEu<PREC, TM>, 8)))
void k_mlp_bwd(MlpArgs a, int ldx, int ldh) {
  const int E = live_edges(a);
  if ((int)blockIdx.x * TM >= E) return;   // tiles beyond the live edges (capacity launches)
  using P = PT<PREC>;
  using T = typename P::T;
  constexpr int RT = TM / 16;
  extern __shared__ __align__(16) char smem[];
  T* X = (T*)smem;
  T* H = X + TM * ldx;
  T* Pb = H + TM * ldh;                 // nl-1 pre-activation buffers [TM][ldh]
  __shared__ float red[kNW][TM];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int e0 = blockIdx.x * TM;
  const int d = a.d;
  const int nl = a.w.nl;

  // 1. G = dE/dx_out (columns < d all lie in pass 0); loads first, then masks
  f32x4 G[RT][MAXCT];
  {
    const float* gsrc = KIND == kLatentFinal ? a.g_const : a.g_x;
    uint32_t rowoff[RT][4];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int e = e0 + rt * 16 + 4 * (lane >> 4) + i;
        e = e < E ? e : E - 1;
        rowoff[rt][i] = (uint32_t)(KIND == kLatentFinal ? (int)a.eb[(uint32_t)e * kEB + kEB_ZI] : e) * d;
      }
#pragma unroll
    for (int q = 0; q < MAXCT; ++q) {
      const int col = tile_of<MAXCT>(0, q, wave) * 16 + (lane & 15);
      const int cc = col < d ? col : d - 1;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) G[rt][q][i] = gsrc ? gsrc[rowoff[rt][i] + cc] : 0.0f;
    }
  }
  // G is masked (rows beyond E, columns beyond d) only after the head part,
  // so that its loads and the head staging loads are in flight together
  auto mask_g = [&] {
#pragma unroll
    for (int q = 0; q < MAXCT; ++q) {
      const int col = tile_of<MAXCT>(0, q, wave) * 16 + (lane & 15);
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int e = e0 + rt * 16 + 4 * (lane >> 4) + i;
          if (!(e < E && col < d)) G[rt][q][i] = 0.0f;
        }
    }
  };
  // u of the tile's rows (zero beyond E), kept in LDS until the chain is recomputed
  __shared__ float us[TM];
  if ((int)threadIdx.x < TM) {
    const int e = e0 + threadIdx.x;
    us[threadIdx.x] = e < E ? a.eb[(uint32_t)e * kEB + kEB_U] : 0.0f;
  }
  f32x4 acc[RT][MAXCT];
  bool input_ready = false;
  if (KIND != kLatentFinal && a.head_bwd.p != nullptr) {
    // G += g_head @ W_head^T
    const int Kh = a.head_bwd.K, nkb = a.head_bwd.Kp >> 5;
    const int ldg = a.head_bwd.Kp + (PREC ? 8 : 4);
    if (ldg <= nl * ldh) {
      // the whole head gradient fits the H / pre-activation region (a
      // [TM][ldg] view of it): stage it there while the chain's input rows
      // gather into X, both in one memory round trip
      stage_rows<PREC, TM>(a.g_head, Kh, Kh, E, H, ldg, e0, 0, nkb * 32);
      build_input<PREC, KIND, TM, true>(a, X, ldx, e0, a.w.fwd[0].Kp, E);
      __syncthreads();
      gemm_tile<PREC, RT, MAXCT>(acc, H, ldg, a.head_bwd, wave, lane, 0);
      __syncthreads();   // H is rewritten by the recomputation
      input_ready = true;
    } else {
      // K staged through X in chunks of its width
      const int chunk = ldx >> 5;
      for (int kb0 = 0; kb0 < nkb; kb0 += chunk) {
        const int kb1 = kb0 + chunk < nkb ? kb0 + chunk : nkb;
        const int w = (kb1 - kb0) * 32;
        stage_rows<PREC, TM>(a.g_head, Kh, Kh, E, X, ldx, e0, kb0 * 32, w);
        __syncthreads();
        gemm_tile<PREC, RT, MAXCT>(acc, X, ldx, a.head_bwd, wave, lane, 0, kb0, kb1, kb0 == 0);
        __syncthreads();
      }
    }
    // (the K sum continues across chunks in the accumulators); G = g_x + sum
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int q = 0; q < MAXCT; ++q) G[rt][q] += acc[rt][q];
  }
  mask_g();

  // 2. recompute the chain, keeping hidden pre-activations
  if (!input_ready) {
    build_input<PREC, KIND, TM, true>(a, X, ldx, e0, a.w.fwd[0].Kp, E);
    __syncthreads();
  }
  int ldin;
  const T* in = hidden_layers<PREC, TM, MAXCT>(a, X, ldx, H, ldh, Pb, ldh, &ldin, wave, lane);
  gemm_tile<PREC, RT, MAXCT>(acc, in, ldin, a.w.fwd[nl - 1], wave, lane, 0);   // acc = h
  const float rs = (KIND == kTwoBody) ? 1.0f : a.res_scale;
  // dE/du = rs sum_c G h
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float sum = 0.0f;
#pragma unroll
      for (int q = 0; q < MAXCT; ++q) sum = fmaf(G[rt][q][i], acc[rt][q][i], sum);
      sum = group_sum_dpp<16>(sum);
      if ((lane & 15) == 0) red[wave][rt * 16 + 4 * (lane >> 4) + i] = sum;
    }
  __syncthreads();   // also: every wave is done reading `in`
  if ((int)threadIdx.x < TM) {
    const int e = e0 + threadIdx.x;
    if (e < E) {
      const float gu = rs * wave_partials_sum(red, threadIdx.x);
      a.g_u[e] = a.gu_accum ? a.g_u[e] + gu : gu;
    }
  }
  // dE/dh = rs u G into the buffer the last layer did not read
  T* cur = (in == X) ? H : X;
  int ldc = (in == X) ? ldh : ldx;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int q = 0; q < MAXCT; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[rt][q][i] = rs * us[rt * 16 + 4 * (lane >> 4) + i] * G[rt][q][i];
  store_tile<PREC, RT, MAXCT>(acc, cur, ldc, a.w.fwd[nl - 1].Np, wave, lane, 0,
                              [](float v, int, int) { return v; });
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
          if (e >= E) continue;
          const float g = acc[rt][q][i];
          if constexpr (KIND == kTwoBody) {
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

// ---------------------------------------------------------------------------
// Tall tiles: 128 edges per block.  Every wave computes all 128 rows of its
// column tiles (RT = 8), so each weight fragment read from L2 feeds eight row
// tiles (half the L2 traffic per MFMA of a 64-row tile).  Activations live in
// one LDS buffer and are updated in place: a layer's output overwrites its
// input after a barrier.  Requires every hidden width to fit one pass
// (<= 16 kNW MAXCT columns).  The backward kernel writes the hidden
// pre-activations of its recomputation to a global scratch array in register
// (fragment) order, and dE/dx_out to the output row it is added to at the
// end.  Per element the arithmetic is the same as in the 64- and 32-row
// kernels, so all tile shapes give identical results.
constexpr int kTallRows = 128;

// Scratch slot of fragment (rt, q) of this wave for hidden layer l.
template <int MAXCT>
__device__ __forceinline__ size_t zslot(int l, int wave, int q, int rt, int lane) {
  return (((((size_t)blockIdx.x * 2 + l) * kNW + wave) * MAXCT + q) * 8 + rt) * 64 + lane;
}

template <int PREC, int KIND, int MAXCT>
__global__ __launch_bounds__(kThreads, 1) void k_mlp_fwd_t(MlpArgs a, int ldx, int) {
  const int E = live_edges(a);
  if ((int)blockIdx.x * kTallRows >= E) return;   // tiles beyond the live edges (capacity launches)
  using T = typename PT<PREC>::T;
  constexpr int TM = kTallRows, RT = 8;
  extern __shared__ __align__(16) char smem[];
  T* X = (T*)smem;
  __shared__ float red[kNW][TM];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int e0 = blockIdx.x * TM;
  const int d = a.d, nl = a.w.nl;

  build_input<PREC, KIND, TM>(a, X, ldx, e0, a.w.fwd[0].Kp, E);
  __syncthreads();
  f32x4 acc[RT][MAXCT];
  for (int l = 0; l + 1 < nl; ++l) {
    gemm_tile<PREC, RT, MAXCT, false>(acc, X, ldx, a.w.fwd[l], wave, lane, 0);
    __syncthreads();
    store_tile<PREC, RT, MAXCT>(acc, X, ldx, a.w.fwd[l].Np, wave, lane, 0,
                                [](float v, int, int) { return silu(v); });
    __syncthreads();
  }
  gemm_tile<PREC, RT, MAXCT, false>(acc, X, ldx, a.w.fwd[nl - 1], wave, lane, 0);
  // epilogue in row-tile pairs (loads of a pair issued together):
  // x = u h (two-body) or rs (x_prev + u h), zero beyond E and d
#pragma unroll
  for (int r0 = 0; r0 < RT; r0 += 2) {
    float ur[2][4], xp[2][MAXCT][4];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int e = e0 + (r0 + h) * 16 + 4 * (lane >> 4) + i;
        e = e < E ? e : E - 1;
        ur[h][i] = a.eb[(uint32_t)e * kEB + kEB_U];
        if constexpr (KIND != kTwoBody) {
#pragma unroll
          for (int q = 0; q < MAXCT; ++q) {
            int col = tile_of<MAXCT>(0, q, wave) * 16 + (lane & 15);
            col = col < d ? col : d - 1;
            xp[h][q][i] = a.x_prev[(uint32_t)e * d + col];
          }
        }
      }
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int q = 0; q < MAXCT; ++q) {
        const int col = tile_of<MAXCT>(0, q, wave) * 16 + (lane & 15);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int e = e0 + (r0 + h) * 16 + 4 * (lane >> 4) + i;
          float v = ur[h][i] * acc[r0 + h][q][i];
          if constexpr (KIND != kTwoBody) v = a.res_scale * (xp[h][q][i] + v);
          const bool ok = e < E && col < d;
          v = ok ? v : 0.0f;
          acc[r0 + h][q][i] = v;
          if (ok && a.x_out) a.x_out[(uint32_t)e * d + col] = v;
        }
      }
  }
  if constexpr (KIND == kLatentFinal) {
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
        sum = group_sum_dpp<16>(sum);
        if ((lane & 15) == 0) red[wave][rt * 16 + 4 * (lane >> 4) + i] = sum;
      }
    __syncthreads();
    if ((int)threadIdx.x < TM) {
      const int e = e0 + threadIdx.x;
      if (e < E)
        a.eij[e] = wave_partials_sum(red, threadIdx.x);
    }
    return;
  } else {
    if (a.head.p == nullptr) return;
    __syncthreads();   // every wave is done reading X
    store_tile<PREC, RT, MAXCT>(acc, X, ldx, a.w.fwd[nl - 1].Np, wave, lane, 0, [](float v, int, int) { return v; });
    __syncthreads();
    const int Nh = a.head.N;
    for (int p = 0; p < npasses<MAXCT>(a.head.Np); ++p) {
      gemm_tile<PREC, RT, MAXCT, false>(acc, X, ldx, a.head, wave, lane, p);
#pragma unroll
      for (int q = 0; q < MAXCT; ++q) {
        const int col = tile_of<MAXCT>(p, q, wave) * 16 + (lane & 15);
        if (col >= Nh) continue;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int e = e0 + rt * 16 + 4 * (lane >> 4) + i;
            if (e < E) a.head_out[(uint32_t)e * Nh + col] = acc[rt][q][i];
          }
      }
    }
  }
}

template <int PREC, int KIND, int MAXCT>
__global__ __launch_bounds__(kThreads, 1) void k_mlp_bwd_t(MlpArgs a, int ldx, int) {
  const int E = live_edges(a);
  if ((int)blockIdx.x * kTallRows >= E) return;   // tiles beyond the live edges (capacity launches)
  using T = typename PT<PREC>::T;
  typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
  constexpr int TM = kTallRows, RT = 8;
  extern __shared__ __align__(16) char smem[];
  T* X = (T*)smem;
  __shared__ float red[kNW][TM];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int e0 = blockIdx.x * TM;
  const int d = a.d, nl = a.w.nl;
  const float rs = (KIND == kTwoBody) ? 1.0f : a.res_scale;
  bf16x4* zs = (bf16x4*)a.act_scratch;
  float* gst = a.g_store;

  // 1. G = dE/dx_out -> g_store (head part on MFMA, K staged through X)
  f32x4 acc[RT][MAXCT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int q = 0; q < MAXCT; ++q) acc[rt][q] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  if constexpr (KIND != kLatentFinal) {
    if (a.head_bwd.p != nullptr) {
      const int Kh = a.head_bwd.K, nkb = a.head_bwd.Kp >> 5, chunk = ldx >> 5;
      for (int kb0 = 0; kb0 < nkb; kb0 += chunk) {
        const int kb1 = kb0 + chunk < nkb ? kb0 + chunk : nkb;
        stage_rows<PREC, TM>(a.g_head, Kh, Kh, E, X, ldx, e0, kb0 * 32, (kb1 - kb0) * 32);
        __syncthreads();
        gemm_tile<PREC, RT, MAXCT, false>(acc, X, ldx, a.head_bwd, wave, lane, 0, kb0, kb1, false);
        __syncthreads();
      }
    }
  }
  {
    const float* gsrc = KIND == kLatentFinal ? a.g_const : a.g_x;
#pragma unroll
    for (int r0 = 0; r0 < RT; r0 += 2) {
      float gv[2][MAXCT][4];
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          int e = e0 + (r0 + h) * 16 + 4 * (lane >> 4) + i;
          e = e < E ? e : E - 1;
          const uint32_t ro = (uint32_t)(KIND == kLatentFinal ? (int)a.eb[(uint32_t)e * kEB + kEB_ZI] : e) * d;
#pragma unroll
          for (int q = 0; q < MAXCT; ++q) {
            int col = tile_of<MAXCT>(0, q, wave) * 16 + (lane & 15);
            col = col < d ? col : d - 1;
            gv[h][q][i] = gsrc ? gsrc[ro + col] : 0.0f;
          }
        }
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int q = 0; q < MAXCT; ++q) {
          const int col = tile_of<MAXCT>(0, q, wave) * 16 + (lane & 15);
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int e = e0 + (r0 + h) * 16 + 4 * (lane >> 4) + i;
            if (e < E && col < d) gst[(uint32_t)e * d + col] = gv[h][q][i] + acc[r0 + h][q][i];
          }
        }
    }
  }

  // 2. recompute the chain; hidden pre-activations to the scratch array
  build_input<PREC, KIND, TM, true>(a, X, ldx, e0, a.w.fwd[0].Kp, E);
  __syncthreads();
  for (int l = 0; l + 1 < nl; ++l) {
    gemm_tile<PREC, RT, MAXCT, false>(acc, X, ldx, a.w.fwd[l], wave, lane, 0);
#pragma unroll
    for (int q = 0; q < MAXCT; ++q)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const f32x4 v = acc[rt][q];
        zs[zslot<MAXCT>(l, wave, q, rt, lane)] = bf16x4{(__bf16)v[0], (__bf16)v[1], (__bf16)v[2], (__bf16)v[3]};
      }
    __syncthreads();
    store_tile<PREC, RT, MAXCT>(acc, X, ldx, a.w.fwd[l].Np, wave, lane, 0,
                                [](float v, int, int) { return silu(v); });
    __syncthreads();
  }
  gemm_tile<PREC, RT, MAXCT, false>(acc, X, ldx, a.w.fwd[nl - 1], wave, lane, 0);   // acc = h

  // 3. dE/du = rs sum_c G h ; dE/dh = rs u G
#pragma unroll
  for (int r0 = 0; r0 < RT; r0 += 2) {
    float gv[2][MAXCT][4], ur[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int e = e0 + (r0 + h) * 16 + 4 * (lane >> 4) + i;
        const bool ok = e < E;
        e = ok ? e : E - 1;
        ur[h][i] = ok ? a.eb[(uint32_t)e * kEB + kEB_U] : 0.0f;
#pragma unroll
        for (int q = 0; q < MAXCT; ++q) {
          int col = tile_of<MAXCT>(0, q, wave) * 16 + (lane & 15);
          const bool okc = ok && col < d;
          col = col < d ? col : d - 1;
          const float g = gst[(uint32_t)e * d + col];
          gv[h][q][i] = okc ? g : 0.0f;
        }
      }
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float sum = 0.0f;
#pragma unroll
        for (int q = 0; q < MAXCT; ++q) {
          sum = fmaf(gv[h][q][i], acc[r0 + h][q][i], sum);
          acc[r0 + h][q][i] = rs * ur[h][i] * gv[h][q][i];
        }
        sum = group_sum_dpp<16>(sum);
        if ((lane & 15) == 0) red[wave][(r0 + h) * 16 + 4 * (lane >> 4) + i] = sum;
      }
  }
  __syncthreads();   // red complete; every wave is done reading X
  if ((int)threadIdx.x < TM) {
    const int e = e0 + threadIdx.x;
    if (e < E) {
      const float gu = rs * wave_partials_sum(red, threadIdx.x);
      a.g_u[e] = a.gu_accum ? a.g_u[e] + gu : gu;
    }
  }
  store_tile<PREC, RT, MAXCT>(acc, X, ldx, a.w.fwd[nl - 1].Np, wave, lane, 0, [](float v, int, int) { return v; });
  __syncthreads();

  // 4. back through the hidden layers, in place
  for (int l = nl - 1; l > 0; --l) {
    gemm_tile<PREC, RT, MAXCT, false>(acc, X, ldx, a.w.bwd[l], wave, lane, 0);
#pragma unroll
    for (int q = 0; q < MAXCT; ++q)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const bf16x4 z = zs[zslot<MAXCT>(l - 1, wave, q, rt, lane)];
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[rt][q][i] *= silu_grad((float)z[i]);
      }
    __syncthreads();
    store_tile<PREC, RT, MAXCT>(acc, X, ldx, a.w.bwd[l].Np, wave, lane, 0, [](float v, int, int) { return v; });
    __syncthreads();
  }

  // 5. dE/dz, written to the outputs (g_xprev holds dE/dx_out)
  const int S = a.n_species;
  const GemmB& B0 = a.w.bwd[0];
  for (int p = 0; p < npasses<MAXCT>(B0.Np); ++p) {
    gemm_tile<PREC, RT, MAXCT, false>(acc, X, ldx, B0, wave, lane, p);
#pragma unroll
    for (int q = 0; q < MAXCT; ++q) {
      const int col = tile_of<MAXCT>(p, q, wave) * 16 + (lane & 15);
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int e = e0 + rt * 16 + 4 * (lane >> 4) + i;
          if (e >= E) continue;
          const float g = acc[rt][q][i];
          if constexpr (KIND == kTwoBody) {
            if (col >= 2 * S && col < 2 * S + a.n_bessel) a.g_R[(uint32_t)e * a.n_bessel + col - 2 * S] = g;
          } else if (col < d) {
            float* o = a.g_xprev + (uint32_t)e * d + col;
            *o = rs * *o + g;
          } else if (col < d + a.n) {
            a.g_s[(uint32_t)e * a.n + col - d] = g;
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
  const int kx = kh > a.w.fwd[0].Kp ? kh : a.w.fwd[0].Kp;
  const int pad = PREC ? 8 : 4;
  *ldx = kx + pad;
  *ldh = kh + pad;
  const int nbuf_h = bwd ? a.w.nl : 1;
  *bytes = (size_t)TM * ((size_t)*ldx + (size_t)nbuf_h * *ldh) * (PREC ? 2 : 4);
}

// Accumulator tiles per wave: the latent width d must fit one pass.
inline int max_ct(const MlpArgs& a) {
  const int dt = (a.d + 15) / 16;
  return (dt + kNW - 1) / kNW;
}

// Tall tiles (BF16 only): one LDS buffer [128][ldx]; every hidden width and
// d must fit one pass of 64 MAXCT columns; the backward kernel needs its
// scratch arrays.
inline bool tall_ok(const MlpArgs& a, int prec, bool bwd) {
  if (prec == 0) return false;
  const int cols = 16 * kNW * max_ct(a);
  for (int l = 0; l < a.w.nl; ++l)
    if (a.w.fwd[l].Np > cols) return false;
  if (bwd && (a.g_store == nullptr || (a.w.nl > 1 && a.act_scratch == nullptr))) return false;
  return a.w.nl <= 3;
}

inline void tall_dims(const MlpArgs& a, bool bwd, int* ldx, size_t* bytes) {
  int k = a.w.fwd[0].Kp;
  for (int l = 0; l < a.w.nl; ++l) k = k > a.w.fwd[l].Np ? k : a.w.fwd[l].Np;
  if (bwd && a.head_bwd.p != nullptr && a.head_bwd.Kp > k) k = a.head_bwd.Kp;
  *ldx = k + 8;
  *bytes = (size_t)kTallRows * *ldx * 2;
}

// Bytes of the pre-activation scratch array for E rows (two hidden layers of
// 64 MAXCT columns per 128-row tile, BF16).
inline size_t tall_scratch_bytes(int64_t E, int d) {
  const int ct = ((d + 15) / 16 + kNW - 1) / kNW;
  return (size_t)((E + kTallRows - 1) / kTallRows) * 2 * kTallRows * 16 * kNW * ct * 2;
}

constexpr size_t kLdsLimit = 160 * 1024 - 4096;

template <int PREC, int KIND, int TM, int MAXCT>
hipError_t launch_one(const MlpArgs& a, bool bwd, hipStream_t s) {
  int ldx, ldh;
  size_t bytes;
  lds_dims<PREC>(a, TM, bwd, &ldx, &ldh, &bytes);
  const dim3 grid((a.E + TM - 1) / TM), block(kThreads);
  auto k = bwd ? k_mlp_bwd<PREC, KIND, TM, MAXCT> : k_mlp_fwd<PREC, KIND, TM, MAXCT>;
  hipError_t st = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (st != hipSuccess) return st;
  hipLaunchKernelGGL(k, grid, block, bytes, s, a, ldx, ldh);
  return hipGetLastError();
}

template <int PREC, int KIND, int MAXCT>
hipError_t launch_tall(const MlpArgs& a, bool bwd, hipStream_t s) {
  int ldx;
  size_t bytes;
  tall_dims(a, bwd, &ldx, &bytes);
  const dim3 grid((a.E + kTallRows - 1) / kTallRows), block(kThreads);
  auto k = bwd ? k_mlp_bwd_t<PREC, KIND, MAXCT> : k_mlp_fwd_t<PREC, KIND, MAXCT>;
  hipError_t st = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (st != hipSuccess) return st;
  hipLaunchKernelGGL(k, grid, block, bytes, s, a, ldx, 0);
  return hipGetLastError();
}

template <int PREC, int KIND>
hipError_t dispatch_tall(const MlpArgs& a, bool bwd, hipStream_t s) {
  const int ct = max_ct(a);
  if (ct <= 1) return launch_tall<PREC, KIND, 1>(a, bwd, s);
  if (ct <= 2) return launch_tall<PREC, KIND, 2>(a, bwd, s);
  return hipErrorInvalidValue;
}

// d <= 256 (the interface's limit): at most two column tiles per wave
template <int PREC, int KIND, int TM>
hipError_t dispatch_ct(const MlpArgs& a, bool bwd, hipStream_t s) {
  const int ct = max_ct(a);
  if (ct <= 1) return launch_one<PREC, KIND, TM, 1>(a, bwd, s);
  if (ct <= 2) return launch_one<PREC, KIND, TM, 2>(a, bwd, s);
  return hipErrorInvalidValue;
}

// Tile rows per precision: {larger, smaller}.
template <int PREC> constexpr int kTileRows[2] = {PREC ? 64 : 32, PREC ? 32 : 16};

// Launches the chain of `a` (kind a.kind) with TM rows per tile (one of
// kTileRows<PREC>); instantiated once per precision in its own source file.
template <int PREC>
hipError_t launch_prec(const MlpArgs& a, int tm, bool bwd, hipStream_t s) {
  constexpr int T0 = kTileRows<PREC>[0], T1 = kTileRows<PREC>[1];
  if constexpr (PREC != 0) {
    if (tm == kTallRows) {
      switch (a.kind) {
        case kTwoBody: return dispatch_tall<PREC, kTwoBody>(a, bwd, s);
        case kLatent: return dispatch_tall<PREC, kLatent>(a, bwd, s);
        case kLatentFinal: return dispatch_tall<PREC, kLatentFinal>(a, bwd, s);
      }
      return hipErrorInvalidValue;
    }
  }
  switch (a.kind) {
    case kTwoBody:
      return tm == T0 ? dispatch_ct<PREC, kTwoBody, T0>(a, bwd, s) : dispatch_ct<PREC, kTwoBody, T1>(a, bwd, s);
    case kLatent:
      return tm == T0 ? dispatch_ct<PREC, kLatent, T0>(a, bwd, s) : dispatch_ct<PREC, kLatent, T1>(a, bwd, s);
    case kLatentFinal:
      return tm == T0 ? dispatch_ct<PREC, kLatentFinal, T0>(a, bwd, s)
                      : dispatch_ct<PREC, kLatentFinal, T1>(a, bwd, s);
  }
  return hipErrorInvalidValue;
}

extern template hipError_t launch_prec<0>(const MlpArgs&, int, bool, hipStream_t);
extern template hipError_t launch_prec<1>(const MlpArgs&, int, bool, hipStream_t);
extern template hipError_t launch_prec<2>(const MlpArgs&, int, bool, hipStream_t);

}  // namespace mlpk
}  // namespace allegro
