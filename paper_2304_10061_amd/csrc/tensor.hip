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
// a dense contraction over channels run on FP32 MFMA, or, in the BF16 modes,
// as three BF16 MFMAs per product: with x = x_hi + x_lo split into two BF16
// numbers for both operands, hi*hi + hi*lo + lo*hi keeps about 16
// significant bits (more than the TF32 of section "Mixed-precision
// calculations") at a fifth of the FP32 MFMA time.
//
// Deeper models (three or more layers) also carry unnatural-parity irreps
// (1e, 2o, 3e): the features of those layers hold 2 dim components (natural
// block, then unnatural block), and each (l, parity) has its own mixing
// matrix.  Kernels are instantiated per pattern, TpPattern<l_max, input kind,
// output kind>.
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

constexpr int lof(int c) { return l_of(c); }

// Mixing-matrix slot of strided component c of a feature with D natural components.
template <int LMAX>
constexpr int mix_slot(int c) {
  constexpr int D = (LMAX + 1) * (LMAX + 1);
  return c < D ? l_of(c) : LMAX + 1 + l_of(c - D);
}

// Fused-table weights: by value for small tables, else from device memory
// read through the constant address space (the table is not written while a
// kernel runs), which lets the compiler use scalar loads.
typedef const __attribute__((address_space(4))) float* ConstFloatPtr;

template <class Pat>
__device__ __forceinline__ auto tp_weights(const TensorArgs& a) {
  if constexpr (Pat::NNZ <= kTpwArgs) return (const float*)a.tpw_v;
  else return (ConstFloatPtr)a.tpw;
}

// Inside a loop, a large table's pointer is passed through an empty asm
// statement at each iteration: its loads then stay inside the loop instead of
// being hoisted out of it, which would keep hundreds of loop-invariant
// weights live in registers.  The kernel-argument array is returned as is.
__device__ __forceinline__ const float* per_iteration(const float* w) { return w; }
__device__ __forceinline__ ConstFloatPtr per_iteration(ConstFloatPtr w) {
  asm volatile("" : "+s"(w));
  return w;
}

template <int LMAX, int DIN>
__device__ __forceinline__ void load_v(const VSrc& v, const float* eb_e, int64_t e, int u, int n,
                                       float* V) {
  constexpr int DIM = (LMAX + 1) * (LMAX + 1);
  const float* p = v.p + (size_t)e * v.ld + u;
  if (v.from_a0) {
    static_assert(DIN >= DIM, "first-layer features are natural");
    float a0[LMAX + 1];
#pragma unroll
    for (int l = 0; l <= LMAX; ++l) a0[l] = p[l * n];
#pragma unroll
    for (int c = 0; c < DIM; ++c) V[c] = a0[lof(c)] * eb_e[eb_y(c)];
#pragma unroll
    for (int c = DIM; c < DIN; ++c) V[c] = 0.0f;
  } else {
#pragma unroll
    for (int c = 0; c < DIN; ++c) V[c] = p[c * n];
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
    for (int b = 0; b < DIM; ++b) acc[b] = fmaf(wl[lof(b)], Y[eb_y(b)], acc[b]);
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
// Edge-tile kernels staging a [w][TT][n] block in LDS, then mixing channels
// on MFMA.  B operands are the packed mixing matrices (one per irrep slot).

__device__ __forceinline__ f32x4 mma8(const float* a, const float* b, f32x4 c) {
  // the K = 32 block as eight K = 4 steps (lane group g holds k = 8 g + s)
#pragma unroll
  for (int s = 0; s < 8; ++s) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], b[s], c, 0, 0, 0);
  return c;
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// The K = 32 block in one step per product term: lane group g holds
// k = 8 g .. 8 g + 7, the same assignment as mma8's.
__device__ __forceinline__ f32x4 mma3(const bf16x8& ah, const bf16x8& al, const bf16x8& bh, const bf16x8& bl,
                                      f32x4 c) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
}

// x = hi + lo with hi = bf16(x), lo = bf16(x - hi).
__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

// Channel mixing out[e][c][v] = scale * sum_k S[c][e][k] B_{slot(c)}[k][v] for
// the rows of an edge tile.  Each wave owns one 16-wide column tile of the
// output (with fewer column tiles than waves, the waves also split the
// components).  Natural-parity layers keep the B fragments of every slot in
// registers for all the tiles a block processes; the wider parity layouts,
// whose tensor-product phase needs those registers, load one slot's
// fragments per component instead.
constexpr int kMixKB = 2;   // K = n <= 64

// B fragments of NS slots: FP32, or (BF3) split into BF16 hi and lo parts.
template <int NS, bool BF3 = false>
struct MixB {
  float b[NS][kMixKB][8];
  int nt, csub, wpt;
};
template <int NS>
struct MixB<NS, true> {
  bf16x8 bh[NS][kMixKB], bl[NS][kMixKB];
  int nt, csub, wpt;
};

template <class MB>
__device__ __forceinline__ void mix_geometry(MB& m, int Np) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nct = Np >> 4;   // 2 or 4 (Np a multiple of 32, n <= 64)
  m.nt = wave % nct;
  m.wpt = nct >= 4 ? 1 : 4 / nct;
  m.csub = nct >= 4 ? 0 : wave / nct;
}

__device__ __forceinline__ void load_mix_slot(float (&b)[kMixKB][8], const float* Bslot, int nt, int nkb) {
  const int lane = lane_id();
#pragma unroll
  for (int kb = 0; kb < kMixKB; ++kb) {
    const int kk = kb < nkb ? kb : 0;
    const float* bp = Bslot + ((size_t)(nt * nkb + kk) * 64 + lane) * 8;
    const float4 lo = *(const float4*)bp, hi = *(const float4*)(bp + 4);
    b[kb][0] = lo.x; b[kb][1] = lo.y; b[kb][2] = lo.z; b[kb][3] = lo.w;
    b[kb][4] = hi.x; b[kb][5] = hi.y; b[kb][6] = hi.z; b[kb][7] = hi.w;
  }
}

__device__ __forceinline__ void split_mix_slot(const float (&b)[kMixKB][8], bf16x8 (&bh)[kMixKB],
                                               bf16x8 (&bl)[kMixKB]) {
#pragma unroll
  for (int kb = 0; kb < kMixKB; ++kb)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      __bf16 h, l;
      split_bf16(b[kb][j], h, l);
      bh[kb][j] = h;
      bl[kb][j] = l;
    }
}

template <int NS, bool BF3>
__device__ __forceinline__ void load_mix_b(MixB<NS, BF3>& m, const float* Bbase, int b_stride, int Kp, int Np) {
  mix_geometry(m, Np);
  const int nkb = Kp >> 5;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if constexpr (BF3) {
      float b[kMixKB][8];
      load_mix_slot(b, Bbase + (size_t)s * b_stride, m.nt, nkb);
      split_mix_slot(b, m.bh[s], m.bl[s]);
    } else {
      load_mix_slot(m.b[s], Bbase + (size_t)s * b_stride, m.nt, nkb);
    }
  }
}

// One strided component c of the tile: rows e0.., output row stride ldo components.
template <int TT>
__device__ __forceinline__ void mix_one(const float* S, int lds_ld, int c, const float (&b)[kMixKB][8], int nt,
                                        int n, int Kp, float scale, float* out, int ldo, int64_t e0, int E) {
  constexpr int RT = TT / 16;
  const int lane = lane_id();
  const int nkb = Kp >> 5;
  const int col = nt * 16 + (lane & 15);
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
        acc[rt] = mma8(af, b[kb], acc[rt]);
      }
    }
  }
  if (col < n) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = rt * 16 + 4 * (lane >> 4) + i;
        if (e0 + r < E) out[((size_t)(e0 + r) * ldo + c) * n + col] = acc[rt][i] * scale;
      }
  }
}

// The BF16 x 3 form of mix_one: the tile is staged as two BF16 planes (hi
// parts, then lo parts, row stride lds_ld elements, a multiple of 8), and the
// B fragments come pre-split.
template <int TT>
__device__ __forceinline__ void mix_one3(const __bf16* Sh, const __bf16* Sl, int lds_ld, int c,
                                         const bf16x8 (&bh)[kMixKB], const bf16x8 (&bl)[kMixKB], int nt, int n,
                                         int Kp, float scale, float* out, int ldo, int64_t e0, int E) {
  constexpr int RT = TT / 16;
  const int lane = lane_id();
  const int nkb = Kp >> 5;
  const int col = nt * 16 + (lane & 15);
  f32x4 acc[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) acc[rt] = f32x4{0, 0, 0, 0};
#pragma unroll
  for (int kb = 0; kb < kMixKB; ++kb) {
    if (kb < nkb) {
      const size_t at = ((size_t)c * TT + (lane & 15)) * lds_ld + kb * 32 + 8 * (lane >> 4);
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const bf16x8 ah = *(const bf16x8*)(Sh + at + (size_t)rt * 16 * lds_ld);
        const bf16x8 al = *(const bf16x8*)(Sl + at + (size_t)rt * 16 * lds_ld);
        acc[rt] = mma3(ah, al, bh[kb], bl[kb], acc[rt]);
      }
    }
  }
  if (col < n) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = rt * 16 + 4 * (lane >> 4) + i;
        if (e0 + r < E) out[((size_t)(e0 + r) * ldo + c) * n + col] = acc[rt][i] * scale;
      }
  }
}

// Writes value v of component c, tile row r, channel u into the staged tile:
// FP32, or (BF3) its hi and lo BF16 parts into the two planes of DIMS
// components each.
template <bool BF3, int DIMS, int TT>
__device__ __forceinline__ void stage_value(float* S, int lds_ld, int c, int r, int u, float v) {
  const size_t at = ((size_t)c * TT + r) * lds_ld + u;
  if constexpr (BF3) {
    __bf16* Sh = (__bf16*)S;
    __bf16 h, l;
    split_bf16(v, h, l);
    Sh[at] = h;
    Sh[(size_t)DIMS * TT * lds_ld + at] = l;
  } else {
    S[at] = v;
  }
}

// HOLD: m holds the fragments of slots 0..LMAX (natural-parity output).
// Otherwise each component's slot is loaded from Bbase; the unnatural l = 0
// slot (component D of a 2 D wide feature) is never kept and is skipped.
template <int LMAX, int DOUT, int TT, bool HOLD, int NS, bool BF3>
__device__ void mix_tile(const float* S, int lds_ld, const MixB<NS, BF3>& m, const float* Bbase, int b_stride, int n,
                         int Kp, float scale, float* out, int64_t e0, int E) {
  constexpr int D = (LMAX + 1) * (LMAX + 1);
  const __bf16* Sh = (const __bf16*)S;
  const __bf16* Sl = Sh + (size_t)DOUT * TT * lds_ld;
  if constexpr (HOLD) {
#pragma unroll
    for (int l = 0; l <= LMAX; ++l) {
#pragma unroll 1
      for (int c = l * l; c < (l + 1) * (l + 1); ++c) {
        if (c % m.wpt != m.csub) continue;
        if constexpr (BF3) mix_one3<TT>(Sh, Sl, lds_ld, c, m.bh[l], m.bl[l], m.nt, n, Kp, scale, out, DOUT, e0, E);
        else mix_one<TT>(S, lds_ld, c, m.b[l], m.nt, n, Kp, scale, out, DOUT, e0, E);
      }
    }
  } else {
#pragma unroll 1
    for (int c = 0; c < DOUT; ++c) {
      if (c % m.wpt != m.csub || (DOUT > D && c == D)) continue;
      float b[kMixKB][8];
      load_mix_slot(b, Bbase + (size_t)mix_slot<LMAX>(c) * b_stride, m.nt, Kp >> 5);
      if constexpr (BF3) {
        bf16x8 bh[kMixKB], bl[kMixKB];
        split_mix_slot(b, bh, bl);
        mix_one3<TT>(Sh, Sl, lds_ld, c, bh, bl, m.nt, n, Kp, scale, out, DOUT, e0, E);
      } else {
        mix_one<TT>(S, lds_ld, c, b, m.nt, n, Kp, scale, out, DOUT, e0, E);
      }
    }
  }
}

template <int DOUT, int TT>
__device__ void copy_tile(const float* S, int lds_ld, int n, float* out, int64_t e0, int E) {
  for (int p = threadIdx.x; p < TT * DOUT * n; p += 256) {
    const int r = p / (DOUT * n), rem = p - r * DOUT * n, c = rem / n, u = rem - c * n;
    if (e0 + r < E) out[((size_t)(e0 + r) * DOUT + c) * n + u] = S[((size_t)c * TT + r) * lds_ld + u];
  }
}

// The centres of an edge tile's TT edges, for the tile kernels below.  Thread
// t < TT requests centre t of the block's next tile before the current
// tile's mixing and publishes it after the mixing, so the next tile's
// gathers of centre rows read the index from LDS and wait on no other load.
template <int TT>
struct TileCentres {
  int next = 0;
  __device__ __forceinline__ void request(const TensorArgs& a, int64_t e0, int E) {
    if (threadIdx.x < TT) next = e0 + threadIdx.x < E ? a.ei[e0 + threadIdx.x] - a.centre_base : 0;
  }
  __device__ __forceinline__ void publish(int* cent) const {
    if (threadIdx.x < TT) cent[threadIdx.x] = next;
  }
};

// Whether a layer's mixing keeps every slot's fragments in registers.
template <class Pat>
constexpr bool kHoldMix = Pat::In == kNatural && Pat::Out == kNatural && Pat::Lmax <= 2;

// Tensor product (non-final layers) + channel mixing -> V^L.  Each block
// walks edge tiles blockIdx.x, blockIdx.x + gridDim.x, ... with the mixing
// fragments loaded once.
template <class Pat, int TT, bool BF3>
__global__ __launch_bounds__(256) void k_tp_mix(TensorArgs a, int lds_ld, int Kp, int Np) {
  const int E = live_edges(a);
  constexpr int LMAX = Pat::Lmax, DIM = Pat::DIM, DIN = Pat::DIN, DOUT = Pat::DOUT;
  constexpr bool HOLD = kHoldMix<Pat>;
  extern __shared__ __align__(16) float S[];   // [DOUT][TT][lds_ld] (BF3: two BF16 planes of that shape)
  const int n = a.n;
  const auto w = tp_weights<Pat>(a);   // uniform: read with scalar loads
  MixB<HOLD ? LMAX + 1 : 1, BF3> mb;
  if (a.channel_mix) {
    if constexpr (HOLD) load_mix_b(mb, (const float*)a.mixB, a.mix_stride, Kp, Np);
    else mix_geometry(mb, Np);
  }
  const int ntiles = (E + TT - 1) / TT;
  __shared__ int cent[TT];
  TileCentres<TT> tc;
  tc.request(a, (int64_t)blockIdx.x * TT, E);
  tc.publish(cent);
  __syncthreads();
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t e0 = (int64_t)tile * TT;
    // TT * Kp is a multiple of 512: two (edge, channel) items per thread per
    // step, loads of both issued before either is used
    for (int p0 = threadIdx.x; p0 < TT * Kp; p0 += 512) {
      float V[2][DIN], G[2][DIM];
      bool ok[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int p = p0 + 256 * h;
        const int r = p / Kp, u = p - r * Kp;
        const int64_t e = e0 + r;
        ok[h] = e < E && u < n;
        const int64_t ee = ok[h] ? e : 0;
        const int uu = ok[h] ? u : 0;
        load_v<LMAX, DIN>(a.v, a.eb + (size_t)ee * kEB, ee, uu, n, V[h]);
        const float* gp = a.gam + (size_t)cent[ok[h] ? r : 0] * DIM * n + uu;
#pragma unroll
        for (int b = 0; b < DIM; ++b) G[h][b] = gp[b * n];
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int p = p0 + 256 * h;
        const int r = p / Kp, u = p - r * Kp;
        float T[DOUT];
#pragma unroll
        for (int c = 0; c < DOUT; ++c) T[c] = 0.0f;
        if (ok[h]) tp_forward<Pat>(V[h], G[h], T, per_iteration(w));
#pragma unroll
        for (int c = 0; c < DOUT; ++c) stage_value<BF3, DOUT, TT>(S, lds_ld, c, r, u, T[c]);
      }
    }
    tc.request(a, e0 + (int64_t)gridDim.x * TT, E);
    __syncthreads();
    if (BF3 || a.channel_mix)   // the BF16 x 3 form is only launched with mixing on
      mix_tile<LMAX, DOUT, TT, HOLD>(S, lds_ld, mb, (const float*)a.mixB, a.mix_stride, n, Kp, a.mix_scale,
                                     a.v_out, e0, E);
    else copy_tile<DOUT, TT>(S, lds_ld, n, a.v_out, e0, E);
    tc.publish(cent);   // every read of this tile's centres was before the barrier
    __syncthreads();    // S and cent are rewritten by the next tile
  }
}

// Adjoint of channel mixing for a non-final layer L, given the next layer's
// pattern PatN.  dE/dV^L is rebuilt from layer L+1:
//   final next layer:  dE/dV[a][u] = w_a Gamma'[a][u] dE/dT'[u]
//   otherwise:         dE/dV[a][u] = sum_{b,c} W'[a][b][c] Gamma'[b][u] dE/dT'[c][u]
// plus dE/ds at a = 0 (the scalars read by layer L's latent MLP); then the
// transposed mixing gives dE/dT^L.  The launch's tpw / tpw_v hold layer
// L+1's table.
template <class PatN, int TT, bool BF3>
__global__ __launch_bounds__(256) void k_mix_adjoint(TensorArgs a, int lds_ld, int Kp, int Np) {
  const int E = live_edges(a);
  constexpr int LMAX = PatN::Lmax, DIM = PatN::DIM, DW = PatN::DIN, DN = PatN::DOUT;
  constexpr bool NEXT_FINAL = PatN::Out == kScalarOut;
  constexpr bool HOLD = NEXT_FINAL && PatN::In == kNatural && LMAX <= 2;
  static_assert(!NEXT_FINAL || DW == DIM, "the final layer reads natural-parity features");
  extern __shared__ __align__(16) float S[];
  const int n = a.n;
  const auto wn = tp_weights<PatN>(a);
  MixB<HOLD ? LMAX + 1 : 1, BF3> mb;
  if (a.channel_mix) {
    if constexpr (HOLD) load_mix_b(mb, (const float*)a.mixB, a.mix_stride, Kp, Np);
    else mix_geometry(mb, Np);
  }
  const int ntiles = (E + TT - 1) / TT;
  __shared__ int cent[TT];
  TileCentres<TT> tc;
  tc.request(a, (int64_t)blockIdx.x * TT, E);
  tc.publish(cent);
  __syncthreads();
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t e0 = (int64_t)tile * TT;
    for (int p0 = threadIdx.x; p0 < TT * Kp; p0 += 512) {
      float gam[2][DIM], gt[2][DN], gs[2];
      bool ok[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int p = p0 + 256 * h;
        const int r = p / Kp, u = p - r * Kp;
        const int64_t e = e0 + r;
        ok[h] = e < E && u < n;
        const int64_t ee = ok[h] ? e : 0;
        const int uu = ok[h] ? u : 0;
#pragma unroll
        for (int c = 0; c < DN; ++c) gt[h][c] = a.g_tnext[((size_t)ee * DN + c) * n + uu];
        gs[h] = a.g_s[(size_t)ee * n + uu];
        const float* gp = a.gam_next + (size_t)cent[ok[h] ? r : 0] * DIM * n + uu;
#pragma unroll
        for (int c = 0; c < DIM; ++c) gam[h][c] = gp[c * n];
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int p = p0 + 256 * h;
        const int r = p / Kp, u = p - r * Kp;
        if constexpr (NEXT_FINAL) {
#pragma unroll
          for (int c = 0; c < DIM; ++c) {
            // one explicit fma per element: rows of both item halves round alike
            const float gV = ok[h] ? fmaf(a.tp_wnext[c] * gam[h][c], gt[h][0], c == 0 ? gs[h] : 0.0f) : 0.0f;
            stage_value<BF3, DW, TT>(S, lds_ld, c, r, u, gV);
          }
        } else {
          float gV[DW];
#pragma unroll
          for (int c = 0; c < DW; ++c) gV[c] = 0.0f;
          if (ok[h]) {
            tp_adjoint_v<PatN>(gam[h], gt[h], gV, per_iteration(wn));
            gV[0] += gs[h];
          }
#pragma unroll
          for (int c = 0; c < DW; ++c) stage_value<BF3, DW, TT>(S, lds_ld, c, r, u, gV[c]);
        }
      }
    }
    tc.request(a, e0 + (int64_t)gridDim.x * TT, E);
    __syncthreads();
    if (BF3 || a.channel_mix)   // the BF16 x 3 form is only launched with mixing on
      mix_tile<LMAX, DW, TT, HOLD>(S, lds_ld, mb, (const float*)a.mixB, a.mix_stride, n, Kp, a.mix_scale,
                                   a.g_tout, e0, E);
    else copy_tile<DW, TT>(S, lds_ld, n, a.g_tout, e0, E);
    tc.publish(cent);   // every read of this tile's centres was before the barrier
    __syncthreads();    // S and cent are rewritten by the next tile
  }
}

// ---------------------------------------------------------------------------
// Adjoint of the tensor product and the environment sum, in two kernels.
//
// k_tp_adjoint_gamma (one wavefront per centre; lane = channel u, and with
// n < 64 the G = 64/n lane groups take interleaved edges) accumulates
//   dE/dGamma_i[b][u] = sum_{e in N(i)} sum_{a,c} W[a][b][c] V_e[a][u] dE/dT_e[c][u]
// in registers and writes it once per centre (without the factor c).  When
// V_e = a0_e[l(a)][u] Y_e[a] (first layer) the same pass, which already holds
// each edge's dE/dT_e, a0_e and Y_e, also forms the per-edge terms that need
// only the centre's Gamma_i:
//   dE/dV_e[a][u] = sum_{b,c} W[a][b][c] Gamma_i[b][u] dE/dT_e[c][u]
//   dE/da0_e[l][u] = sum_{a: l(a)=l} dE/dV_e[a][u] Y_e[a]
//   dE/dY_e[a]   += sum_u dE/dV_e[a][u] a0_e[l(a)][u],
// so that dE/dT_e is read once.  (For later layers dE/dV_e is formed by the
// previous layer's mixing adjoint.)
//
// k_tp_adjoint_edges (edge-parallel; G edges per wavefront step, each wave a
// contiguous run of edges) then produces the per-edge gradients that need
// dE/dGamma_i:
//   dE/dw_e[l][u] = c sum_{b: l(b)=l} dE/dGamma_i[b][u] Y_e[b]
//   dE/dY_e[b]   += c sum_u dE/dGamma_i[b][u] w_e[l(b)][u].
// The sums over channels use DPP lane moves within each group of n lanes, in
// a fixed order: deterministic.

// Edges per lane group whose loads are issued together: as many as fit a
// register budget of about 80 values.
template <class Pat, bool A0>
constexpr int kGammaBatch = A0 ? (4 * (Pat::Lmax + 1 + Pat::DIM + Pat::DOUT) <= 80 ? 4 : 2)
                               : (4 * (Pat::DIN + Pat::DOUT) <= 80 ? 4 : (2 * (Pat::DIN + Pat::DOUT) <= 80 ? 2 : 1));

// A0: the layer's V is the rank-1 first-layer form a0[l(a)][u] Y[a]; the pass
// then also writes dE/da0_e and its part of dE/dY_e.
template <class Pat, int G, bool A0>
__global__ __launch_bounds__(256) void k_tp_adjoint_gamma(TensorArgs a) {
  constexpr int LMAX = Pat::Lmax, DIM = Pat::DIM, DIN = Pat::DIN, DOUT = Pat::DOUT;
  constexpr int GYW = gy_width(LMAX);
  constexpr int KB = kGammaBatch<Pat, A0>;
  constexpr int n = kWave / G;
  const int lane = lane_id();
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= a.n_centres) return;
  const int u = lane & (n - 1), g = lane / n;
  // The rank-1 form runs two contractions per edge: its weights come from the
  // table in memory, reloaded (scalar loads) at each iteration, since the
  // kernel-argument copy would be hoisted whole into vector registers.
  const auto w = [&] {
    if constexpr (A0) return (ConstFloatPtr)a.tpw;
    else return tp_weights<Pat>(a);
  }();
  float gG[DIM];
#pragma unroll
  for (int b = 0; b < DIM; ++b) gG[b] = 0.0f;
  const int eb0 = a.row_ptr[c], eb1 = a.row_ptr[c + 1];
  float Gm[A0 ? DIM : 1];
  if constexpr (A0) {
    static_assert(Pat::In == kNatural, "the rank-1 form is natural");
    const float* gmp = a.gam + c * (uint32_t)(DIM * n) + u;
#pragma unroll
    for (int b = 0; b < DIM; ++b) Gm[b] = gmp[b * n];
  }
  const bool keep_gy = a.gy_accum != 0;
  for (int e0 = eb0; e0 < eb1; e0 += G * KB) {
    float V[A0 ? 1 : KB][DIN], gT[KB][DOUT];
    float Yv[A0 ? KB : 1][DIM], a0v[A0 ? KB : 1][LMAX + 1];
    float gyo[A0 ? KB : 1][DIM];   // the edge's dE/dY row so far (every lane of its group)
    bool act[KB];
    uint32_t eev[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      const int e = e0 + g + G * j;
      act[j] = e < eb1;
      const uint32_t ee = act[j] ? e : eb0;
      eev[j] = ee;
      const float* vp = a.v.p + ee * (uint32_t)a.v.ld + u;
      const float* gtp = a.g_t + ee * (uint32_t)(DOUT * n) + u;
      if constexpr (A0) {
        const float* Y = a.eb + ee * kEB;
#pragma unroll
        for (int l = 0; l <= LMAX; ++l) a0v[j][l] = vp[l * n];
#pragma unroll
        for (int k = 0; k < DIM; ++k) Yv[j][k] = Y[eb_y(k)];
        if (keep_gy) {
          const float* o = a.g_Y + ee * (uint32_t)GYW;
#pragma unroll
          for (int k = 0; k < DIM; ++k) gyo[j][k] = o[k];
        }
      } else {
#pragma unroll
        for (int k = 0; k < DIN; ++k) V[j][k] = vp[k * n];
      }
#pragma unroll
      for (int k = 0; k < DOUT; ++k) gT[j][k] = act[j] ? gtp[k * n] : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      if constexpr (A0) {
        float Vj[DIN];
#pragma unroll
        for (int k = 0; k < DIN; ++k) Vj[k] = k < DIM ? a0v[j][lof(k < DIM ? k : 0)] * Yv[j][k < DIM ? k : 0] : 0.0f;
        tp_adjoint_g<Pat>(Vj, gT[j], gG, per_iteration(w));
        float gV[DIN];
#pragma unroll
        for (int k = 0; k < DIN; ++k) gV[k] = 0.0f;
        tp_adjoint_v<Pat>(Gm, gT[j], gV, per_iteration(w));
        float ga[LMAX + 1], r[DIM];
#pragma unroll
        for (int l = 0; l <= LMAX; ++l) ga[l] = 0.0f;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
          ga[lof(k)] = fmaf(gV[k], Yv[j][k], ga[lof(k)]);
          r[k] = gV[k] * a0v[j][lof(k)];
        }
        const uint32_t ee = eev[j];
        if (act[j]) {
#pragma unroll
          for (int l = 0; l <= LMAX; ++l) a.g_a0[ee * (uint32_t)a.ld_gw + l * n + u] = ga[l];
        }
        // sums over the group's channels (DPP; the group's last lane holds them)
#pragma unroll
        for (int k = 0; k < DIM; ++k) r[k] = group_sum_dpp<n>(r[k]);
        if (act[j] && u == n - 1) {
#pragma unroll
          for (int k = 0; k < GYW; ++k) {
            const int kk = k < DIM ? k : 0;
            if (k < DIM || !keep_gy) a.g_Y[ee * (uint32_t)GYW + k] = k < DIM ? (keep_gy ? gyo[j][kk] + r[kk] : r[kk]) : 0.0f;
          }
        }
      } else {
        tp_adjoint_g<Pat>(V[j], gT[j], gG, per_iteration(w));
      }
    }
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

// KEEP: adds its terms to the dE/dY_e rows written before it (by a later
// layer, or by the first layer's gamma pass) instead of writing them.
template <class Pat, int G, bool KEEP>
__global__ __launch_bounds__(256) void k_tp_adjoint_edges(TensorArgs a) {
  const int E = live_edges(a);
  constexpr int LMAX = Pat::Lmax, DIM = Pat::DIM;
  constexpr int GYW = gy_width(LMAX);
  constexpr int n = kWave / G;
  // edges per lane group whose loads are issued together (two when the
  // earlier dE/dY rows come along: four then costs more occupancy than the
  // extra loads in flight return)
  constexpr int KB = (DIM > 9 || KEEP) ? 2 : 4;
  const int lane = lane_id();
  const int u = lane & (n - 1), g = lane / n;
  const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t w0 = (int64_t)wave * kEdgesPerWave;
  const float cn = a.c_norm;
  // centres of the wave's edges: one load per lane, read out per edge.  With
  // one edge per wave step (G = 1) the centre is wave-uniform and its
  // dE/dGamma rows stay in registers until it changes (CACHE).
  constexpr bool CACHE = G == 1;
  const int64_t el = w0 + (lane & (kEdgesPerWave - 1));
  const int ci_lane = el < E ? a.ei[el] - a.centre_base : 0;
  int cur = -1;
  float cG[CACHE ? DIM : 1];
  for (int j0 = 0; j0 < kEdgesPerWave; j0 += G * KB) {
    float gG[CACHE ? 1 : KB][DIM], Yv[KB][DIM], wv[KB][LMAX + 1];
    float gyo[KEEP ? KB : 1][DIM];   // the edge's dE/dY row so far (every lane of its group)
    bool act[KB];
    uint32_t eev[KB], civ[KB];
#pragma unroll
    for (int q = 0; q < KB; ++q) {
      const int jj = j0 + g + G * q;
      const int64_t e = w0 + jj;
      act[q] = jj < kEdgesPerWave && e < E;
      const uint32_t ee = act[q] ? (uint32_t)e : 0u;
      eev[q] = ee;
      uint32_t ci = (uint32_t)__shfl(ci_lane, jj & (kEdgesPerWave - 1), kWave);
      if constexpr (G == 1) ci = __builtin_amdgcn_readfirstlane(ci);
      civ[q] = ci;
      const float* Y = a.eb + ee * kEB;
      const float* wp = a.w_env + ee * (uint32_t)a.ld_w + u;
#pragma unroll
      for (int b = 0; b < DIM; ++b) Yv[q][b] = Y[eb_y(b)];
#pragma unroll
      for (int l = 0; l <= LMAX; ++l) wv[q][l] = wp[l * n];
      if constexpr (KEEP) {
        const float* o = a.g_Y + ee * (uint32_t)GYW;
#pragma unroll
        for (int k = 0; k < DIM; ++k) gyo[q][k] = o[k];
      }
      if constexpr (!CACHE) {
        const float* ggp = a.g_gam + ci * (uint32_t)(DIM * n) + u;
#pragma unroll
        for (int b = 0; b < DIM; ++b) gG[q][b] = ggp[b * n];
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
      if (act[q]) {
#pragma unroll
        for (int l = 0; l <= LMAX; ++l) a.g_w[ee * (uint32_t)a.ld_gw + l * n + u] = gw[l] * cn;
      }
      // sums over the group's channels (DPP; the group's last lane holds them)
#pragma unroll
      for (int k = 0; k < DIM; ++k) r[k] = group_sum_dpp<n>(r[k]);
      if (act[q] && u == n - 1) {
#pragma unroll
        for (int k = 0; k < GYW; ++k) {
          const int kk = k < DIM ? k : 0;
          if (k < DIM || !KEEP) a.g_Y[ee * (uint32_t)GYW + k] = k < DIM ? (KEEP ? gyo[KEEP ? q : 0][kk] + r[kk] : r[kk]) : 0.0f;
        }
      }
    }
  }
}

inline unsigned blocks(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// Blocks of the edge-tile mixing kernels: a few per compute unit, each
// walking many tiles with its mixing fragments in registers.
constexpr unsigned kMixBlocks = 256 * 8;

// Staged tile: FP32 rows of Kp + 4 floats, or (bf3) two BF16 planes with
// rows of Kp + 8 elements (16-byte aligned, conflict-free 16-byte reads).
void mix_dims(int n, int dim, int tt, int* lds_ld, int* Kp, int* Np, size_t* bytes, bool bf3 = false) {
  *Kp = ((n + 31) / 32) * 32;
  *Np = ((n + 31) / 32) * 32;
  *lds_ld = bf3 ? *Kp + 8 : *Kp + 4;
  *bytes = bf3 ? (size_t)2 * dim * tt * (*lds_ld) * sizeof(__bf16) : (size_t)dim * tt * (*lds_ld) * sizeof(float);
}

template <class K>
hipError_t launch_lds(K kern, unsigned grid, size_t bytes, hipStream_t s, const TensorArgs& a, int ld, int Kp,
                      int Np) {
  hipError_t st = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (st != hipSuccess) return st;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(256), bytes, s, a, ld, Kp, Np);
  return hipGetLastError();
}

// Calls fn(TpPattern<l_max, in, out>{}) for the supported patterns: natural
// input with scalar, natural or both-parity output, and both-parity input
// with natural or both-parity output, for l_max 1..3.
template <int LMAX, class Fn>
hipError_t with_pattern_l(int in, int out, Fn&& fn) {
  if (in == kNatural) {
    if (out == kScalarOut) return fn(TpPattern<LMAX, kNatural, kScalarOut>{});
    if (out == kNatural) return fn(TpPattern<LMAX, kNatural, kNatural>{});
    if (out == kBothParities) return fn(TpPattern<LMAX, kNatural, kBothParities>{});
  } else if (in == kBothParities) {
    if (out == kNatural) return fn(TpPattern<LMAX, kBothParities, kNatural>{});
    if (out == kBothParities) return fn(TpPattern<LMAX, kBothParities, kBothParities>{});
  }
  return hipErrorInvalidValue;
}

template <class Fn>
hipError_t with_pattern(int l_max, int in, int out, Fn&& fn) {
  switch (l_max) {
    case 1: return with_pattern_l<1>(in, out, fn);
    case 2: return with_pattern_l<2>(in, out, fn);
    case 3: return with_pattern_l<3>(in, out, fn);
  }
  return hipErrorInvalidValue;
}

// Whether a pattern is one of the natural-parity ones with l_max <= 2, which
// support every channel count and both tile heights; the others run with 32
// or 64 channels and 16-edge tiles.
template <class Pat>
constexpr bool kBasePattern = Pat::Lmax <= 2 && Pat::In == kNatural && Pat::Out != kBothParities;

}  // namespace

hipError_t launch_env(const TensorArgs& a, hipStream_t s) {
  if (a.n_centres <= 0) return hipSuccess;
  const dim3 grid(blocks(a.n_centres, 4));
  if (a.l_max == 1) hipLaunchKernelGGL(k_env<1>, grid, dim3(256), 0, s, a);
  else if (a.l_max == 2) hipLaunchKernelGGL(k_env<2>, grid, dim3(256), 0, s, a);
  else if (a.l_max == 3) hipLaunchKernelGGL(k_env<3>, grid, dim3(256), 0, s, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

namespace {

template <class Pat, int TT>
hipError_t launch_tp_mix_pt(const TensorArgs& a, hipStream_t s) {
  const bool bf3 = a.mix_bf3 && a.channel_mix;
  int ld, Kp, Np;
  size_t bytes;
  mix_dims(a.n, Pat::DOUT, TT, &ld, &Kp, &Np, &bytes, bf3);
  // one tile per block: the tensor-product phase's load latency is hidden by
  // many resident blocks rather than by a tile loop
  const unsigned grid = blocks(a.E, TT);
  if (bf3) return launch_lds(k_tp_mix<Pat, TT, true>, grid, bytes, s, a, ld, Kp, Np);
  return launch_lds(k_tp_mix<Pat, TT, false>, grid, bytes, s, a, ld, Kp, Np);
}

template <class PatN, int TT>
hipError_t launch_mix_adjoint_pt(const TensorArgs& a, hipStream_t s) {
  const bool bf3 = a.mix_bf3 && a.channel_mix;
  int ld, Kp, Np;
  size_t bytes;
  mix_dims(a.n, PatN::DIN, TT, &ld, &Kp, &Np, &bytes, bf3);
  const unsigned grid = std::min<unsigned>(blocks(a.E, TT), kMixBlocks);
  if (bf3) return launch_lds(k_mix_adjoint<PatN, TT, true>, grid, bytes, s, a, ld, Kp, Np);
  return launch_lds(k_mix_adjoint<PatN, TT, false>, grid, bytes, s, a, ld, Kp, Np);
}

// The rank-1 first layer's gamma pass writes dE/dY_e first (accumulating
// when the layer's arguments say so); the edge pass then always adds to it.
template <class Pat, int G>
hipError_t launch_adjoint_g(const TensorArgs& a, hipStream_t s) {
  bool a0 = false;
  if constexpr (Pat::In == kNatural) a0 = a.v.from_a0 != 0;
  if (a.n_centres > 0) {
    const dim3 grid(blocks(a.n_centres, 4));
    if constexpr (Pat::In == kNatural) {
      if (a0) hipLaunchKernelGGL((k_tp_adjoint_gamma<Pat, G, true>), grid, dim3(256), 0, s, a);
    }
    if (!a0) hipLaunchKernelGGL((k_tp_adjoint_gamma<Pat, G, false>), grid, dim3(256), 0, s, a);
  }
  if (a.E > 0) {
    const dim3 grid(blocks(a.E, 4 * kEdgesPerWave));
    if (a0 || a.gy_accum) hipLaunchKernelGGL((k_tp_adjoint_edges<Pat, G, true>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_tp_adjoint_edges<Pat, G, false>), grid, dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_tp_mix(const TensorArgs& a, bool final_layer, hipStream_t s) {
  if (final_layer) return hipErrorInvalidValue;   // the final layer is fused into the last MLP
  if (a.E <= 0) return hipSuccess;
  return with_pattern(a.l_max, a.in_kind, a.out_kind, [&](auto pat) -> hipError_t {
    using Pat = decltype(pat);
    if constexpr (Pat::Out == kScalarOut) {
      return hipErrorInvalidValue;
    } else if constexpr (kBasePattern<Pat>) {
      return a.tile == 16 ? launch_tp_mix_pt<Pat, 16>(a, s) : launch_tp_mix_pt<Pat, 32>(a, s);
    } else {
      if (a.n != 32 && a.n != 64) return hipErrorInvalidValue;
      return launch_tp_mix_pt<Pat, 16>(a, s);
    }
  });
}

hipError_t launch_mix_adjoint(const TensorArgs& a, hipStream_t s) {
  if (a.E <= 0) return hipSuccess;
  return with_pattern(a.l_max, a.next_in, a.next_out, [&](auto pat) -> hipError_t {
    using PatN = decltype(pat);
    if constexpr (PatN::Out == kScalarOut && PatN::Lmax <= 2) {
      return a.tile == 16 ? launch_mix_adjoint_pt<PatN, 16>(a, s) : launch_mix_adjoint_pt<PatN, 32>(a, s);
    } else if constexpr (PatN::In == kBothParities || PatN::Out == kScalarOut) {
      if (a.n != 32 && a.n != 64) return hipErrorInvalidValue;
      return launch_mix_adjoint_pt<PatN, 16>(a, s);
    } else {
      return hipErrorInvalidValue;   // a layer after the first reads both parities
    }
  });
}

hipError_t launch_tp_env_adjoint(const TensorArgs& a, bool final_layer, hipStream_t s) {
  const int out = final_layer ? (int)kScalarOut : a.out_kind;
  return with_pattern(a.l_max, a.in_kind, out, [&](auto pat) -> hipError_t {
    using Pat = decltype(pat);
    if constexpr (kBasePattern<Pat>) {
      switch (a.n) {
        case 64: return launch_adjoint_g<Pat, 1>(a, s);
        case 32: return launch_adjoint_g<Pat, 2>(a, s);
        case 16: return launch_adjoint_g<Pat, 4>(a, s);
        case 8: return launch_adjoint_g<Pat, 8>(a, s);
      }
    } else {
      switch (a.n) {
        case 64: return launch_adjoint_g<Pat, 1>(a, s);
        case 32: return launch_adjoint_g<Pat, 2>(a, s);
      }
    }
    return hipErrorInvalidValue;
  });
}

}  // namespace allegro
