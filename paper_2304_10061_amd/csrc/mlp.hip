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

// acc[rt][q] = A[TM x Kp] (LDS) @ B; wave w owns column tiles nt = w + 4 q.
template <int PREC, int RT, int MAXCT>
__device__ __forceinline__ void gemm_tile(f32x4 (&acc)[RT][MAXCT], const typename PT<PREC>::T* A,
                                          int lda, const GemmB& B, int wave, int lane) {
  using P = PT<PREC>;
  using T = typename P::T;
  using F = typename P::F;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int q = 0; q < MAXCT; ++q) acc[rt][q] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  const int nkb = B.Kp >> 5, nct = B.Np >> 4;
  const T* Bp = (const T*)B.p;
  const T* Arow = A + (lane & 15) * lda + 8 * (lane >> 4);
  for (int kb = 0; kb < nkb; ++kb) {
    F a[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) a[rt] = P::load(Arow + rt * 16 * lda + kb * 32);
#pragma unroll
    for (int q = 0; q < MAXCT; ++q) {
      const int nt = wave + 4 * q;
      if (nt < nct) {
        const F b = P::load(Bp + ((size_t)(nt * nkb + kb) * 64 + lane) * 8);
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) acc[rt][q] = P::mma(a[rt], b, acc[rt][q]);
      }
    }
  }
}

template <class T> __device__ __forceinline__ T to_t(float v) { return (T)v; }

// Input rows of the chain for edges e0 .. e0+TM-1, zero padded to Kp.
template <int PREC, int TM>
__device__ void build_input(const MlpArgs& a, typename PT<PREC>::T* X, int lda, int e0, int Kp) {
  using T = typename PT<PREC>::T;
  const int S = a.n_species;
  for (int idx = threadIdx.x; idx < TM * Kp; idx += 256) {
    const int r = idx / Kp, c = idx - r * Kp;
    const int e = e0 + r;
    float v = 0.0f;
    if (e < a.E) {
      if (a.kind == kTwoBody) {
        if (c < S) v = (a.species[a.ei[e]] == c) ? 1.0f : 0.0f;
        else if (c < 2 * S) v = (a.species[a.ej[e]] == c - S) ? 1.0f : 0.0f;
        else if (c < 2 * S + a.n_bessel) v = a.eb[(size_t)e * kEB + kEB_R + (c - 2 * S)];
      } else if (c < a.d) {
        v = a.x_prev[(size_t)e * a.d + c];
      } else if (c < a.d + a.n) {
        const int u = c - a.d;
        if (a.kind == kLatent) {
          v = a.s_in[(size_t)e * a.s_ld + u];
        } else {
          // final-layer scalar tensor product: T = sum_c w_c V[c][u] Gamma[c][u]
          const int dim = (a.l_max + 1) * (a.l_max + 1);
          const float* gam = a.tp_gam + (size_t)(a.ei[e] - a.centre_base) * dim * a.n + u;
          const float* vp = a.tp_v.p + (size_t)e * a.tp_v.ld + u;
          const float* Y = a.eb + (size_t)e * kEB;
          for (int cc = 0; cc < dim; ++cc) {
            const int l = cc == 0 ? 0 : (cc < 4 ? 1 : 2);
            const float vv = a.tp_v.from_a0 ? vp[l * a.n] * Y[cc] : vp[cc * a.n];
            v = fmaf(a.tp_w[cc] * vv, gam[cc * a.n], v);
          }
        }
      }
    }
    X[r * lda + c] = to_t<T>(v);
  }
}

// Writes f(acc) into an LDS tile (row-major, T) over columns [0, Np).
template <int PREC, int RT, int MAXCT, class Fn>
__device__ __forceinline__ void store_tile(const f32x4 (&acc)[RT][MAXCT], typename PT<PREC>::T* out,
                                           int ldo, int Np, int wave, int lane, Fn fn) {
  using T = typename PT<PREC>::T;
#pragma unroll
  for (int q = 0; q < MAXCT; ++q) {
    const int nt = wave + 4 * q;
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

template <int PREC, int TM, int MAXCT>
__global__ __launch_bounds__(256) void k_mlp_fwd(MlpArgs a, int lda, int ldh) {
  using P = PT<PREC>;
  using T = typename P::T;
  constexpr int RT = TM / 16;
  extern __shared__ __align__(16) char smem[];
  T* X = (T*)smem;
  T* H = X + TM * lda;
  __shared__ float red[4][TM];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int e0 = blockIdx.x * TM;

  build_input<PREC, TM>(a, X, lda, e0, a.w.fwd[0].Kp);
  __syncthreads();

  T* bufs[2] = {H, X};
  const int ldb[2] = {ldh, lda};
  const T* in = X;
  int ldin = lda;
  f32x4 acc[RT][MAXCT];
  const int nl = a.w.nl;
  for (int l = 0; l < nl; ++l) {
    gemm_tile<PREC, RT, MAXCT>(acc, in, ldin, a.w.fwd[l], wave, lane);
    if (l < nl - 1) {
      T* out = bufs[l & 1];
      store_tile<PREC, RT, MAXCT>(acc, out, ldb[l & 1], a.w.fwd[l].Np, wave, lane,
                                  [](float v, int, int) { return silu(v); });
      __syncthreads();
      in = out;
      ldin = ldb[l & 1];
    }
  }
  // epilogue: x = u h (two-body) or rs (x_prev + u h) (latent)
  const int d = a.d;
  float xr[RT][MAXCT][4];
#pragma unroll
  for (int q = 0; q < MAXCT; ++q) {
    const int col = (wave + 4 * q) * 16 + (lane & 15);
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = rt * 16 + 4 * (lane >> 4) + i;
        const int e = e0 + row;
        float v = 0.0f;
        if (e < a.E && col < d) {
          const float u = a.eb[(size_t)e * kEB + kEB_U];
          if (a.kind == kTwoBody) v = u * acc[rt][q][i];
          else v = a.res_scale * (a.x_prev[(size_t)e * d + col] + u * acc[rt][q][i]);
          if (a.x_out) a.x_out[(size_t)e * d + col] = v;
        }
        xr[rt][q][i] = v;
      }
  }
  if (a.kind == kLatentFinal) {
    // E_ij = x . we : per-lane partial over its columns, then across lanes and waves
    float part[RT][4];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float s = 0.0f;
#pragma unroll
        for (int q = 0; q < MAXCT; ++q) {
          const int col = (wave + 4 * q) * 16 + (lane & 15);
          if (col < d) s = fmaf(xr[rt][q][i], a.we[col], s);
        }
        s = group_inner_sum(s, 16);
        part[rt][i] = s;
      }
    if ((lane & 15) == 0)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) red[wave][rt * 16 + 4 * (lane >> 4) + i] = part[rt][i];
    __syncthreads();
    if ((int)threadIdx.x < TM) {
      const int e = e0 + threadIdx.x;
      if (e < a.E)
        a.eij[e] = ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
    }
    return;
  }
  if (a.head.p == nullptr) return;
  // head GEMM on x (written to the buffer the last layer did not read)
  T* xb = (in == X) ? H : X;
  const int ldx = (in == X) ? ldh : lda;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXCT; ++q) {
    const int nt = wave + 4 * q;
    if (nt * 16 >= a.w.fwd[nl - 1].Np) continue;
    const int col = nt * 16 + (lane & 15);
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int i = 0; i < 4; ++i) xb[(rt * 16 + 4 * (lane >> 4) + i) * ldx + col] = to_t<T>(xr[rt][q][i]);
  }
  __syncthreads();
  gemm_tile<PREC, RT, MAXCT>(acc, xb, ldx, a.head, wave, lane);
  const int Nh = a.head.N;
#pragma unroll
  for (int q = 0; q < MAXCT; ++q) {
    const int col = (wave + 4 * q) * 16 + (lane & 15);
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

template <int PREC, int TM, int MAXCT>
__global__ __launch_bounds__(256) void k_mlp_bwd(MlpArgs a, int lda, int ldh) {
  using P = PT<PREC>;
  using T = typename P::T;
  constexpr int RT = TM / 16;
  extern __shared__ __align__(16) char smem[];
  T* X = (T*)smem;
  T* H = X + TM * lda;
  T* Pb = H + TM * ldh;                 // nl-1 buffers of [TM][ldh]
  __shared__ float red[4][TM];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int e0 = blockIdx.x * TM;
  const int d = a.d;
  const int nl = a.w.nl;

  // 1. G = dE/dx_out
  f32x4 G[RT][MAXCT];
#pragma unroll
  for (int q = 0; q < MAXCT; ++q) {
    const int col = (wave + 4 * q) * 16 + (lane & 15);
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
    const int Kh = a.head_bwd.K, Khp = a.head_bwd.Kp;
    for (int idx = threadIdx.x; idx < TM * Khp; idx += 256) {
      const int r = idx / Khp, c = idx - r * Khp;
      const int e = e0 + r;
      float v = 0.0f;
      if (e < a.E && c < Kh) v = a.g_head[(size_t)e * Kh + c];
      X[r * lda + c] = to_t<T>(v);
    }
    __syncthreads();
    gemm_tile<PREC, RT, MAXCT>(acc, X, lda, a.head_bwd, wave, lane);
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int q = 0; q < MAXCT; ++q) G[rt][q] += acc[rt][q];
    __syncthreads();
  }

  // 2. recompute the chain, keeping pre-activations of hidden layers
  build_input<PREC, TM>(a, X, lda, e0, a.w.fwd[0].Kp);
  __syncthreads();
  const T* in = X;
  int ldin = lda;
  for (int l = 0; l < nl; ++l) {
    gemm_tile<PREC, RT, MAXCT>(acc, in, ldin, a.w.fwd[l], wave, lane);
    if (l < nl - 1) {
      const int Np = a.w.fwd[l].Np;
      store_tile<PREC, RT, MAXCT>(acc, Pb + l * TM * ldh, ldh, Np, wave, lane,
                                  [](float v, int, int) { return v; });
      if (in == H) __syncthreads();
      store_tile<PREC, RT, MAXCT>(acc, H, ldh, Np, wave, lane, [](float v, int, int) { return silu(v); });
      __syncthreads();
      in = H;
      ldin = ldh;
    }
  }
  // acc = h.  dE/du and dE/dh.
  const float rs = (a.kind == kTwoBody) ? 1.0f : a.res_scale;
  {
    float part[RT][4];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float s = 0.0f;
#pragma unroll
        for (int q = 0; q < MAXCT; ++q) s = fmaf(G[rt][q][i], acc[rt][q][i], s);
        part[rt][i] = group_inner_sum(s, 16);
      }
    if ((lane & 15) == 0)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) red[wave][rt * 16 + 4 * (lane >> 4) + i] = part[rt][i];
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
  {
    const int Np = a.w.fwd[nl - 1].Np;
#pragma unroll
    for (int q = 0; q < MAXCT; ++q) {
      const int nt = wave + 4 * q;
      if (nt * 16 >= Np) continue;
      const int col = nt * 16 + (lane & 15);
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = rt * 16 + 4 * (lane >> 4) + i;
          const int e = e0 + row;
          const float u = e < a.E ? a.eb[(size_t)e * kEB + kEB_U] : 0.0f;
          X[row * lda + col] = to_t<T>(rs * u * G[rt][q][i]);
        }
    }
  }
  __syncthreads();
  // 3. back through the layers
  for (int l = nl - 1; l >= 0; --l) {
    gemm_tile<PREC, RT, MAXCT>(acc, X, lda, a.w.bwd[l], wave, lane);
    if (l > 0) {
      const T* Pl = Pb + (l - 1) * TM * ldh;
      __syncthreads();
      store_tile<PREC, RT, MAXCT>(acc, X, lda, a.w.bwd[l].Np, wave, lane, [&](float v, int row, int col) {
        return v * silu_grad((float)Pl[row * ldh + col]);
      });
      __syncthreads();
    }
  }
  // acc = dE/dz (input of the chain)
  const int S = a.n_species;
#pragma unroll
  for (int q = 0; q < MAXCT; ++q) {
    const int col = (wave + 4 * q) * 16 + (lane & 15);
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
          a.g_xprev[(size_t)e * d + col] = rs * G[rt][q][i] + g;
        } else if (col < d + a.n) {
          a.g_s[(size_t)e * a.n + col - d] = g;
        }
      }
  }
}

template <int PREC>
void lds_dims(const MlpArgs& a, int TM, bool bwd, int* lda, int* ldh, size_t* bytes) {
  int kx = a.w.fwd[0].Kp;
  int kh = 32;
  for (int l = 0; l < a.w.nl; ++l) {
    kx = kx > a.w.fwd[l].Np ? kx : a.w.fwd[l].Np;
    if (l < a.w.nl - 1) kh = kh > a.w.fwd[l].Np ? kh : a.w.fwd[l].Np;
    if (bwd) kx = kx > a.w.bwd[l].Np ? kx : a.w.bwd[l].Np;
  }
  if (a.head.p) kx = kx > a.head.Kp ? kx : a.head.Kp;
  if (bwd && a.head_bwd.p) kx = kx > a.head_bwd.Kp ? kx : a.head_bwd.Kp;
  if (!bwd) kh = kh > kx ? kh : kx;     // forward ping-pongs any width through H
  const int pad = PREC ? 8 : 4;
  *lda = kx + pad;
  *ldh = kh + pad;
  const int nbuf_h = bwd ? a.w.nl : 1;  // H plus nl-1 pre-activation buffers
  *bytes = (size_t)TM * ((size_t)*lda + (size_t)nbuf_h * *ldh) * (PREC ? 2 : 4);
}

int max_ct(const MlpArgs& a, bool bwd) {
  int n = 0;
  for (int l = 0; l < a.w.nl; ++l) {
    n = n > a.w.fwd[l].Np ? n : a.w.fwd[l].Np;
    if (bwd) n = n > a.w.bwd[l].Np ? n : a.w.bwd[l].Np;
  }
  if (!bwd && a.head.p) n = n > a.head.Np ? n : a.head.Np;
  if (bwd && a.head_bwd.p) n = n > a.head_bwd.Np ? n : a.head_bwd.Np;
  return (n / 16 + 3) / 4;
}

constexpr size_t kLdsLimit = 160 * 1024 - 4096;

template <int PREC, int TM, int MAXCT>
hipError_t launch_one(const MlpArgs& a, bool bwd, hipStream_t s) {
  int lda, ldh;
  size_t bytes;
  lds_dims<PREC>(a, TM, bwd, &lda, &ldh, &bytes);
  const dim3 grid((a.E + TM - 1) / TM), block(256);
  if (bwd) {
    auto k = k_mlp_bwd<PREC, TM, MAXCT>;
    hipError_t st = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (st != hipSuccess) return st;
    hipLaunchKernelGGL(k, grid, block, bytes, s, a, lda, ldh);
  } else {
    auto k = k_mlp_fwd<PREC, TM, MAXCT>;
    hipError_t st = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (st != hipSuccess) return st;
    hipLaunchKernelGGL(k, grid, block, bytes, s, a, lda, ldh);
  }
  return hipGetLastError();
}

template <int PREC, int TM>
hipError_t dispatch_ct(const MlpArgs& a, bool bwd, hipStream_t s) {
  const int ct = max_ct(a, bwd);
  if (ct <= 2) return launch_one<PREC, TM, 2>(a, bwd, s);
  if (ct <= 4) return launch_one<PREC, TM, 4>(a, bwd, s);
  if (ct <= 6) return launch_one<PREC, TM, 6>(a, bwd, s);
  return hipErrorInvalidValue;
}

template <int PREC>
int pick_tm(const MlpArgs& a, bool bwd) {
  const int cands[2] = {PREC ? 64 : 32, PREC ? 32 : 16};
  for (int t : cands) {
    int lda, ldh;
    size_t bytes;
    lds_dims<PREC>(a, t, bwd, &lda, &ldh, &bytes);
    if (bytes <= kLdsLimit) return t;
  }
  return 0;
}

hipError_t launch(const MlpArgs& a, int prec, bool bwd, hipStream_t s) {
  if (a.E <= 0) return hipSuccess;
  if (prec == 1) {
    const int tm = pick_tm<1>(a, bwd);
    if (tm == 64) return dispatch_ct<1, 64>(a, bwd, s);
    if (tm == 32) return dispatch_ct<1, 32>(a, bwd, s);
  } else {
    const int tm = pick_tm<0>(a, bwd);
    if (tm == 32) return dispatch_ct<0, 32>(a, bwd, s);
    if (tm == 16) return dispatch_ct<0, 16>(a, bwd, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

size_t mlp_lds_bytes(const MlpArgs& a, int prec, bool bwd) {
  int lda, ldh;
  size_t bytes;
  const int tm = prec ? pick_tm<1>(a, bwd) : pick_tm<0>(a, bwd);
  if (tm == 0) return (size_t)-1;
  if (prec) lds_dims<1>(a, tm, bwd, &lda, &ldh, &bytes);
  else lds_dims<0>(a, tm, bwd, &lda, &ldh, &bytes);
  if (max_ct(a, bwd) > 6) return (size_t)-1;
  return bytes;
}

hipError_t launch_mlp_fwd(const MlpArgs& a, int prec, hipStream_t s) { return launch(a, prec, false, s); }
hipError_t launch_mlp_bwd(const MlpArgs& a, int prec, hipStream_t s) { return launch(a, prec, true, s); }

}  // namespace allegro
