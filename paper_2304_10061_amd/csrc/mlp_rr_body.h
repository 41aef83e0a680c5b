// mlp_rr_body.h - kernels of mlp_rr.h, included once per edges-per-wave
// setting inside a namespace that defines kNE (32-edge N blocks per wave),
// kOcc (waves per SIMD the kernels are compiled for), kWaves (waves per block)
// and kPD (weight K steps requested ahead of their use).
constexpr int kEdgesPerWave = 32 * kNE;

__device__ __forceinline__ bf16x8 ldfrag(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
__device__ __forceinline__ f32x16 mma(const bf16x8& a, const bf16x8& b, const f32x16& c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x16 zero16() {
  f32x16 z;
#pragma unroll
  for (int i = 0; i < 16; ++i) z[i] = 0.0f;
  return z;
}

// Compile-time loop: f(std::integral_constant<int, i>) for i = I .. N-1, so
// that every register-array index below is a constant expression.
template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}
template <int V> using ic = std::integral_constant<int, V>;

// Prefetch distance (K steps) of a GEMM with KS steps per pass: a divisor of
// KS, so that every K step of every pass uses the same register slot.
constexpr int pd_for(int ks) { return ks % kPD == 0 ? kPD : (ks % 2 == 0 ? 2 : 1); }

// GEMM of one wave: for every pass p (rr_nbp(MB) output blocks each) the
// accumulators acc[b][nb] = init + sum_ks W(p, ks, b) x in[nb][ks].  pre(p, acc)
// sets the initial accumulators at the start of pass p (and issues loads its
// epilogue needs), epi(p, acc) consumes them at its end.  The K steps of a
// pass are unrolled (the B operand is a register array); the passes are a
// loop, so the code stays small.  Weight fragments are requested pd_for(KS)
// steps ahead, across pass boundaries.  SPLIT: each weight is a pair of BF16
// numbers (hi, lo fragments adjacent), two MFMAs.
template <int KS, int MB, bool SPLIT, class Pre, class Epi>
__device__ __forceinline__ void gemm(const bf16x8 (&in)[kNE][KS], const void* W, Pre pre, Epi epi) {
  constexpr int NBP = rr_nbp(MB);
  constexpr int NP = MB / NBP;
  constexpr int PD = pd_for(KS);
  constexpr uint32_t S = SPLIT ? 2u : 1u;
  const __amdgpu_buffer_rsrc_t r = mlpk::ro_rsrc(W, (uint32_t)(NP * KS * NBP) * S * 1024u);
  const uint32_t voff = (threadIdx.x & 63) * 16u;
  bf16x8 hi[PD][NBP], lo[PD][SPLIT ? NBP : 1];
  auto issue = [&](auto slotc, uint32_t st) {
    constexpr int slot = decltype(slotc)::value;
#pragma unroll
    for (int b = 0; b < NBP; ++b) {
      const uint32_t f = (st * NBP + b) * S;
      hi[slot][b] = ldfrag(r, voff, f * 1024u);
      if constexpr (SPLIT) lo[slot][b] = ldfrag(r, voff, (f + 1) * 1024u);
    }
  };
  static_for<0, PD>([&](auto j) { issue(j, (uint32_t)decltype(j)::value); });
#pragma unroll 1
  for (int p = 0; p < NP; ++p) {
    f32x16 acc[NBP][kNE];
    pre(p, acc);
    const uint32_t st0 = (uint32_t)p * KS;
    const uint32_t nx0 = (uint32_t)(p + 1 < NP ? p + 1 : p) * KS;   // next pass (or this one again)
    static_for<0, KS>([&](auto kc) {
      constexpr int ks = decltype(kc)::value;
      bf16x8 h[NBP], l[SPLIT ? NBP : 1];
#pragma unroll
      for (int b = 0; b < NBP; ++b) {
        h[b] = hi[ks % PD][b];
        if constexpr (SPLIT) l[b] = lo[ks % PD][b];
      }
      issue(ic<ks % PD>{}, ks + PD < KS ? st0 + ks + PD : nx0 + (ks + PD - KS));
#pragma unroll
      for (int b = 0; b < NBP; ++b)
#pragma unroll
        for (int nb = 0; nb < kNE; ++nb) acc[b][nb] = mma(h[b], in[nb][ks], acc[b][nb]);
      if constexpr (SPLIT)
#pragma unroll
        for (int b = 0; b < NBP; ++b)
#pragma unroll
          for (int nb = 0; nb < kNE; ++nb) acc[b][nb] = mma(l[b], in[nb][ks], acc[b][nb]);
      __builtin_amdgcn_sched_barrier(0);
    });
    epi(p, acc);
  }
}

// Pass prologue that only clears the accumulators.
struct Zero {
  template <int NBP>
  __device__ __forceinline__ void operator()(int, f32x16 (&acc)[NBP][kNE]) const {
#pragma unroll
    for (int b = 0; b < NBP; ++b)
#pragma unroll
      for (int nb = 0; nb < kNE; ++nb) acc[b][nb] = zero16();
  }
};

// Slots 8 h .. 8 h + 7 of an accumulator block, through f, as a B operand.
template <class F>
__device__ __forceinline__ bf16x8 bform(const f32x16& a, int h, F f) {
  bf16x8 r;
#pragma unroll
  for (int j = 0; j < 8; ++j) r[j] = (__bf16)f(a[8 * h + j]);
  return r;
}
struct Ident {
  __device__ float operator()(float v) const { return v; }
};
struct Silu {
  __device__ float operator()(float v) const { return silu(v); }
};

// Accumulator block `mb` of a row-major FP32 array (row stride ld, column
// offset c0): features c0 + 32 mb + 8 q + 4 g + (0..3) are slots 4 q .. 4 q + 3.
// Stores of the kernel's outputs.  The forward kernels store non-temporally:
// their outputs (rows for later kernels, the activation store for the
// backward pass) would otherwise displace the weight fragments that every
// wave streams from L2.  The backward kernels' outputs are read by the very
// next kernels and keep ordinary stores.
__device__ __forceinline__ void out_store4(float* p, float4 v) {
  typedef float v4 __attribute__((ext_vector_type(4)));
  const v4 w = {v.x, v.y, v.z, v.w};
  if constexpr (kNonTemporalOut) __builtin_nontemporal_store(w, (v4*)p);
  else *(v4*)p = w;
}
__device__ __forceinline__ void out_store8(bf16x8* p, const bf16x8& v) {
  if constexpr (kNonTemporalOut) __builtin_nontemporal_store(v, p);
  else *p = v;
}

__device__ __forceinline__ f32x16 load_c(const float* p, uint32_t ld, int c0, int mb, int e, int g) {
  const float* q0 = p + (uint32_t)e * ld + (uint32_t)(c0 + 32 * mb + 4 * g);
  f32x16 a;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float4 v = *(const float4*)(q0 + 8 * q);
    a[4 * q] = v.x; a[4 * q + 1] = v.y; a[4 * q + 2] = v.z; a[4 * q + 3] = v.w;
  }
  return a;
}
__device__ __forceinline__ void store_c(float* p, uint32_t ld, int c0, int mb, int e, int g, const f32x16& a) {
  float* q0 = p + (uint32_t)e * ld + (uint32_t)(c0 + 32 * mb + 4 * g);
#pragma unroll
  for (int q = 0; q < 4; ++q) out_store4(q0 + 8 * q, make_float4(a[4 * q], a[4 * q + 1], a[4 * q + 2], a[4 * q + 3]));
}

// K steps [k0, k0 + KN) of the B operand from row-major FP32 rows: step k0 + k
// holds features c0 + 16 k + 4 g + (0..3) and c0 + 16 k + 8 + 4 g + (0..3).
// With dv set, dot[nb] also accumulates the FP32 row . dv over the lane's
// features (dv indexed like the row, from column c0).
template <int KS, int KN>
__device__ __forceinline__ void load_bform(bf16x8 (&dst)[kNE][KS], int k0, const float* src, uint32_t ld, int c0,
                                           const int (&ec)[kNE], int g, const float* dv = nullptr,
                                           float* dot = nullptr) {
  // batches of four K steps (eight 16-byte loads per lane and N block), each
  // converted before the next batch is requested
  static_for<0, (KN + 3) / 4>([&](auto bc) {
    constexpr int kb = 4 * decltype(bc)::value;
#pragma unroll
    for (int k = kb; k < (kb + 4 < KN ? kb + 4 : KN); ++k)
#pragma unroll
      for (int nb = 0; nb < kNE; ++nb) {
        const uint32_t col = (uint32_t)(c0 + 16 * k + 4 * g);
        const float* p = src + (uint32_t)ec[nb] * ld + col;
        const float4 v0 = *(const float4*)p, v1 = *(const float4*)(p + 8);
        if (dv) {
          const float4 w0 = *(const float4*)(dv + col - c0), w1 = *(const float4*)(dv + col - c0 + 8);
          float s = dot[nb];
          s = fmaf(v0.x, w0.x, s); s = fmaf(v0.y, w0.y, s); s = fmaf(v0.z, w0.z, s); s = fmaf(v0.w, w0.w, s);
          s = fmaf(v1.x, w1.x, s); s = fmaf(v1.y, w1.y, s); s = fmaf(v1.z, w1.z, s); s = fmaf(v1.w, w1.w, s);
          dot[nb] = s;
        }
        bf16x8 r;
        r[0] = (__bf16)v0.x; r[1] = (__bf16)v0.y; r[2] = (__bf16)v0.z; r[3] = (__bf16)v0.w;
        r[4] = (__bf16)v1.x; r[5] = (__bf16)v1.y; r[6] = (__bf16)v1.z; r[7] = (__bf16)v1.w;
        dst[nb][k0 + k] = r;
      }
    __builtin_amdgcn_sched_barrier(0);
  });
}

// Activation slot l (of NL per wave tile), block mb, N block nb of wave tile
// t: the 16 accumulator values of the block in BF16, as two halves of
// 64 lanes x 16 bytes (z[0] and z[kZHalf]), so that each half is one fully
// coalesced 1 KB access of the wave.  Slots 0 .. NL-2 hold the hidden
// pre-activations; slot NL-1 the last layer's output h before the envelope
// factor (two-body and latent chains).
constexpr int kZHalf = 64;
template <int NL, int MBD>
__device__ __forceinline__ bf16x8* zslot(void* base, int t, int l, int mb, int nb, int lane) {
  const size_t i = (((size_t)t * NL + l) * MBD + mb) * kNE + nb;
  return (bf16x8*)base + i * 2 * kZHalf + lane;
}

// Per-wave LDS area holding one layer's output as the next layer's B operand:
// [K step][N block][64 lanes] x 16 bytes (KS steps).  Each wave writes and
// reads only its own area, so no barrier is needed.
template <int KS>
__device__ __forceinline__ bf16x8* lds_area() {
  extern __shared__ __align__(16) char smem[];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  return (bf16x8*)smem + (size_t)wave * KS * kNE * 64;
}
// Per-wave 4 KB staging area after the B-operand areas of the block, for
// storing one 32 x 32 FP32 accumulator block as whole row segments.
template <int KS>
__device__ __forceinline__ float* stage_area() {
  extern __shared__ __align__(16) char smem[];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  return (float*)(smem + (size_t)kWaves * KS * kNE * 64 * 16 + (size_t)wave * 4096);
}

// Accumulator block `mb` of N block nb (edges e_nb .. e_nb + 31, those below E
// stored) into row-major FP32 rows (row stride ld, column offset c0),
// transposed through the wave's staging area so that each store instruction
// writes eight whole 128-byte row segments.  Chunks of 4 features are
// XOR-swizzled by row in the staging area.
__device__ __forceinline__ void store_c_rows(float* p, uint32_t ld, int c0, int mb, int e_nb, int E, int lane,
                                             const f32x16& a, float* st) {
  const int g = lane >> 5, col = lane & 31;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    *(float4*)(st + col * 32 + (((2 * q + g) ^ (col & 7)) * 4)) =
        make_float4(a[4 * q], a[4 * q + 1], a[4 * q + 2], a[4 * q + 3]);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int ch = lane & 7;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int row = 8 * k + (lane >> 3);
    const float4 v = *(const float4*)(st + row * 32 + ((ch ^ (row & 7)) * 4));
    const int e = e_nb + row;
    if (e < E) out_store4(p + (uint32_t)e * ld + (uint32_t)(c0 + 32 * mb + 4 * ch), v);
  }
  // the next block overwrites the staging area
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void stash(bf16x8* area, int k, int nb, int lane, const bf16x8& v) {
  area[(k * kNE + nb) * 64 + lane] = v;
}
template <int KS>
__device__ __forceinline__ void unstash(const bf16x8* area, bf16x8 (&in)[kNE][KS], int lane) {
#pragma unroll
  for (int k = 0; k < KS; ++k)
#pragma unroll
    for (int nb = 0; nb < kNE; ++nb) in[nb][k] = area[(k * kNE + nb) * 64 + lane];
}

// Per-lane edges of the wave's tile: clamped index and validity.
struct Rows {
  int ec[kNE];
  bool ok[kNE];
};
__device__ __forceinline__ Rows rows_of(int e0, int E, int lane) {
  Rows r;
#pragma unroll
  for (int nb = 0; nb < kNE; ++nb) {
    const int e = e0 + 32 * nb + (lane & 31);
    r.ok[nb] = e < E;
    r.ec[nb] = e < E ? e : E - 1;
  }
  return r;
}

// Chain input (K steps KIN): two-body [onehot(Z_i), onehot(Z_j), R] from the
// edge record; latent [x_prev, s_in]; final [x_prev, scalar tensor product]
// (computed from V and Gamma, and stored to tp_out when set), or the stored
// scalars from s_in (backward).
// Final-layer scalar tensor product of edge e for channels u0 .. u0+3 and
// u0+8 .. u0+11: T[u] = sum_c w_c V[c][u] Gamma[c][u] over the DIM
// components (V stored, or the rank-1 first-layer form a0[l(c)][u] Y_c), in
// batches of three components.
template <int DIM>
__device__ __forceinline__ void final_scalars(const MlpArgs& a, int e, int centre, int u0, float4 (&t)[2]) {
  const uint32_t gb = (uint32_t)(centre - a.centre_base) * DIM * a.n + u0;
  const uint32_t vb = (uint32_t)e * a.tp_v.ld + u0;
  t[0] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  t[1] = t[0];
  static_for<0, (DIM + 2) / 3>([&](auto bc) {
    constexpr int c0 = 3 * decltype(bc)::value;
    constexpr int NC = c0 + 3 <= DIM ? 3 : DIM - c0;
    float4 gv[NC][2], vv[NC][2];
    float w[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const int c = c0 + k;
      const int l = c == 0 ? 0 : (c < 4 ? 1 : (c < 9 ? 2 : 3));
      const uint32_t vo = vb + (a.tp_v.from_a0 ? l : c) * a.n;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        gv[k][h] = *(const float4*)(a.tp_gam + gb + c * a.n + 8 * h);
        vv[k][h] = *(const float4*)(a.tp_v.p + vo + 8 * h);
      }
      w[k] = a.tp_w[c] * (a.tp_v.from_a0 ? a.eb[(uint32_t)e * kEB + eb_y(c)] : 1.0f);
    }
#pragma unroll
    for (int k = 0; k < NC; ++k)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        t[h].x = fmaf(w[k] * vv[k][h].x, gv[k][h].x, t[h].x);
        t[h].y = fmaf(w[k] * vv[k][h].y, gv[k][h].y, t[h].y);
        t[h].z = fmaf(w[k] * vv[k][h].z, gv[k][h].z, t[h].z);
        t[h].w = fmaf(w[k] * vv[k][h].w, gv[k][h].w, t[h].w);
      }
    __builtin_amdgcn_sched_barrier(0);
  });
}


// Chain input of the two-body and latent kinds (K steps KIN): two-body
// [onehot(Z_i), onehot(Z_j), R] from the edge record; latent [x_prev, s_in].
template <int KIND, int D, int NT, int KIN>
__device__ __forceinline__ void chain_input(const MlpArgs& a, bf16x8 (&in)[kNE][KIN], const Rows& R, int g) {
  if constexpr (KIND == kTwoBody) {
    const int S = a.n_species, nb_ = a.n_bessel;
#pragma unroll
    for (int nb = 0; nb < kNE; ++nb) {
      const float* rec = a.eb + (uint32_t)R.ec[nb] * kEB;
      const int zi = (int)rec[kEB_ZI], zj = (int)rec[kEB_ZJ];
#pragma unroll
      for (int k = 0; k < KIN; ++k) {
        bf16x8 r;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int f = 16 * k + (j < 4 ? 4 * g + j : 8 + 4 * g + (j - 4));
          const int rc = f - 2 * S;
          const float rv = rec[kEB_R + (rc >= 0 && rc < nb_ ? rc : 0)];
          const float v = f < S ? (zi == f ? 1.0f : 0.0f)
                                : f < 2 * S ? (zj == f - S ? 1.0f : 0.0f) : (rc < nb_ ? rv : 0.0f);
          r[j] = (__bf16)v;
        }
        in[nb][k] = r;
      }
    }
  } else {
    load_bform<KIN, D / 16>(in, 0, a.x_prev, (uint32_t)D, 0, R.ec, g);
    load_bform<KIN, NT / 16>(in, D / 16, a.s_in, (uint32_t)a.s_ld, 0, R.ec, g);
  }
}

// Final-layer input [x_prev, T] (T computed from V and Gamma and stored to
// tp_out when set, or read back from s_in when `stored`); dot[nb] receives the
// lane's part of x_prev . w_e in FP32.
template <int D, int NT, int DIM, int KIN>
__device__ __forceinline__ void final_input(const MlpArgs& a, bf16x8 (&in)[kNE][KIN], const Rows& R, int g,
                                            bool stored, float (&dot)[kNE]) {
  load_bform<KIN, D / 16>(in, 0, a.x_prev, (uint32_t)D, 0, R.ec, g, a.we, dot);
  if (stored) {
    load_bform<KIN, NT / 16>(in, D / 16, a.s_in, (uint32_t)a.s_ld, 0, R.ec, g);
    return;
  }
#pragma unroll
  for (int nb = 0; nb < kNE; ++nb) {
    const int e = R.ec[nb];
    const int centre = a.ei[e];
#pragma unroll
    for (int k = 0; k < NT / 16; ++k) {
      float4 t[2];
      final_scalars<DIM>(a, e, centre, 16 * k + 4 * g, t);
      if (a.tp_out && R.ok[nb]) {
        float* o = a.tp_out + (uint32_t)e * NT + 16 * k + 4 * g;
        *(float4*)o = t[0];
        *(float4*)(o + 8) = t[1];
      }
      bf16x8 r;
      r[0] = (__bf16)t[0].x; r[1] = (__bf16)t[0].y; r[2] = (__bf16)t[0].z; r[3] = (__bf16)t[0].w;
      r[4] = (__bf16)t[1].x; r[5] = (__bf16)t[1].y; r[6] = (__bf16)t[1].z; r[7] = (__bf16)t[1].w;
      in[nb][D / 16 + k] = r;
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

template <int KIND, int D, int NT>
constexpr int kin_steps() { return KIND == kTwoBody ? 1 : (D + NT) / 16; }

// Epilogue that writes f(acc) as the next layer's B operand into the wave's
// LDS area (and, with a scratch array, the pre-activations there too).
template <class F, int NL, int MBD>
struct ToArea {
  bf16x8* area;
  int lane;
  void* scratch = nullptr;   // pre-activations of hidden layer l (backward recomputation)
  int tile = 0, l = 0;
  template <int NBP>
  __device__ __forceinline__ void operator()(int p, f32x16 (&acc)[NBP][kNE]) const {
#pragma unroll
    for (int b = 0; b < NBP; ++b)
#pragma unroll
      for (int nb = 0; nb < kNE; ++nb) {
        const int mb = p * NBP + b;
        if (scratch) {
          bf16x8* z = zslot<NL, MBD>(scratch, tile, l, mb, nb, lane);
          out_store8(&z[0], bform(acc[b][nb], 0, Ident()));
          out_store8(&z[kZHalf], bform(acc[b][nb], 1, Ident()));
        }
        stash(area, 2 * mb, nb, lane, bform(acc[b][nb], 0, F()));
        stash(area, 2 * mb + 1, nb, lane, bform(acc[b][nb], 1, F()));
      }
  }
};

// Hidden layers 0 .. NH-1 of a chain (SiLU), input x0 in registers; the last
// hidden activation is left in the wave's LDS area.  With `scratch`, the
// pre-activations of hidden layer l go to scratch slot l.
template <int D, int NL, int KIN, int NH, bool SF, bool SR>
__device__ __forceinline__ void hidden(const MlpArgs& a, const bf16x8 (&x0)[kNE][KIN], bf16x8* area, int lane,
                                       void* scratch, int tile) {
  constexpr int KD = D / 16, MBD = D / 32;
  if constexpr (NH >= 1)
    gemm<KIN, MBD, SF>(x0, a.rr.fwd[0], Zero(), ToArea<Silu, NL, MBD>{area, lane, scratch, tile, 0});
  if constexpr (NH >= 2) {
    bf16x8 a1[kNE][KD];
    unstash<KD>(area, a1, lane);
    gemm<KD, MBD, SR>(a1, a.rr.fwd[1], Zero(), ToArea<Silu, NL, MBD>{area, lane, scratch, tile, 1});
  }
}

// Forward chain of the two-body and latent kinds.  SF / SR: weight pairs in
// the first layer / in the other layers and the head.
template <int KIND, int D, int NT, int HN, int NL, bool SF, bool SR>
__global__ __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(kOcc, kOcc)))
void k_rr_fwd(MlpArgs a) {
  constexpr int KD = D / 16, MBD = D / 32, NBP = rr_nbp(MBD);
  constexpr int KIN = kin_steps<KIND, D, NT>();
  const int E = live_edges(a);
  const int lane = threadIdx.x & 63, g = lane >> 5;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tile = blockIdx.x * kWaves + wave;
  const int e0 = tile * kEdgesPerWave;
  if (e0 >= E) return;
  const Rows R = rows_of(e0, E, lane);
  float u[kNE];
#pragma unroll
  for (int nb = 0; nb < kNE; ++nb) u[nb] = R.ok[nb] ? a.eb[(uint32_t)R.ec[nb] * kEB + kEB_U] : 0.0f;
  float* st = stage_area<KD>();
  bf16x8* area = lds_area<KD>();
  {
    bf16x8 x0[kNE][KIN];
    chain_input<KIND, D, NT, KIN>(a, x0, R, g);
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (NL == 1) {
      // no hidden layer: the input is the last layer's operand
      static_assert(NL > 1, "register-resident chains have a hidden layer");
    }
    // with act_store, the hidden pre-activations are kept for the backward pass
    hidden<D, NL, KIN, NL - 1, SF, SR>(a, x0, area, lane, a.act_store, tile);
  }
  // last layer: x = u h (two-body) or rs (x_prev + u h) -> x_out rows and the
  // head's B operand
  {
    bf16x8 ah[kNE][KD];
    unstash<KD>(area, ah, lane);
    f32x16 xp[NBP][kNE];
    gemm<KD, MBD, SR>(
        ah, a.rr.fwd[NL - 1],
        [&](int p, f32x16 (&acc)[NBP][kNE]) {
          Zero()(p, acc);
          if constexpr (KIND != kTwoBody)
#pragma unroll
            for (int b = 0; b < NBP; ++b)
#pragma unroll
              for (int nb = 0; nb < kNE; ++nb) xp[b][nb] = load_c(a.x_prev, (uint32_t)D, 0, p * NBP + b, R.ec[nb], g);
        },
        [&](int p, f32x16 (&acc)[NBP][kNE]) {
#pragma unroll
          for (int b = 0; b < NBP; ++b)
#pragma unroll
            for (int nb = 0; nb < kNE; ++nb) {
              f32x16 x;
#pragma unroll
              for (int i = 0; i < 16; ++i) {
                const float h = u[nb] * acc[b][nb][i];
                x[i] = KIND == kTwoBody ? h : a.res_scale * (xp[b][nb][i] + h);
              }
              const int mb = p * NBP + b;
              if (a.act_store) {   // h, for dE/du in the backward pass
                bf16x8* z = zslot<NL, MBD>(a.act_store, tile, NL - 1, mb, nb, lane);
                out_store8(&z[0], bform(acc[b][nb], 0, Ident()));
                out_store8(&z[kZHalf], bform(acc[b][nb], 1, Ident()));
              }
              if (a.x_out) store_c_rows(a.x_out, (uint32_t)D, 0, mb, e0 + 32 * nb, E, lane, x, st);
              stash(area, 2 * mb, nb, lane, bform(x, 0, Ident()));
              stash(area, 2 * mb + 1, nb, lane, bform(x, 1, Ident()));
            }
        });
  }
  if (a.head_out == nullptr) return;
  constexpr int HB = rr_nbp(HN / 32);
  bf16x8 xb[kNE][KD];
  unstash<KD>(area, xb, lane);
  gemm<KD, HN / 32, SR>(xb, a.rr.head, Zero(), [&](int p, f32x16 (&acc)[HB][kNE]) {
#pragma unroll
    for (int b = 0; b < HB; ++b)
#pragma unroll
      for (int nb = 0; nb < kNE; ++nb)
        store_c_rows(a.head_out, (uint32_t)HN, 0, p * HB + b, e0 + 32 * nb, E, lane, acc[b][nb], st);
  });
}

// Final layer, forward (NL >= 2): hidden layers, the last one reduced to
// a . v, and E_ij = rs (x_prev . w_e + u a . v).
template <int D, int NT, int DIM, int NL, bool SF, bool SR>
__global__ __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(kOcc, kOcc)))
void k_rr_fwd_final(MlpArgs a) {
  static_assert(NL >= 2, "folded final layer needs a hidden layer");
  constexpr int KD = D / 16, MBD = D / 32, NBP = rr_nbp(MBD);
  constexpr int KIN = (D + NT) / 16;
  const int E = live_edges(a);
  const int lane = threadIdx.x & 63, g = lane >> 5;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tile = blockIdx.x * kWaves + wave;
  const int e0 = tile * kEdgesPerWave;
  if (e0 >= E) return;
  const Rows R = rows_of(e0, E, lane);
  float xw[kNE], av[kNE];
#pragma unroll
  for (int nb = 0; nb < kNE; ++nb) { xw[nb] = 0.0f; av[nb] = 0.0f; }
  bf16x8* area = lds_area<KD>();
  f32x16 vb[NBP];
  auto pre_dot = [&](int p, f32x16 (&acc)[NBP][kNE]) {
    Zero()(p, acc);
#pragma unroll
    for (int b = 0; b < NBP; ++b) vb[b] = load_c(a.fold_v, 0u, 0, p * NBP + b, 0, g);
  };
  auto epi_dot = [&](int p, f32x16 (&acc)[NBP][kNE]) {
#pragma unroll
    for (int b = 0; b < NBP; ++b)
#pragma unroll
      for (int nb = 0; nb < kNE; ++nb) {
#pragma unroll
        for (int i = 0; i < 16; ++i) av[nb] = fmaf(silu(acc[b][nb][i]), vb[b][i], av[nb]);
        if (a.act_store) {   // the last hidden layer's pre-activations
          bf16x8* z = zslot<NL, MBD>(a.act_store, tile, NL - 2, p * NBP + b, nb, lane);
          out_store8(&z[0], bform(acc[b][nb], 0, Ident()));
          out_store8(&z[kZHalf], bform(acc[b][nb], 1, Ident()));
        }
      }
  };
  {
    bf16x8 x0[kNE][KIN];
    final_input<D, NT, DIM, KIN>(a, x0, R, g, false, xw);
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (NL == 2) gemm<KIN, MBD, SF>(x0, a.rr.fwd[0], pre_dot, epi_dot);
    else hidden<D, NL, KIN, NL - 2, SF, SR>(a, x0, area, lane, a.act_store, tile);
  }
  if constexpr (NL > 2) {
    bf16x8 ah[kNE][KD];
    unstash<KD>(area, ah, lane);
    gemm<KD, MBD, SR>(ah, a.rr.fwd[NL - 2], pre_dot, epi_dot);
  }
#pragma unroll
  for (int nb = 0; nb < kNE; ++nb) {
    const float xs = xw[nb] + __shfl_xor(xw[nb], 32, 64);
    const float as = av[nb] + __shfl_xor(av[nb], 32, 64);
    if (g == 0 && R.ok[nb]) {
      const float u = a.eb[(uint32_t)R.ec[nb] * kEB + kEB_U];
      a.eij[R.ec[nb]] = a.res_scale * (xs + u * as);
      if (a.act_store) a.av_store[R.ec[nb]] = as;
    }
  }
}

// One hidden layer of the backward pass: LDS area <- (in @ W^T) silu'(z_l),
// with the pre-activations z_l read back from the scratch array.
template <int D, int NL, bool SPLIT>
__device__ __forceinline__ void back_layer(void* scratch, int tile, int lane, int l, const bf16x8 (&in)[kNE][D / 16],
                                           const void* W, bf16x8* area) {
  constexpr int MBD = D / 32, NBP = rr_nbp(MBD);
  // the pass's pre-activations are requested before its MFMAs and turned
  // into silu'(z) after them
  bf16x8 zr[NBP][kNE][2];
  gemm<D / 16, MBD, SPLIT>(
      in, W,
      [&](int p, f32x16 (&acc)[NBP][kNE]) {
        Zero()(p, acc);
#pragma unroll
        for (int b = 0; b < NBP; ++b)
#pragma unroll
          for (int nb = 0; nb < kNE; ++nb) {
            const bf16x8* z = zslot<NL, MBD>(scratch, tile, l, p * NBP + b, nb, lane);
            zr[b][nb][0] = z[0];
            zr[b][nb][1] = z[kZHalf];
          }
      },
      [&](int p, f32x16 (&acc)[NBP][kNE]) {
#pragma unroll
        for (int b = 0; b < NBP; ++b)
#pragma unroll
          for (int nb = 0; nb < kNE; ++nb) {
            f32x16 t;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              t[j] = acc[b][nb][j] * silu_grad((float)zr[b][nb][0][j]);
              t[8 + j] = acc[b][nb][8 + j] * silu_grad((float)zr[b][nb][1][j]);
            }
            const int mb = p * NBP + b;
            stash(area, 2 * mb, nb, lane, bform(t, 0, Ident()));
            stash(area, 2 * mb + 1, nb, lane, bform(t, 1, Ident()));
          }
      });
}

// Head gradient in K chunks of at most 12 steps (192 features): chunk c of the
// packed head transpose starts 12 c MB (1 + SPLIT) fragments in.
constexpr int kHeadChunk = 12;

// Last GEMM of the backward pass, dE/d(input), with its outputs: two-body
// g_R; latent and final g_xprev = rs G + dE/dx_prev (rs G preloaded into the
// accumulators) and g_s.
template <int KIND, int D, int NT, int KIN, bool SPLIT, class LoadG>
__device__ __forceinline__ void input_grad(const MlpArgs& a, const bf16x8 (&dz)[kNE][D / 16], const Rows& R, int g,
                                           float rs, LoadG load_G) {
  constexpr int MBD = D / 32;
  constexpr int MBIN = (KIN * 16 + 31) / 32;
  constexpr int NBI = rr_nbp(MBIN);
  gemm<D / 16, MBIN, SPLIT>(
      dz, a.rr.bwd[0],
      [&](int p, f32x16 (&acc)[NBI][kNE]) {
#pragma unroll
        for (int b = 0; b < NBI; ++b)
#pragma unroll
          for (int nb = 0; nb < kNE; ++nb) {
            const int mb = p * NBI + b;
            acc[b][nb] = zero16();
            if constexpr (KIND != kTwoBody) {
              if (mb < MBD) {
                const f32x16 G = load_G(mb, nb);
#pragma unroll
                for (int i = 0; i < 16; ++i) acc[b][nb][i] = rs * G[i];
              }
            }
          }
      },
      [&](int p, f32x16 (&acc)[NBI][kNE]) {
#pragma unroll
        for (int b = 0; b < NBI; ++b)
#pragma unroll
          for (int nb = 0; nb < kNE; ++nb) {
            if (!R.ok[nb]) continue;
            const int mb = p * NBI + b, e = R.ec[nb];
            if constexpr (KIND == kTwoBody) {
              const int S = a.n_species;
#pragma unroll
              for (int i = 0; i < 16; ++i) {
                const int f = 32 * mb + 8 * (i >> 2) + 4 * g + (i & 3);
                if (f >= 2 * S && f < 2 * S + a.n_bessel) a.g_R[(uint32_t)e * a.n_bessel + f - 2 * S] = acc[b][nb][i];
              }
            } else if (mb < MBD) {
              store_c(a.g_xprev, (uint32_t)D, 0, mb, e, g, acc[b][nb]);
            } else {
              store_c(a.g_s, (uint32_t)NT, -D, mb, e, g, acc[b][nb]);
            }
          }
      });
}

// Backward chain of the two-body and latent kinds: G = dE/dx_out (the head's
// contribution on MFMA) into g_store, recomputation with the pre-activations
// kept in scratch, dE/du = rs sum G h, then back through the layers.
template <int KIND, int D, int NT, int HN, int NL, bool SF, bool SR>
__global__ __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(kOcc, kOcc)))
void k_rr_bwd(MlpArgs a) {
  static_assert(NL >= 2, "register-resident chains have a hidden layer");
  constexpr int KD = D / 16, MBD = D / 32, NBP = rr_nbp(MBD);
  constexpr int KIN = kin_steps<KIND, D, NT>();
  constexpr int KH = HN / 16, NCH = (KH + kHeadChunk - 1) / kHeadChunk;
  const int E = live_edges(a);
  const int lane = threadIdx.x & 63, g = lane >> 5;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tile = blockIdx.x * kWaves + wave;
  const int e0 = tile * kEdgesPerWave;
  if (e0 >= E) return;
  const Rows R = rows_of(e0, E, lane);
  const float rs = KIND == kTwoBody ? 1.0f : a.res_scale;
  float u[kNE];
#pragma unroll
  for (int nb = 0; nb < kNE; ++nb) u[nb] = R.ok[nb] ? a.eb[(uint32_t)R.ec[nb] * kEB + kEB_U] : 0.0f;
  float* gst = a.g_store;
  auto load_G = [&](int mb, int nb) { return load_c(gst, (uint32_t)D, 0, mb, R.ec[nb], g); };
  bf16x8* area = lds_area<KD>();

  // 1. G = g_x + g_head @ W_head^T -> g_store rows, in K chunks.  With the
  // activations stored by the forward pass, the last chunk's epilogue also
  // does step 3 below on the G it holds, and the two-body kind, which needs
  // G nowhere else, neither stores it nor passes the partial sums between
  // chunks through memory: they stay in the wave's (then unused) LDS area in
  // BF16, the precision of the operand G then becomes.
  void* const zs = a.act_store ? a.act_store : a.act_scratch;
  const bool fused = a.act_store != nullptr;
  const bool lds_partial = fused && KIND == kTwoBody;
  float gu[kNE];
#pragma unroll
  for (int nb = 0; nb < kNE; ++nb) gu[nb] = 0.0f;
  bf16x8 hz[NBP][kNE][2];   // the pass's stored h, requested before its MFMAs
  f32x16 gxp[NBP][kNE];     // the pass's g_x rows (first chunk), added after its MFMAs
  static_for<0, NCH>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    constexpr int KC = KH - c * kHeadChunk < kHeadChunk ? KH - c * kHeadChunk : kHeadChunk;
    bf16x8 gh[kNE][KC];
    load_bform<KC, KC>(gh, 0, a.g_head, (uint32_t)HN, 16 * kHeadChunk * c, R.ec, g);
    const char* W = (const char*)a.rr.head_bwd + (size_t)c * kHeadChunk * MBD * (SR ? 2 : 1) * 1024;
    gemm<KC, MBD, SR>(
        gh, W,
        [&](int p, f32x16 (&acc)[NBP][kNE]) {
#pragma unroll
          for (int b = 0; b < NBP; ++b)
#pragma unroll
            for (int nb = 0; nb < kNE; ++nb) {
              const int mb = p * NBP + b;
              if (c == NCH - 1 && fused) {
                const bf16x8* z = zslot<NL, MBD>(zs, tile, NL - 1, mb, nb, lane);
                hz[b][nb][0] = z[0];
                hz[b][nb][1] = z[kZHalf];
              }
              if constexpr (c == 0) {
                acc[b][nb] = zero16();
                if (a.g_x) gxp[b][nb] = load_c(a.g_x, (uint32_t)D, 0, mb, R.ec[nb], g);
              } else if (lds_partial) {
                const bf16x8 q0 = area[(2 * mb * kNE + nb) * 64 + lane];
                const bf16x8 q1 = area[((2 * mb + 1) * kNE + nb) * 64 + lane];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                  acc[b][nb][j] = (float)q0[j];
                  acc[b][nb][8 + j] = (float)q1[j];
                }
              } else {
                acc[b][nb] = load_G(mb, nb);
              }
            }
        },
        [&](int p, f32x16 (&acc)[NBP][kNE]) {
          const bool last = c == NCH - 1 && fused;
#pragma unroll
          for (int b = 0; b < NBP; ++b)
#pragma unroll
            for (int nb = 0; nb < kNE; ++nb) {
              const int mb = p * NBP + b;
              if constexpr (c == 0) {
                if (a.g_x)
#pragma unroll
                  for (int i = 0; i < 16; ++i) acc[b][nb][i] += gxp[b][nb][i];
              }
              if (!last && lds_partial) {   // partial sums for the next chunk
                stash(area, 2 * mb, nb, lane, bform(acc[b][nb], 0, Ident()));
                stash(area, 2 * mb + 1, nb, lane, bform(acc[b][nb], 1, Ident()));
              } else if (R.ok[nb] && !(last && KIND == kTwoBody)) {
                store_c(gst, (uint32_t)D, 0, mb, R.ec[nb], g, acc[b][nb]);
              }
              if (last) {
                const bf16x8 h0 = hz[b][nb][0], h1 = hz[b][nb][1];
                f32x16 t;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                  gu[nb] = fmaf(acc[b][nb][j], (float)h0[j], gu[nb]);
                  gu[nb] = fmaf(acc[b][nb][8 + j], (float)h1[j], gu[nb]);
                }
#pragma unroll
                for (int i = 0; i < 16; ++i) t[i] = rs * u[nb] * acc[b][nb][i];
                stash(area, 2 * mb, nb, lane, bform(t, 0, Ident()));
                stash(area, 2 * mb + 1, nb, lane, bform(t, 1, Ident()));
              }
            }
        });
    __builtin_amdgcn_sched_barrier(0);
  });

  // 2. recompute the chain (pre-activations to scratch), unless the forward
  // pass stored them; 3. dE/du = rs sum G h and dE/dh = rs u G into the LDS
  // area (done in step 1's epilogue with stored activations)
  if (!fused) {
    {
      bf16x8 x0[kNE][KIN];
      chain_input<KIND, D, NT, KIN>(a, x0, R, g);
      __builtin_amdgcn_sched_barrier(0);
      hidden<D, NL, KIN, NL - 1, SF, SR>(a, x0, area, lane, zs, tile);
    }
    bf16x8 ah[kNE][KD];
    unstash<KD>(area, ah, lane);
    f32x16 Gb[NBP][kNE];
    gemm<KD, MBD, SR>(
        ah, a.rr.fwd[NL - 1],
        [&](int p, f32x16 (&acc)[NBP][kNE]) {
          Zero()(p, acc);
#pragma unroll
          for (int b = 0; b < NBP; ++b)
#pragma unroll
            for (int nb = 0; nb < kNE; ++nb) Gb[b][nb] = load_G(p * NBP + b, nb);
        },
        [&](int p, f32x16 (&acc)[NBP][kNE]) {
#pragma unroll
          for (int b = 0; b < NBP; ++b)
#pragma unroll
            for (int nb = 0; nb < kNE; ++nb) {
              const int mb = p * NBP + b;
              f32x16 t;
#pragma unroll
              for (int i = 0; i < 16; ++i) {
                gu[nb] = fmaf(Gb[b][nb][i], acc[b][nb][i], gu[nb]);
                t[i] = rs * u[nb] * Gb[b][nb][i];
              }
              stash(area, 2 * mb, nb, lane, bform(t, 0, Ident()));
              stash(area, 2 * mb + 1, nb, lane, bform(t, 1, Ident()));
            }
        });
  }
#pragma unroll
  for (int nb = 0; nb < kNE; ++nb) {
    const float s = rs * (gu[nb] + __shfl_xor(gu[nb], 32, 64));
    if (g == 0 && R.ok[nb]) {
      float* o = a.g_u + R.ec[nb];
      *o = a.gu_accum ? *o + s : s;
    }
  }
  __builtin_amdgcn_sched_barrier(0);

  // 4. back through the hidden layers; 5. dE/d(input)
  static_for<0, NL - 1>([&](auto lc) {
    constexpr int l = NL - 2 - decltype(lc)::value;   // hidden layer NL-2 down to 0
    bf16x8 d[kNE][KD];
    unstash<KD>(area, d, lane);
    back_layer<D, NL, SR>(zs, tile, lane, l, d, a.rr.bwd[l + 1], area);
  });
  bf16x8 dz[kNE][KD];
  unstash<KD>(area, dz, lane);
  input_grad<KIND, D, NT, KIN, SF>(a, dz, R, g, rs, load_G);
}

// Final layer, backward (NL >= 2): G = sigma_Z w_e; recompute the hidden
// layers, the last one giving dE/du = rs sigma_Z a . v and
// dE/dz = rs u sigma_Z v silu'(z) directly; then back to dE/d(input).
template <int D, int NT, int NL, bool SF, bool SR>
__global__ __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(kOcc, kOcc)))
void k_rr_bwd_final(MlpArgs a) {
  static_assert(NL >= 2, "folded final layer needs a hidden layer");
  constexpr int KD = D / 16, MBD = D / 32, NBP = rr_nbp(MBD);
  constexpr int KIN = (D + NT) / 16;
  const int E = live_edges(a);
  const int lane = threadIdx.x & 63, g = lane >> 5;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tile = blockIdx.x * kWaves + wave;
  const int e0 = tile * kEdgesPerWave;
  if (e0 >= E) return;
  const Rows R = rows_of(e0, E, lane);
  const float rs = a.res_scale;
  float ce[kNE], sg[kNE], av[kNE], xw[kNE];
  int zr[kNE];
#pragma unroll
  for (int nb = 0; nb < kNE; ++nb) {
    const float* rec = a.eb + (uint32_t)R.ec[nb] * kEB;
    zr[nb] = (int)rec[kEB_ZI];
    sg[nb] = a.sigma[zr[nb]];
    ce[nb] = R.ok[nb] ? rs * rec[kEB_U] * sg[nb] : 0.0f;
    av[nb] = 0.0f;
    xw[nb] = 0.0f;
  }
  auto load_G = [&](int mb, int nb) { return load_c(a.g_const, (uint32_t)D, 0, mb, zr[nb], g); };
  bf16x8* area = lds_area<KD>();
  f32x16 vb[NBP];
  auto pre_dot = [&](int p, f32x16 (&acc)[NBP][kNE]) {
    Zero()(p, acc);
#pragma unroll
    for (int b = 0; b < NBP; ++b) vb[b] = load_c(a.fold_v, 0u, 0, p * NBP + b, 0, g);
  };
  auto epi_dot = [&](int p, f32x16 (&acc)[NBP][kNE]) {
#pragma unroll
    for (int b = 0; b < NBP; ++b)
#pragma unroll
      for (int nb = 0; nb < kNE; ++nb) {
        f32x16 t;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const float z = acc[b][nb][i];
          av[nb] = fmaf(silu(z), vb[b][i], av[nb]);
          t[i] = ce[nb] * vb[b][i] * silu_grad(z);
        }
        const int mb = p * NBP + b;
        stash(area, 2 * mb, nb, lane, bform(t, 0, Ident()));
        stash(area, 2 * mb + 1, nb, lane, bform(t, 1, Ident()));
      }
  };
  void* const zs = a.act_store ? a.act_store : a.act_scratch;
  if (a.act_store) {
    // the forward pass stored the last hidden layer's pre-activations and a . v;
    // the next block's are requested while this block's are used
    bf16x8 zn[kNE][2];
#pragma unroll
    for (int nb = 0; nb < kNE; ++nb) {
      const bf16x8* z = zslot<NL, MBD>(zs, tile, NL - 2, 0, nb, lane);
      zn[nb][0] = z[0];
      zn[nb][1] = z[kZHalf];
    }
    for (int mb = 0; mb < MBD; ++mb) {
      const f32x16 v = load_c(a.fold_v, 0u, 0, mb, 0, g);
      bf16x8 zc[kNE][2];
#pragma unroll
      for (int nb = 0; nb < kNE; ++nb) {
        zc[nb][0] = zn[nb][0];
        zc[nb][1] = zn[nb][1];
        if (mb + 1 < MBD) {
          const bf16x8* z = zslot<NL, MBD>(zs, tile, NL - 2, mb + 1, nb, lane);
          zn[nb][0] = z[0];
          zn[nb][1] = z[kZHalf];
        }
      }
#pragma unroll
      for (int nb = 0; nb < kNE; ++nb) {
        const bf16x8 z0 = zc[nb][0], z1 = zc[nb][1];
        f32x16 t;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          t[j] = ce[nb] * v[j] * silu_grad((float)z0[j]);
          t[8 + j] = ce[nb] * v[8 + j] * silu_grad((float)z1[j]);
        }
        stash(area, 2 * mb, nb, lane, bform(t, 0, Ident()));
        stash(area, 2 * mb + 1, nb, lane, bform(t, 1, Ident()));
      }
    }
#pragma unroll
    for (int nb = 0; nb < kNE; ++nb)
      if (g == 0) av[nb] = a.av_store[R.ec[nb]];   // the full sum, in one half-wave
  } else {
    {
      bf16x8 x0[kNE][KIN];
      final_input<D, NT, 9, KIN>(a, x0, R, g, true, xw);
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (NL == 2) gemm<KIN, MBD, SF>(x0, a.rr.fwd[0], pre_dot, epi_dot);
      else hidden<D, NL, KIN, NL - 2, SF, SR>(a, x0, area, lane, zs, tile);
    }
    if constexpr (NL > 2) {
      bf16x8 ah[kNE][KD];
      unstash<KD>(area, ah, lane);
      gemm<KD, MBD, SR>(ah, a.rr.fwd[NL - 2], pre_dot, epi_dot);
    }
  }
#pragma unroll
  for (int nb = 0; nb < kNE; ++nb) {
    const float s = rs * sg[nb] * (av[nb] + __shfl_xor(av[nb], 32, 64));
    if (g == 0 && R.ok[nb]) {
      float* o = a.g_u + R.ec[nb];
      *o = a.gu_accum ? *o + s : s;
    }
  }
  __builtin_amdgcn_sched_barrier(0);
  static_for<0, NL - 2>([&](auto lc) {
    constexpr int l = NL - 3 - decltype(lc)::value;   // hidden layer NL-3 down to 0
    bf16x8 d[kNE][KD];
    unstash<KD>(area, d, lane);
    back_layer<D, NL, SR>(zs, tile, lane, l, d, a.rr.bwd[l + 1], area);
  });
  bf16x8 dz[kNE][KD];
  unstash<KD>(area, dz, lane);
  input_grad<kLatentFinal, D, NT, KIN, SF>(a, dz, R, g, rs, load_G);
}

// Bytes of an activation array (recomputation scratch of the backward
// kernels, or the stored activations of one chain) for E edges: NL slots of
// D BF16 values per edge.
inline size_t scratch_bytes(int64_t E, int D, int NL) {
  const int64_t tiles = (E + kEdgesPerWave - 1) / kEdgesPerWave;
  return (size_t)tiles * NL * (D / 32) * kNE * 64 * 32;
}

// LDS bytes of a block (one B-operand area of D/16 K steps per wave).
constexpr size_t lds_bytes(int D) { return (size_t)kWaves * ((D / 16) * kNE * 64 * 16 + 4096); }

template <class K>
hipError_t launch_kernel(K k, const MlpArgs& a, int D, hipStream_t s) {
  const int tiles = (a.E + kEdgesPerWave - 1) / kEdgesPerWave;
  const dim3 grid((tiles + kWaves - 1) / kWaves), block(64 * kWaves);
  const size_t bytes = lds_bytes(D);
  hipError_t st = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (st != hipSuccess) return st;
  hipLaunchKernelGGL(k, grid, block, bytes, s, a);
  return hipGetLastError();
}

template <int KIND, int D, int NT, int HN, int NL, bool SF, bool SR>
hipError_t launch_fwd(const MlpArgs& a, hipStream_t s) {
  if constexpr (KIND == kLatentFinal)
    return launch_kernel(k_rr_fwd_final<D, NT, (HN / NT) * (HN / NT), NL, SF, SR>, a, D, s);
  else
    return launch_kernel(k_rr_fwd<KIND, D, NT, HN, NL, SF, SR>, a, D, s);
}

template <int KIND, int D, int NT, int HN, int NL, bool SF, bool SR>
hipError_t launch_bwd(const MlpArgs& a, hipStream_t s) {
  if constexpr (KIND == kLatentFinal)
    return launch_kernel(k_rr_bwd_final<D, NT, NL, SF, SR>, a, D, s);
  else
    return launch_kernel(k_rr_bwd<KIND, D, NT, HN, NL, SF, SR>, a, D, s);
}
