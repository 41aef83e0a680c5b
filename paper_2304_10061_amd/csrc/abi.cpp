// abi.cpp - the C interface: model construction (weight packing, coupling
// tables), the neighbour-list driver and the energy/force driver.
//
// Host-side work happens once per model (allegro_create) or once per neighbour
// build (allocation of the edge workspace, which depends on the edge count);
// allegro_energy_forces only enqueues kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/allegro_mi355x.h"
#include "coupling.h"
#include "internal.h"

using namespace allegro;

// Workspace of allegro_energy_forces_noalloc: one array per GPU, created with
// the code object and held until the process ends.  Host code never uses the
// array's name as an address (on the host it names a stand-in): each device's
// address is looked up once, by allegro_create with that device current, and
// kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[ALLEGRO_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string g_create_error;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch`, per device

struct Fail {
  int code;
  std::string msg;
};

#define HIP_OK(expr)                                                                         \
  do {                                                                                       \
    hipError_t _e = (expr);                                                                  \
    if (_e != hipSuccess)                                                                    \
      throw Fail{ALLEGRO_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)};       \
  } while (0)

#define REQUIRE(cond, msg)                                  \
  do {                                                      \
    if (!(cond)) throw Fail{ALLEGRO_E_INVAL, (msg)};        \
  } while (0)

// Device allocation that only grows.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  void ensure(size_t want) {
    if (want <= bytes && p) return;
    release();
    if (want == 0) want = 256;
    if (hipMalloc(&p, want) != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      throw Fail{ALLEGRO_E_NOMEM, "hipMalloc of " + std::to_string(want) + " bytes failed"};
    }
    bytes = want;
  }
  template <class T> T* as() const { return (T*)p; }
};

void upload(DevBuf& b, const void* src, size_t bytes) {
  b.ensure(bytes);
  HIP_OK(hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice));
}

int rup(int v, int m) { return ((v + m - 1) / m) * m; }

// Packs a K x N row-major matrix (y = x @ W) into MFMA B fragments.
// prec 0: FP32; prec 1: BF16 pairs (hi fragments, then lo = W - hi); prec 2: BF16.
void pack_b(const std::vector<double>& W, int K, int N, int prec, std::vector<char>& out, GemmB& g) {
  const int Kp = rup(K, 32), Np = rup(N, 32), nkb = Kp / 32;
  const size_t count = (size_t)Kp * Np;
  const int esz = prec ? 2 : 4;
  out.assign(count * esz * (prec == 1 ? 2 : 1), 0);
  for (int k = 0; k < K; ++k)
    for (int n = 0; n < N; ++n) {
      const int nt = n / 16, kb = k / 32, lane = (n % 16) + 16 * ((k % 32) / 8), el = k % 8;
      const size_t idx = ((size_t)(nt * nkb + kb) * 64 + lane) * 8 + el;
      const double w = W[(size_t)k * N + n];
      if (prec) {
        const __bf16 hi = (__bf16)(float)w;
        std::memcpy(out.data() + idx * 2, &hi, 2);
        if (prec == 1) {
          const __bf16 lo = (__bf16)(float)(w - (double)(float)hi);
          std::memcpy(out.data() + (count + idx) * 2, &lo, 2);
        }
      } else {
        const float v = (float)w;
        std::memcpy(out.data() + idx * 4, &v, 4);
      }
    }
  g.K = K; g.N = N; g.Kp = Kp; g.Np = Np;
  g.split = prec == 1 ? 1 : 0;
}

std::vector<double> transpose(const std::vector<double>& W, int K, int N) {
  std::vector<double> T((size_t)K * N);
  for (int k = 0; k < K; ++k)
    for (int n = 0; n < N; ++n) T[(size_t)n * K + k] = W[(size_t)k * N + n];
  return T;
}

// Packs M (Kin x Nout, row-major: out = in @ M) as A fragments of the
// register-resident kernels (layout in internal.h, RRW).  split: BF16 pairs
// (hi fragment, then lo = M - hi) instead of single-rounded BF16.
void pack_rr(const double* M, int Kin, int Nout, bool split, std::vector<char>& out) {
  const int KS = (Kin + 15) / 16, MB = (Nout + 31) / 32, NBP = rr_nbp(MB), NP = MB / NBP, S = split ? 2 : 1;
  const size_t base = out.size();
  out.resize(base + (size_t)NP * KS * NBP * S * 1024, 0);
  for (int p = 0; p < NP; ++p)
    for (int ks = 0; ks < KS; ++ks)
      for (int b = 0; b < NBP; ++b)
        for (int lane = 0; lane < 64; ++lane)
          for (int j = 0; j < 8; ++j) {
            const int m = 32 * (p * NBP + b) + lane % 32, gq = lane / 32;
            const int f = 16 * ks + (j < 4 ? 4 * gq + j : 8 + 4 * gq + (j - 4));
            const double w = (m < Nout && f < Kin) ? M[(size_t)f * Nout + m] : 0.0;
            const __bf16 hi = (__bf16)(float)w;
            const size_t frag = ((size_t)(p * KS + ks) * NBP + b) * S;
            std::memcpy(out.data() + base + ((frag * 64 + lane) * 8 + j) * 2, &hi, 2);
            if (split) {
              const __bf16 lo = (__bf16)(float)(w - (double)(float)hi);
              std::memcpy(out.data() + base + (((frag + 1) * 64 + lane) * 8 + j) * 2, &lo, 2);
            }
          }
}

// The same for a head transpose, in K chunks of 192 rows (the backward kernels
// take the head gradient 12 K steps at a time).
void pack_rr_chunked(const std::vector<double>& M, int Kin, int Nout, bool split, std::vector<char>& out) {
  for (int r0 = 0; r0 < Kin; r0 += 192) pack_rr(M.data() + (size_t)r0 * Nout, std::min(192, Kin - r0), Nout, split, out);
}

struct PackedMat {
  DevBuf buf;
  GemmB g;
};

void make_packed(PackedMat& pm, const std::vector<double>& W, int K, int N, int prec) {
  std::vector<char> host;
  pack_b(W, K, N, prec, host, pm.g);
  upload(pm.buf, host.data(), host.size());
  pm.g.p = pm.buf.p;
}

struct Validated {
  int S, nb, p, lmax, nl, n, d, dim, LW, h;
  // irrep kinds (TpKind) of each layer's input and output features, the
  // output width in strided components, and whether the weight file uses the
  // parity-extended alpha / mixing layouts (models with unnatural irreps)
  int in_kind[kMaxLayers], out_kind[kMaxLayers], w_out[kMaxLayers];
  bool parity = false;
  std::vector<int> dims2b, dimsL;
  int64_t n_weights;
};

bool pow2_in(int n) { return n == 8 || n == 16 || n == 32 || n == 64; }

Validated validate(const AllegroConfig* c) {
  REQUIRE(c != nullptr, "config is NULL");
  Validated v{};
  v.S = c->n_species; v.nb = c->n_bessel; v.p = c->envelope_p; v.lmax = c->l_max;
  v.nl = c->n_layers; v.n = c->n_tensor;
  REQUIRE(v.S >= 1 && v.S <= 12, "n_species must be in 1..12");
  REQUIRE(v.nb >= 1 && v.nb <= 16, "n_bessel must be in 1..16");
  REQUIRE(2 * v.S + v.nb <= 32, "2 n_species + n_bessel must be at most 32");
  REQUIRE(v.p >= 2 && v.p <= 12, "envelope_p must be in 2..12");
  REQUIRE(v.lmax >= 1 && v.lmax <= 3, "l_max must be 1, 2 or 3");
  REQUIRE(v.nl >= 1 && v.nl <= kMaxLayers, "n_layers must be 1..4");
  REQUIRE(pow2_in(v.n), "n_tensor must be 8, 16, 32 or 64");
  REQUIRE((v.lmax <= 2 && v.nl <= 2) || v.n == 32 || v.n == 64,
          "l_max 3 and models of 3 or more layers need n_tensor 32 or 64");
  REQUIRE(v.lmax <= 2 || v.nb <= 8, "l_max 3 allows at most 8 Bessel functions");
  REQUIRE(c->n_twobody >= 1 && c->n_twobody <= 3, "n_twobody must be 1..3");
  REQUIRE(c->n_latent >= 1 && c->n_latent <= 3, "n_latent must be 1..3");
  REQUIRE(c->n_edge == 1, "edge MLP must have exactly one hidden layer");
  for (int k = 0; k < c->n_twobody; ++k) v.dims2b.push_back(c->twobody_dims[k]);
  for (int k = 0; k < c->n_latent; ++k) v.dimsL.push_back(c->latent_dims[k]);
  v.d = v.dims2b.back();
  REQUIRE(v.dimsL.back() == v.d, "last latent width must equal last two-body width");
  REQUIRE(v.d <= 256, "latent width d must be at most 256");
  for (int w : v.dims2b) REQUIRE(w >= 16 && w <= 512 && w % 16 == 0, "MLP widths must be multiples of 16 in 16..512");
  for (int w : v.dimsL) REQUIRE(w >= 16 && w <= 512 && w % 16 == 0, "MLP widths must be multiples of 16 in 16..512");
  v.h = c->edge_dims[0];
  REQUIRE(v.h >= 1 && v.h <= 4096, "edge hidden width must be in 1..4096");
  REQUIRE(c->r_cut > 0 && std::isfinite(c->r_cut), "r_cut must be positive");
  REQUIRE(c->avg_num_neighbors > 0 && std::isfinite(c->avg_num_neighbors), "avg_num_neighbors must be positive");
  REQUIRE(c->precision == ALLEGRO_PREC_FP32 || c->precision == ALLEGRO_PREC_BF16 ||
              c->precision == ALLEGRO_PREC_BF16_SINGLE || c->precision == ALLEGRO_PREC_BF16_MIXED,
          "precision must be 0, 1, 2 or 3");
  REQUIRE(c->edge_chunk >= 0, "edge_chunk must be >= 0");
  REQUIRE(c->neighbor_skin >= 0 && std::isfinite(c->neighbor_skin), "neighbor_skin must be >= 0");
  REQUIRE(c->edge_capacity_hint >= 0, "edge_capacity_hint must be >= 0");
  if (c->atomic_numbers)
    for (int k = 0; k < v.S; ++k)
      REQUIRE(c->atomic_numbers[k] >= 1 && c->atomic_numbers[k] <= 118, "atomic_numbers must lie in 1..118");
  if (c->r_cut_pair)
    for (int k = 0; k < v.S * v.S; ++k)
      REQUIRE(std::isfinite(c->r_cut_pair[k]) && c->r_cut_pair[k] > 0 && c->r_cut_pair[k] <= c->r_cut,
              "r_cut_pair entries must lie in (0, r_cut]");
  v.dim = (v.lmax + 1) * (v.lmax + 1);
  v.LW = (v.lmax + 1) * v.n;
  // with three or more layers the first layer's cross-parity products (such as
  // 1o x 1o -> 1e) reach the scalar output through a later layer, so the
  // features of every layer but the last two hold both parities
  for (int L = 0; L < v.nl; ++L) {
    const bool last = L == v.nl - 1, penult = L == v.nl - 2;
    v.in_kind[L] = (L == 0 || last) ? kNatural : kBothParities;
    v.out_kind[L] = last ? kScalarOut : ((v.nl >= 3 && !penult) ? kBothParities : kNatural);
    v.w_out[L] = kind_width(v.out_kind[L], v.lmax);
  }
  v.parity = v.nl >= 3;
  // weight count, in the documented order
  int64_t cnt = 0;
  int prev = 2 * v.S + v.nb;
  for (int w : v.dims2b) { cnt += (int64_t)prev * w; prev = w; }
  cnt += (int64_t)v.d * v.LW;                              // embed0
  const int L1 = v.lmax + 1;
  for (int L = 0; L < v.nl; ++L) {
    cnt += (int64_t)v.d * v.LW;                            // env
    cnt += (int64_t)(v.parity ? 2 : 1) * L1 * L1 * L1;      // alpha
    cnt += (int64_t)(v.parity ? 2 : 1) * L1 * v.n * v.n;    // mix
    prev = v.d + v.n;
    for (int w : v.dimsL) { cnt += (int64_t)prev * w; prev = w; }
  }
  cnt += (int64_t)v.d * v.h + v.h;                         // edge MLP
  v.n_weights = cnt;
  return v;
}

// Widest row, in floats, of any array the kernels index by (chunk-local edge
// or centre) x (row stride) with 32-bit element offsets: the edge record,
// latent rows, heads and their gradients, tensor features and their adjoints
// (up to 2 dim n floats per edge with both parities), per-centre environment
// sums (dim n per centre, and a chunk never has more centres than edges).
int64_t widest_row(const Validated& v) {
  int64_t w = std::max<int64_t>(kEB, gy_width(v.lmax));
  w = std::max<int64_t>(w, v.d);
  w = std::max<int64_t>(w, 2 * (int64_t)v.LW);
  w = std::max<int64_t>(w, (int64_t)v.dim * v.n);
  for (int L = 0; L < v.nl; ++L) w = std::max<int64_t>(w, (int64_t)v.w_out[L] * v.n);
  for (int wd : v.dims2b) w = std::max<int64_t>(w, wd);
  for (int wd : v.dimsL) w = std::max<int64_t>(w, wd);
  return w;
}

// Largest number of edges one chunk may hold: every edge-row offset of the
// chunk stays below 2^31 elements (so signed and unsigned 32-bit offset
// arithmetic alike cannot wrap).
int64_t max_chunk_edges(const Validated& v) { return (((int64_t)1 << 31) - 1) / widest_row(v); }

// Splits centres [0, n_centres) into consecutive chunks of whole centre
// segments holding at most `cap` edges each (row_ptr[c] = first edge of centre
// c).  Returns the chunk boundaries (first entry 0, last n_centres); throws
// when a single centre has more than `cap` edges.
std::vector<int64_t> plan_chunks(const int64_t* row_ptr, int64_t n_centres, int64_t cap) {
  std::vector<int64_t> bounds(1, 0);
  int64_t c = 0;
  while (c < n_centres) {
    REQUIRE(row_ptr[c + 1] - row_ptr[c] <= cap,
            "centre " + std::to_string(c) + " has more edges than one chunk may hold");
    int64_t b = c + 1;
    while (b < n_centres && row_ptr[b + 1] - row_ptr[c] <= cap) ++b;
    bounds.push_back(b);
    c = b;
  }
  return bounds;
}

// Edges per chunk for a configuration: edge_chunk (0 = unlimited), capped so
// that 32-bit offsets cannot wrap.
int64_t chunk_cap(const Validated& v, int64_t edge_chunk) {
  const int64_t hard = max_chunk_edges(v);
  return edge_chunk > 0 ? std::min(edge_chunk, hard) : hard;
}

// Paths of a layer with the given kinds, as (l1, s1, l2, l_out, s_out) with s = 0
// for natural and 1 for unnatural parity.
struct PathId { int l1, s1, l2, lo, so; };

std::vector<PathId> layer_path_ids(int lmax, int in_kind, int out_kind) {
  std::vector<PathId> out;
  const int D = (lmax + 1) * (lmax + 1);
  for (int s1 = 0; s1 < 2; ++s1)
    for (int l1 = 0; l1 <= lmax; ++l1)
      for (int l2 = 0; l2 <= lmax; ++l2)
        for (int so = 0; so < 2; ++so)
          for (int lo = 0; lo <= lmax; ++lo) {
            // representative components: the path is kept iff they are
            const int a = s1 * D + l1 * l1, b = l2 * l2, c = so * D + lo * lo;
            if (path_kept(a, b, c, lmax, in_kind, out_kind)) out.push_back(PathId{l1, s1, l2, lo, so});
          }
  return out;
}

// Fused coupling-table values of one layer, in the compile-time pattern order:
// w_k = alpha_p / sqrt(P_out) * C_p[a, b, c] / |C_p|.
template <class Pat>
std::vector<float> fused_values(const double* alpha_raw, bool parity_layout) {
  constexpr int LMAX = Pat::Lmax, L1 = LMAX + 1, D = Pat::DIM;
  int per_out[2][kMaxLmax + 1] = {};
  double norm2[2][kMaxLmax + 1][kMaxLmax + 1][kMaxLmax + 1] = {};
  for (const PathId& p : layer_path_ids(LMAX, Pat::In, Pat::Out)) {
    per_out[p.so][p.lo]++;
    for (int a = p.l1 * p.l1; a < (p.l1 + 1) * (p.l1 + 1); ++a)
      for (int b = p.l2 * p.l2; b < (p.l2 + 1) * (p.l2 + 1); ++b)
        for (int c = p.lo * p.lo; c < (p.lo + 1) * (p.lo + 1); ++c) {
          const double g = coupling_raw(a, b, c);
          norm2[p.s1][p.l1][p.l2][p.lo] += g * g;
        }
  }
  std::vector<float> out(Pat::NNZ);
  for (int k = 0; k < Pat::NNZ; ++k) {
    const TpEntry t = Pat::list.e[k];
    const int s1 = t.a >= D, so = t.c >= D;
    const int a = t.a - s1 * D, c = t.c - so * D;
    const int l1 = l_of(a), l2 = l_of(t.b), lo = l_of(c);
    const double raw = parity_layout ? alpha_raw[((s1 * L1 + l1) * L1 + l2) * L1 + lo] : alpha_raw[(l1 * L1 + l2) * L1 + lo];
    const double al = raw / std::sqrt((double)per_out[so][lo]);
    out[k] = (float)(al * coupling_raw(a, t.b, c) / std::sqrt(norm2[s1][l1][l2][lo]));
  }
  return out;
}

template <int LMAX>
std::vector<float> fused_values_l(int in, int out, const double* alpha, bool parity) {
  if (in == kNatural) {
    if (out == kScalarOut) return fused_values<TpPattern<LMAX, kNatural, kScalarOut>>(alpha, parity);
    if (out == kNatural) return fused_values<TpPattern<LMAX, kNatural, kNatural>>(alpha, parity);
    return fused_values<TpPattern<LMAX, kNatural, kBothParities>>(alpha, parity);
  }
  if (out == kNatural) return fused_values<TpPattern<LMAX, kBothParities, kNatural>>(alpha, parity);
  return fused_values<TpPattern<LMAX, kBothParities, kBothParities>>(alpha, parity);
}

std::vector<float> fused_values_rt(int lmax, int in, int out, const double* alpha, bool parity) {
  if (lmax == 1) return fused_values_l<1>(in, out, alpha, parity);
  if (lmax == 2) return fused_values_l<2>(in, out, alpha, parity);
  return fused_values_l<3>(in, out, alpha, parity);
}

int count_paths(int lmax, int in, int out) { return (int)layer_path_ids(lmax, in, out).size(); }

template <int LMAX>
int count_nonzeros_l(int in, int out) {
  if (in == kNatural) {
    if (out == kScalarOut) return TpPattern<LMAX, kNatural, kScalarOut>::NNZ;
    if (out == kNatural) return TpPattern<LMAX, kNatural, kNatural>::NNZ;
    return TpPattern<LMAX, kNatural, kBothParities>::NNZ;
  }
  if (out == kNatural) return TpPattern<LMAX, kBothParities, kNatural>::NNZ;
  return TpPattern<LMAX, kBothParities, kBothParities>::NNZ;
}

int count_nonzeros(int lmax, int in, int out) {
  return lmax == 1 ? count_nonzeros_l<1>(in, out) : (lmax == 2 ? count_nonzeros_l<2>(in, out) : count_nonzeros_l<3>(in, out));
}


struct Mlp {
  PackedMat fwd[kMaxMlpLayers], bwd[kMaxMlpLayers];
  DevBuf rr_fwd[kMaxMlpLayers], rr_bwd[kMaxMlpLayers];   // register-resident kernels' packing
  int nl = 0;
  MlpW view() const {
    MlpW w;
    w.nl = nl;
    for (int k = 0; k < nl; ++k) { w.fwd[k] = fwd[k].g; w.bwd[k] = bwd[k].g; }
    return w;
  }
};

}  // namespace

// Per-evaluation workspace: every array allegro_energy_forces writes and
// reads back within one call (activations of the current chunk, gradients,
// per-edge dE/dr for the force gather, per-atom energies when the caller
// passes none, partial sums).  Nothing in it carries over between calls, and
// no kernel relies on it starting at zero.  ws_layout carves it out of one
// block starting at `base` (256-byte aligned pieces) and returns its size;
// with base = 0 it only measures.
struct Ws {
  float *eb = nullptr, *x[kMaxLayers] = {}, *head0o = nullptr, *wenv[kMaxLayers] = {}, *V[kMaxLayers] = {},
        *gam[kMaxLayers] = {}, *eij = nullptr, *gxa = nullptr, *gxb = nullptr, *gTf = nullptr, *gs = nullptr,
        *ghead0 = nullptr, *gw2 = nullptr, *gT[2] = {}, *gY = nullptr, *gu = nullptr, *gR = nullptr,
        *ggam = nullptr, *epair = nullptr, *g_e = nullptr;
  void* zscr = nullptr;      // hidden pre-activations of the 128-row backward MLP kernels
  // activations stored by the register-resident forward kernels for their
  // backward (two-body, latent layers 0 .. nl-2, final; a . v of the final)
  void* zst[kMaxLayers + 1] = {};
  float* av = nullptr;
  double *atom_e = nullptr, *partial = nullptr;
};

// Ec / Nc: most edges / centres of one chunk; E: all edges; n_local, n_total:
// atoms of the list.
size_t ws_layout(const Validated& v, int64_t Ec, int64_t Nc, int64_t E, int64_t n_local, int64_t n_total,
                 bool zbl, bool tall, bool rr, uintptr_t base, Ws* w) {
  Ec = std::max<int64_t>(Ec, 1); Nc = std::max<int64_t>(Nc, 1); E = std::max<int64_t>(E, 1);
  const int64_t nt = std::max<int64_t>(n_total, 1), nl = std::max<int64_t>(n_local, 1);
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    const size_t at = off;
    off += (bytes + 255) & ~(size_t)255;
    return base ? (void*)(base + at) : nullptr;
  };
  auto fl = [&](int64_t count) { return (float*)take((size_t)count * sizeof(float)); };
  Ws t;
  t.eb = fl(Ec * kEB);
  for (int L = 0; L < v.nl; ++L) t.x[L] = fl(Ec * v.d);
  t.head0o = fl(Ec * 2 * v.LW);
  if (v.nl >= 2) {
    int wmax = 0;
    for (int L = 0; L + 1 < v.nl; ++L) {
      t.wenv[L + 1] = fl(Ec * v.LW);
      t.V[L] = fl(Ec * v.w_out[L] * v.n);
      wmax = std::max(wmax, v.w_out[L]);
    }
    t.gw2 = fl(Ec * v.LW);
    t.gT[0] = fl(Ec * wmax * v.n);
    if (v.nl >= 3) t.gT[1] = fl(Ec * wmax * v.n);
    t.gxb = fl(Ec * v.d);
    t.gs = fl(Ec * v.n);
  }
  for (int L = 0; L < v.nl; ++L) t.gam[L] = fl(Nc * v.dim * v.n);
  t.ggam = fl(Nc * v.dim * v.n);
  t.eij = fl(Ec);
  t.gxa = fl(Ec * v.d);
  t.gTf = fl(Ec * v.n);
  t.ghead0 = fl(Ec * 2 * v.LW);
  t.gY = fl(Ec * gy_width(v.lmax));
  t.gu = fl(Ec);
  t.gR = fl(Ec * v.nb);
  if (zbl) t.epair = fl(Ec);
  if (tall || rr)
    t.zscr = take(std::max(tall ? mlp_tall_scratch_bytes(Ec, v.d) : (size_t)0,
                           rr ? mlp_rr_scratch_bytes(Ec, v.d, (int)v.dims2b.size()) : (size_t)0));
  if (rr) {
    for (int k = 0; k <= v.nl; ++k) t.zst[k] = take(mlp_rr_scratch_bytes(Ec, v.d, (int)v.dims2b.size()));
    t.av = fl(Ec);
  }
  t.g_e = fl(E * 3);
  t.atom_e = (double*)take((size_t)nl * sizeof(double));
  t.partial = (double*)take((size_t)((nt + 255) / 256) * 10 * sizeof(double));
  if (w) *w = t;
  return off;
}

struct AllegroModel {
  AllegroConfig cfg{};
  Validated v{};
  int prec = 1;
  // kernel precision of the two-body / later MLPs (0 FP32, 1 BF16 with
  // per-matrix hi + lo pairs, 2 BF16 single-rounded) and the packing of the
  // later MLPs' first and other layers (same codes)
  int prec_two = 1, prec_lat = 1, prec_lat_first = 1, prec_lat_rest = 1;
  std::string err;
  int device = 0;

  Mlp twobody, latent[kMaxLayers];
  int rr_cfg = 0;                         // register-resident kernels (rr_config), 0 = none
  DevBuf rr_head0, rr_head0T, rr_envH[kMaxLayers], rr_envHT[kMaxLayers], rr_fold_v;
  PackedMat head0, head0T;                // [embed0 | env of layer 1] after the two-body MLP
  PackedMat envH[kMaxLayers], envHT[kMaxLayers];   // env of layer L+1 after latent MLP L
  // ordered species-pair cutoffs (empty = r_cut for every pair): the host
  // copy, FP32 radii for the edge kernels, squared list radii for the list
  std::vector<double> rc_pair;
  DevBuf rc_pair_f, rc2_pair;
  // ZBL term: atomic numbers (empty = none), their device table [Z | Z^0.23]
  // and the per-edge pair shares of the current chunk
  std::vector<int> znum;
  DevBuf zbl_tab;
  DevBuf mixF[kMaxLayers], mixB[kMaxLayers];   // packed FP32 mixing matrices per layer and irrep slot
  int mix_stride = 0;
  DevBuf tpw[kMaxLayers];                 // fused coupling non-zeros per layer
  std::vector<float> tpw_host[kMaxLayers];
  float tp_final[16] = {0};               // final-layer diagonal weights
  DevBuf we, gconst, scale, shift;
  float sigma_f[16] = {0};                // species scales sigma_Z (FP32 copy)
  double c_norm = 1.0;

  // neighbour list
  int64_t n_local = -1, n_total = 0, E = 0;
  double L[3] = {0, 0, 0};
  DevBuf ei, ej, es, row_ptr, rrow_ptr, redge, keys;
  DevBuf cell_of, img, cell_count, cell_start, cell_cursor, cell_atoms, count, rcount, rcursor;
  DevBuf bbox, scan_tmp, err_flag;
  DevBuf status;                          // sticky device status bits (kStatus*)
  int n_sys = 0;                          // batched mode: number of independent systems
  DevBuf sys_off, sys_id, sys_shift;
  std::vector<int32_t> h_row_ptr;
  std::vector<int64_t> chunk_c;           // centre boundaries of chunks
  std::vector<int64_t> chunk_rp_off;      // offset of each chunk's rebased row pointers
  DevBuf chunk_rp;
  int64_t Ec = 0, Nc = 0;
  // edge capacity of the list buffers, and what an in-graph rebuild needs:
  // the last build's grid and buffers (NbrArgs), its cell count and box
  int64_t cap = 0;
  NbrArgs nbr{};
  int64_t n_cells = 0;
  bool dev_rebuild = false;               // single-chunk list: rebuilds can run on the device
  double last_cell[9] = {0};
  int32_t last_pbc[3] = {0, 0, 0};
  bool last_has_cell = false;
  std::vector<int64_t> last_sys_off;

  // tile shapes chosen by allegro_autotune (0 = default)
  int tm_choice[6] = {0, 0, 0, 0, 0, 0};   // MLP kernels, see kMlpSlotNames
  int tt_choice[2] = {0, 0};               // tp_mix, mix_adjoint

  // molecular dynamics
  uint64_t nbr_version = 0;               // bumped by every neighbour build
  int64_t n_ghost = 0, ghost_n_local = 0;
  DevBuf g_owner, g_offset, g_ptr, g_idx; // ghost images and the owner -> ghosts CSR
  DevBuf pos_ref;                         // positions of the centres at the last neighbour build
  DevBuf md_epot, md_part, md_counter, md_atom_e, tune_forces, md_vir;
  DevBuf md_flags;                        // kFlag* slots of the in-graph rebuild
  DevBuf bak_pos, bak_vel, bak_f;         // state at the start of the step that overflowed
  hipStream_t md_stream = nullptr;
  hipEvent_t md_ev[2] = {nullptr, nullptr};
  hipGraph_t md_graph = nullptr;
  hipGraphExec_t md_exec = nullptr;
  std::vector<uintptr_t> md_key;
  int64_t graph_captures = 0;             // MD step graphs captured so far
  int64_t last_run_rebuilds = 0;          // list rebuilds in the last allegro_md_run
  int64_t need_edges = 0;                 // largest list a device rebuild asked for

  // optional per-kernel timing with HIP events on the caller's stream
  bool timing = false;
  struct KTime { std::string name; double ms = 0.0; int64_t launches = 0; };
  std::vector<KTime> ktimes;
  std::vector<std::pair<size_t, std::pair<hipEvent_t, hipEvent_t>>> pending;

  // workspace of the current neighbour list (ws_layout) and its pieces:
  // x[L]: input of layer L; wenv[L] (L >= 1): its environment weights; V[L]:
  // output features of non-final layer L; gT[2]: dE/dT of consecutive
  // non-final layers during the adjoint; ggam: dE/dGamma of the layer being
  // differentiated [centres][dim][n]
  DevBuf arena;
  size_t ws_bytes = 0;
  Ws ws;
};

namespace {

int fail(AllegroModel* m, const Fail& f) {
  if (m) m->err = f.msg;
  else g_create_error = f.msg;
  return f.code;
}

std::vector<double> slice(const float* w, int64_t& off, int64_t count) {
  std::vector<double> out(w + off, w + off + count);
  off += count;
  return out;
}

// prec_first applies to the first layer, prec_rest to the others.
void build_mlp(Mlp& mlp, const std::vector<std::vector<double>>& Ws, const std::vector<int>& dims, int prec_first,
               int prec_rest, bool rr) {
  mlp.nl = (int)Ws.size();
  for (int k = 0; k < mlp.nl; ++k) {
    const int prec = k == 0 ? prec_first : prec_rest;
    const std::vector<double> T = transpose(Ws[k], dims[k], dims[k + 1]);
    make_packed(mlp.fwd[k], Ws[k], dims[k], dims[k + 1], prec);
    make_packed(mlp.bwd[k], T, dims[k + 1], dims[k], prec);
    if (rr) {
      std::vector<char> f, b;
      pack_rr(Ws[k].data(), dims[k], dims[k + 1], prec == 1, f);
      pack_rr(T.data(), dims[k + 1], dims[k], prec == 1, b);
      upload(mlp.rr_fwd[k], f.data(), f.size());
      upload(mlp.rr_bwd[k], b.data(), b.size());
    }
  }
}

RRW rr_view(const Mlp& mlp, int cfg, const DevBuf* head, const DevBuf* head_bwd) {
  RRW r;
  if (!cfg) return r;
  r.cfg = cfg;
  for (int k = 0; k < mlp.nl; ++k) { r.fwd[k] = mlp.rr_fwd[k].p; r.bwd[k] = mlp.rr_bwd[k].p; }
  r.head = head ? head->p : nullptr;
  r.head_bwd = head_bwd ? head_bwd->p : nullptr;
  return r;
}

// Configurations the register-resident kernels are compiled for (0 = none):
// 1 = latent width 256, 64 tensor channels, l_max 2, three-layer two-body and
// latent MLPs of width 256; 2 = 128, 32, l_max 2, two-layer MLPs of width 128.
// Both need the two-body input (2 species + radial functions) within 16.
int rr_config(const Validated& v, int prec) {
  if (prec == ALLEGRO_PREC_FP32 || v.lmax != 2 || 2 * v.S + v.nb > 16) return 0;
  for (int w : v.dims2b) if (w != v.d) return 0;
  for (int w : v.dimsL) if (w != v.d) return 0;
  const int nl2 = (int)v.dims2b.size(), nlL = (int)v.dimsL.size();
  if (v.d == 256 && v.n == 64 && nl2 == 3 && nlL == 3) return 1;
  if (v.d == 128 && v.n == 32 && nl2 == 2 && nlL == 2) return 2;
  return 0;
}

void create_impl(AllegroModel* m, const float* w, int64_t n_weights, const double* scale, const double* shift) {
  const Validated& v = m->v;
  REQUIRE(w != nullptr, "weights is NULL");
  REQUIRE(n_weights == v.n_weights, "n_weights is " + std::to_string(n_weights) + ", expected " +
                                        std::to_string(v.n_weights));
  for (int64_t k = 0; k < n_weights; ++k) REQUIRE(std::isfinite(w[k]), "weights contain non-finite values");
  HIP_OK(hipGetDevice(&m->device));
  {
    // the static workspace of allegro_energy_forces_noalloc on this device
    REQUIRE(m->device >= 0 && m->device < kMaxDevices, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[m->device]) {
      void* p = nullptr;
      HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
      g_scratch_ptr[m->device] = p;
    }
  }
  const int n = v.n, d = v.d, LW = v.LW, L1 = v.lmax + 1;
  if (!m->rc_pair.empty()) {
    std::vector<float> rf(m->rc_pair.size());
    std::vector<double> r2(m->rc_pair.size());
    for (size_t k = 0; k < rf.size(); ++k) {
      rf[k] = (float)m->rc_pair[k];
      const double rl = m->rc_pair[k] + m->cfg.neighbor_skin;   // list radius of the pair
      r2[k] = rl * rl;
    }
    upload(m->rc_pair_f, rf.data(), rf.size() * sizeof(float));
    upload(m->rc2_pair, r2.data(), r2.size() * sizeof(double));
  }
  if (!m->znum.empty()) {
    std::vector<float> zt(2 * v.S);
    for (int k = 0; k < v.S; ++k) {
      zt[k] = (float)m->znum[k];
      zt[v.S + k] = (float)std::pow((double)m->znum[k], 0.23);
    }
    upload(m->zbl_tab, zt.data(), zt.size() * sizeof(float));
  }
  int64_t off = 0;
  // two-body MLP
  std::vector<int> dims{2 * v.S + v.nb};
  std::vector<std::vector<double>> Ws;
  for (int wd : v.dims2b) {
    Ws.push_back(slice(w, off, (int64_t)dims.back() * wd));
    dims.push_back(wd);
  }
  m->rr_cfg = rr_config(v, m->prec);
  const bool rr = m->rr_cfg != 0;
  build_mlp(m->twobody, Ws, dims, m->prec_two, m->prec_two, rr);
  const std::vector<double> embed0 = slice(w, off, (int64_t)d * LW);
  std::vector<double> env[kMaxLayers], alpha[kMaxLayers], mix[kMaxLayers];
  std::vector<std::vector<double>> mlpW[kMaxLayers];
  const int nslot = (v.parity ? 2 : 1) * L1;   // mixing matrices per layer
  for (int L = 0; L < v.nl; ++L) {
    env[L] = slice(w, off, (int64_t)d * LW);
    alpha[L] = slice(w, off, (int64_t)(v.parity ? 2 : 1) * L1 * L1 * L1);
    mix[L] = slice(w, off, (int64_t)nslot * n * n);
    int prev = d + n;
    for (int wd : v.dimsL) {
      mlpW[L].push_back(slice(w, off, (int64_t)prev * wd));
      prev = wd;
    }
  }
  const std::vector<double> We0 = slice(w, off, (int64_t)d * v.h);
  const std::vector<double> We1 = slice(w, off, (int64_t)v.h);
  const double rn = 1.0 / std::sqrt((double)n);

  // the final layer's scalar channel mixing folds into the rows of its first
  // latent-MLP matrix that read the scalar tensor features
  {
    const int L = v.nl - 1;
    const int N0 = v.dimsL[0];
    std::vector<double>& W0 = mlpW[L][0];
    if (m->cfg.channel_mix) {
      std::vector<double> folded((size_t)n * N0, 0.0);
      for (int u = 0; u < n; ++u)
        for (int vv = 0; vv < n; ++vv) {
          const double mvu = mix[L][(size_t)vv * n + u] * rn;   // mix[0][v][u]
          for (int c = 0; c < N0; ++c) folded[(size_t)u * N0 + c] += mvu * W0[(size_t)(d + vv) * N0 + c];
        }
      for (int u = 0; u < n; ++u)
        for (int c = 0; c < N0; ++c) W0[(size_t)(d + u) * N0 + c] = folded[(size_t)u * N0 + c];
    }
  }
  std::vector<int> ldims{d + n};
  for (int wd : v.dimsL) ldims.push_back(wd);
  for (int L = 0; L < v.nl; ++L) build_mlp(m->latent[L], mlpW[L], ldims, m->prec_lat_first, m->prec_lat_rest, rr);

  // heads: [embed0 | env of layer 1] after the two-body MLP, env of layer L+1
  // after latent MLP L
  {
    std::vector<double> H((size_t)d * 2 * LW);
    for (int r = 0; r < d; ++r)
      for (int c = 0; c < LW; ++c) {
        H[(size_t)r * 2 * LW + c] = embed0[(size_t)r * LW + c];
        H[(size_t)r * 2 * LW + LW + c] = env[0][(size_t)r * LW + c];
      }
    make_packed(m->head0, H, d, 2 * LW, m->prec_two);
    make_packed(m->head0T, transpose(H, d, 2 * LW), 2 * LW, d, m->prec_two);
    for (int L = 0; L + 1 < v.nl; ++L) {
      make_packed(m->envH[L], env[L + 1], d, LW, m->prec_lat_rest);
      make_packed(m->envHT[L], transpose(env[L + 1], d, LW), LW, d, m->prec_lat_rest);
    }
    if (rr) {
      std::vector<char> f, b;
      pack_rr(H.data(), d, 2 * LW, m->prec_two == 1, f);
      pack_rr_chunked(transpose(H, d, 2 * LW), 2 * LW, d, m->prec_two == 1, b);
      upload(m->rr_head0, f.data(), f.size());
      upload(m->rr_head0T, b.data(), b.size());
      for (int L = 0; L + 1 < v.nl; ++L) {
        f.clear(); b.clear();
        pack_rr(env[L + 1].data(), d, LW, m->prec_lat_rest == 1, f);
        pack_rr_chunked(transpose(env[L + 1], d, LW), LW, d, m->prec_lat_rest == 1, b);
        upload(m->rr_envH[L], f.data(), f.size());
        upload(m->rr_envHT[L], b.data(), b.size());
      }
    }
  }
  // channel mixing matrices of non-final layers (FP32): forward W[u][v] = M[v][u],
  // adjoint W[v][u] = M[v][u]
  for (int L = 0; L + 1 < v.nl; ++L) {
    std::vector<char> allF, allB;
    for (int l = 0; l < nslot; ++l) {
      std::vector<double> M(mix[L].begin() + (size_t)l * n * n, mix[L].begin() + (size_t)(l + 1) * n * n);
      std::vector<char> hf, hb;
      GemmB g;
      pack_b(transpose(M, n, n), n, n, 0, hf, g);
      pack_b(M, n, n, 0, hb, g);
      m->mix_stride = (int)(hf.size() / sizeof(float));
      allF.insert(allF.end(), hf.begin(), hf.end());
      allB.insert(allB.end(), hb.begin(), hb.end());
    }
    upload(m->mixF[L], allF.data(), allF.size());
    upload(m->mixB[L], allB.data(), allB.size());
  }
  // fused coupling tables
  for (int L = 0; L < v.nl; ++L) {
    const bool fin = L == v.nl - 1;
    std::vector<float> vals = fused_values_rt(v.lmax, v.in_kind[L], v.out_kind[L], alpha[L].data(), v.parity);
    upload(m->tpw[L], vals.data(), vals.size() * sizeof(float));
    m->tpw_host[L] = vals;
    if (fin) {
      // final pattern entries are (a, a, 0) in ascending a
      for (int k = 0; k < 16; ++k) m->tp_final[k] = k < (int)vals.size() ? vals[k] : 0.0f;
    }
  }
  // folded edge-energy vector and sigma_Z-scaled copies (the constant dE/dx^{N_l})
  std::vector<double> wev(d, 0.0);
  for (int r = 0; r < d; ++r)
    for (int k = 0; k < v.h; ++k) wev[r] += We0[(size_t)r * v.h + k] * We1[k];
  std::vector<float> wef(wev.begin(), wev.end());
  upload(m->we, wef.data(), wef.size() * sizeof(float));
  if (rr) {
    // the final latent MLP's last matrix folded with the edge-energy vector:
    // v = W_last w_e (the register-resident final-layer kernels use a . v)
    const std::vector<double>& Wl = mlpW[v.nl - 1].back();
    std::vector<float> fv(d);
    for (int r = 0; r < d; ++r) {
      double acc = 0.0;
      for (int c = 0; c < d; ++c) acc += Wl[(size_t)r * d + c] * wev[c];
      fv[r] = (float)acc;
    }
    upload(m->rr_fold_v, fv.data(), fv.size() * sizeof(float));
  }
  std::vector<double> sc(v.S, 1.0), sh(v.S, 0.0);
  for (int s = 0; s < v.S; ++s) {
    if (scale) sc[s] = scale[s];
    if (shift) sh[s] = shift[s];
    REQUIRE(std::isfinite(sc[s]) && std::isfinite(sh[s]), "species scale/shift must be finite");
  }
  std::vector<float> gc((size_t)v.S * d);
  for (int s = 0; s < v.S; ++s)
    for (int r = 0; r < d; ++r) gc[(size_t)s * d + r] = (float)(sc[s] * wev[r]);
  upload(m->gconst, gc.data(), gc.size() * sizeof(float));
  upload(m->scale, sc.data(), sc.size() * sizeof(double));
  for (int k = 0; k < v.S && k < 16; ++k) m->sigma_f[k] = (float)sc[k];
  upload(m->shift, sh.data(), sh.size() * sizeof(double));
  m->c_norm = 1.0 / std::sqrt(m->cfg.avg_num_neighbors);
  m->err_flag.ensure(sizeof(int));
  m->status.ensure(sizeof(int));
  HIP_OK(launch_fill_i32(m->status.as<int32_t>(), 0, 1, nullptr));
  HIP_OK(hipDeviceSynchronize());
  // check the MLP kernels fit in LDS for this configuration
  MlpArgs probe;
  probe.d = d; probe.n = n; probe.w = m->twobody.view(); probe.head = m->head0.g; probe.head_bwd = m->head0T.g;
  REQUIRE(mlp_lds_bytes(probe, m->prec_two, false) != (size_t)-1 &&
              mlp_lds_bytes(probe, m->prec_two, true) != (size_t)-1,
          "two-body MLP too wide for the fused kernel");
  for (int L = 0; L < v.nl; ++L) {
    MlpArgs q;
    q.d = d; q.n = n; q.w = m->latent[L].view();
    if (L + 1 < v.nl) { q.head = m->envH[L].g; q.head_bwd = m->envHT[L].g; }
    REQUIRE(mlp_lds_bytes(q, m->prec_lat, false) != (size_t)-1 &&
                mlp_lds_bytes(q, m->prec_lat, true) != (size_t)-1,
            "latent MLP too wide for the fused kernel");
  }
}

template <class T> T* ptr(const DevBuf& b, int64_t off = 0) { return b.as<T>() + off; }

void set_tpw(TensorArgs& t, const std::vector<float>& v) {
  for (size_t k = 0; k < v.size() && k < (size_t)kTpwArgs; ++k) t.tpw_v[k] = v[k];
}

// Runs `launch` and, when timing is on, brackets it with events on `s`.
template <class Fn>
void timed(AllegroModel* m, const char* name, hipStream_t s, Fn launch) {
  if (!m->timing) {
    HIP_OK(launch());
    return;
  }
  size_t k = 0;
  while (k < m->ktimes.size() && m->ktimes[k].name != name) ++k;
  if (k == m->ktimes.size()) {
    m->ktimes.push_back({});
    m->ktimes.back().name = name;
  }
  hipEvent_t a, b;
  HIP_OK(hipEventCreate(&a));
  HIP_OK(hipEventCreate(&b));
  HIP_OK(hipEventRecord(a, s));
  HIP_OK(launch());
  HIP_OK(hipEventRecord(b, s));
  m->pending.push_back({k, {a, b}});
}

void collect_times(AllegroModel* m) {
  for (auto& p : m->pending) {
    HIP_OK(hipEventSynchronize(p.second.second));
    float ms = 0.0f;
    HIP_OK(hipEventElapsedTime(&ms, p.second.first, p.second.second));
    m->ktimes[p.first].ms += ms;
    m->ktimes[p.first].launches += 1;
    (void)hipEventDestroy(p.second.first);
    (void)hipEventDestroy(p.second.second);
  }
  m->pending.clear();
}

void neighbors_impl(AllegroModel* m, int64_t n_local, int64_t n_total, const double* pos, const int32_t* species,
                    const double* cell, const int32_t* pbc, hipStream_t s, int64_t* n_edges,
                    const int64_t* sys_off = nullptr, int n_sys = 0) {
  REQUIRE(n_local >= 0 && n_total >= n_local, "need 0 <= n_local <= n_total");
  REQUIRE(pbc != nullptr, "pbc must not be NULL");
  REQUIRE((pos && species) || n_total == 0, "pos and species must not be NULL");
  REQUIRE(n_total < (int64_t)1 << 30, "at most 2^30 atoms");
  // earlier work on this stream may still use buffers that are regrown below
  HIP_OK(hipStreamSynchronize(s));
  {
    // the box of this build, for rebuilds requested later by allegro_md_run
    // (copied first: the arguments may be these very arrays)
    double cl[9] = {0};
    int32_t pl[3] = {pbc[0], pbc[1], pbc[2]};
    if (cell) std::memcpy(cl, cell, sizeof(cl));
    std::vector<int64_t> so;
    if (sys_off && n_sys > 0) so.assign(sys_off, sys_off + n_sys + 1);
    std::memcpy(m->last_cell, cl, sizeof(cl));
    std::memcpy(m->last_pbc, pl, sizeof(pl));
    m->last_has_cell = cell != nullptr;
    m->last_sys_off = std::move(so);
  }
  const double rc = m->cfg.r_cut + m->cfg.neighbor_skin;   // list radius
  double L[3];
  int pb[3];
  for (int ax = 0; ax < 3; ++ax) {
    pb[ax] = pbc[ax] ? 1 : 0;
    L[ax] = 0.0;
    if (pb[ax]) {
      REQUIRE(cell != nullptr, "cell must be given for periodic axes");
      L[ax] = cell[4 * ax];
      REQUIRE(std::isfinite(L[ax]) && L[ax] > 0, "periodic box lengths must be positive");
    }
  }
  if (cell && (pb[0] || pb[1] || pb[2]))
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c)
        if (r != c) REQUIRE(cell[3 * r + c] == 0.0, "only orthorhombic cells are supported");
  m->n_local = n_local;
  m->n_total = n_total;
  for (int ax = 0; ax < 3; ++ax) m->L[ax] = L[ax];

  NbrArgs a;
  a.n_local = n_local; a.n_total = n_total; a.pos = pos; a.r_cut2 = rc * rc;
  a.species = species; a.n_species = m->v.S;
  a.rc2_pair = m->rc_pair.empty() ? nullptr : ptr<double>(m->rc2_pair);
  for (int ax = 0; ax < 3; ++ax) { a.L[ax] = L[ax]; a.pbc[ax] = pb[ax]; }
  const int64_t nt = std::max<int64_t>(n_total, 1);
  // bounding box of the open axes
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  m->n_sys = n_sys;
  if (n_sys > 0) {
    // independent systems: each is moved (for binning only) into its own slot
    // of a cubic grid of slots wide enough that no cell holds two systems'
    // atoms within the cutoff of each other; the distance test uses the
    // original coordinates and rejects pairs from different systems
    std::vector<int64_t> off(sys_off, sys_off + n_sys + 1);
    upload(m->sys_off, off.data(), off.size() * sizeof(int64_t));
    std::vector<int32_t> sid((size_t)nt, 0);
    for (int k = 0; k < n_sys; ++k)
      for (int64_t q = off[k]; q < off[k + 1]; ++q) sid[q] = k;
    upload(m->sys_id, sid.data(), sid.size() * sizeof(int32_t));
    m->bbox.ensure((size_t)n_sys * 6 * sizeof(double));
    HIP_OK(launch_system_bbox(pos, ptr<int64_t>(m->sys_off), n_sys, ptr<double>(m->bbox), s));
    std::vector<double> bb((size_t)n_sys * 6);
    HIP_OK(hipMemcpyAsync(bb.data(), m->bbox.p, bb.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    double ext = 0.0;
    for (int k = 0; k < n_sys; ++k) {
      if (off[k + 1] == off[k]) continue;
      for (int ax = 0; ax < 3; ++ax) {
        if (!(std::isfinite(bb[6 * k + ax]) && std::isfinite(bb[6 * k + 3 + ax])))
          throw Fail{ALLEGRO_E_NONFINITE, "non-finite positions"};
        ext = std::max(ext, bb[6 * k + 3 + ax] - bb[6 * k + ax]);
      }
    }
    const double slot = ext + 2.0 * rc + 1.0;
    int G = 1;
    while ((int64_t)G * G * G < n_sys) ++G;
    std::vector<double> shift((size_t)n_sys * 3, 0.0);
    for (int k = 0; k < n_sys; ++k) {
      const int sl[3] = {k % G, (k / G) % G, k / (G * G)};
      for (int ax = 0; ax < 3; ++ax)
        shift[3 * k + ax] = (off[k + 1] > off[k]) ? sl[ax] * slot - bb[6 * k + ax] + rc : 0.0;
    }
    upload(m->sys_shift, shift.data(), shift.size() * sizeof(double));
    a.sys = ptr<int32_t>(m->sys_id);
    a.sys_shift = ptr<double>(m->sys_shift);
    for (int ax = 0; ax < 3; ++ax) { lo[ax] = 0.0; hi[ax] = G * slot; }
  } else if (n_total > 0 && (!pb[0] || !pb[1] || !pb[2])) {
    m->bbox.ensure(1024 * 6 * sizeof(double));
    a.bbox = ptr<double>(m->bbox);
    int nb = 0;
    HIP_OK(launch_bbox(a, &nb, s));
    std::vector<double> part((size_t)nb * 6);
    HIP_OK(hipMemcpyAsync(part.data(), a.bbox, part.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    for (int ax = 0; ax < 3; ++ax) { lo[ax] = 1e300; hi[ax] = -1e300; }
    for (int b = 0; b < nb; ++b)
      for (int ax = 0; ax < 3; ++ax) {
        lo[ax] = std::min(lo[ax], part[b * 6 + ax]);
        hi[ax] = std::max(hi[ax], part[b * 6 + 3 + ax]);
      }
    for (int ax = 0; ax < 3; ++ax)
      if (!pb[ax]) {
        if (!(std::isfinite(lo[ax]) && std::isfinite(hi[ax])))
          throw Fail{ALLEGRO_E_NONFINITE, "non-finite positions"};
      }
  }
  const double grow = rc * (1.0 + 1e-10) + 1e-12;
  int64_t ncell = 1;
  for (int ax = 0; ax < 3; ++ax) {
    const double span = pb[ax] ? L[ax] : (hi[ax] - lo[ax]);
    int nc = (int)std::floor(span / grow);
    nc = std::max(1, std::min(nc, 1024));
    a.nc[ax] = nc;
    a.h[ax] = pb[ax] ? L[ax] / nc : (span > 0 ? span / nc : 1.0);
    a.lo[ax] = pb[ax] ? 0.0 : lo[ax];
    // stencil half-width: every image within r_c lies within R cells
    int R = (int)std::ceil(grow / a.h[ax]);
    if (!pb[ax]) R = std::min(std::max(R, 1), nc);
    a.R[ax] = std::max(1, R);
    REQUIRE(!pb[ax] || a.R[ax] <= 64, "box too small for the cutoff (more than 64 images per axis)");
    ncell *= nc;
  }
  m->cell_of.ensure(nt * 4); m->img.ensure(nt * 12); m->cell_count.ensure((ncell + 1) * 4);
  m->cell_start.ensure((ncell + 1) * 4); m->cell_cursor.ensure((ncell + 1) * 4); m->cell_atoms.ensure(nt * 4);
  m->count.ensure(std::max<int64_t>(n_local, 1) * 4); m->row_ptr.ensure((n_local + 1) * 4);
  m->rcount.ensure(nt * 4); m->rcursor.ensure(nt * 4); m->rrow_ptr.ensure((nt + 1) * 4);
  m->scan_tmp.ensure(exclusive_scan_tmp_bytes(std::max<int64_t>(std::max(nt, ncell), n_local) + 1));
  a.cell_of = ptr<int32_t>(m->cell_of); a.img = ptr<int32_t>(m->img);
  a.cell_count = ptr<int32_t>(m->cell_count); a.cell_start = ptr<int32_t>(m->cell_start);
  a.cell_cursor = ptr<int32_t>(m->cell_cursor); a.cell_atoms = ptr<int32_t>(m->cell_atoms);
  a.count = ptr<int32_t>(m->count); a.row_ptr = ptr<int32_t>(m->row_ptr);
  a.rcount = ptr<int32_t>(m->rcount); a.rcursor = ptr<int32_t>(m->rcursor); a.rrow_ptr = ptr<int32_t>(m->rrow_ptr);
  a.scan_tmp = m->scan_tmp.p;
  int* err = ptr<int>(m->err_flag);
  HIP_OK(hipMemsetAsync(err, 0, sizeof(int), s));
  HIP_OK(launch_fill_i32(a.cell_count, 0, ncell, s));
  HIP_OK(launch_fill_i32(a.cell_cursor, 0, ncell, s));
  if (n_total > 0) HIP_OK(launch_bin_atoms_err(a, err, s));
  HIP_OK(launch_exclusive_scan(a.cell_count, a.cell_start, ncell, a.scan_tmp, s));
  if (n_total > 0) HIP_OK(launch_fill_cells(a, s));
  HIP_OK(launch_count_neighbors(a, s));
  HIP_OK(launch_exclusive_scan(a.count, a.row_ptr, n_local, a.scan_tmp, s));
  m->h_row_ptr.resize(n_local + 1);
  int herr = 0;
  HIP_OK(hipMemcpyAsync(m->h_row_ptr.data(), a.row_ptr, (n_local + 1) * 4, hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  if (herr & 2) throw Fail{ALLEGRO_E_NONFINITE, "non-finite positions"};
  if (herr & 1) throw Fail{ALLEGRO_E_INVAL, "positions lie more than 500 box lengths outside the box"};
  if (herr & 4) throw Fail{ALLEGRO_E_INVAL, "species out of range [0, n_species)"};
  // each centre's count is below 2^31, so a running sum that passes 2^31
  // shows as a decrease; the force gather indexes g_e [E][3] with int32
  for (int64_t q = 0; q < n_local; ++q)
    REQUIRE(m->h_row_ptr[q + 1] >= m->h_row_ptr[q], "more than 2^31 - 1 edges");
  const int64_t E = m->h_row_ptr[n_local];
  REQUIRE(E <= ((((int64_t)1 << 31) - 1) / 3), "more than (2^31 - 1) / 3 edges");
  m->E = E;
  // Edge capacity of the list buffers: the list plus 5 % (or the caller's
  // hint), never shrinking.  A list that fits one evaluation chunk, and has
  // not outgrown one in a device rebuild, can be rebuilt on the device
  // (allegro_md_run), within the capacity.
  {
    const int64_t hint = m->cfg.edge_capacity_hint;
    const int64_t want = hint > 0 ? std::max<int64_t>(hint, E) : E + (E + 19) / 20;
    const int64_t one_chunk = chunk_cap(m->v, m->cfg.edge_chunk);
    const int64_t floor_e = std::max<int64_t>(std::max(E, m->need_edges), 1);
    m->cap = std::max(std::max(want, m->cap), floor_e);
    m->cap = std::min<int64_t>(m->cap, ((((int64_t)1 << 31) - 1) / 3));
    m->dev_rebuild = floor_e <= one_chunk;
    if (m->dev_rebuild) m->cap = std::max(std::min(m->cap, one_chunk), floor_e);
  }
  const int64_t Ee = m->cap;
  m->ei.ensure(Ee * 4); m->ej.ensure(Ee * 4); m->es.ensure(Ee * 12); m->keys.ensure(Ee * 8);
  m->redge.ensure(Ee * 4);
  a.keys = ptr<unsigned long long>(m->keys); a.ei = ptr<int32_t>(m->ei); a.ej = ptr<int32_t>(m->ej);
  a.es = ptr<int32_t>(m->es); a.redge = ptr<int32_t>(m->redge);
  HIP_OK(launch_fill_neighbors(a, s));
  HIP_OK(launch_sort_neighbors(a, s));
  HIP_OK(launch_fill_i32(a.rcount, 0, n_total, s));
  HIP_OK(launch_fill_i32(a.rcursor, 0, n_total, s));
  HIP_OK(launch_reverse_csr(a, E, s));
  m->nbr = a;
  m->n_cells = ncell;

  // chunks of whole centres and the workspace they need
  {
    std::vector<int64_t> rp64(m->h_row_ptr.begin(), m->h_row_ptr.end());
    m->chunk_c = plan_chunks(rp64.data(), n_local, chunk_cap(m->v, m->cfg.edge_chunk));
  }
  m->Ec = 0; m->Nc = 0;
  for (size_t k = 0; k + 1 < m->chunk_c.size(); ++k) {
    const int64_t cA = m->chunk_c[k], cB = m->chunk_c[k + 1];
    m->Ec = std::max<int64_t>(m->Ec, m->h_row_ptr[cB] - m->h_row_ptr[cA]);
    m->Nc = std::max<int64_t>(m->Nc, cB - cA);
  }
  if (m->dev_rebuild) m->Ec = std::max(m->Ec, m->cap);   // device rebuilds use the whole capacity
  {
    std::vector<int32_t> crp;
    m->chunk_rp_off.clear();
    for (size_t k = 0; k + 1 < m->chunk_c.size(); ++k) {
      m->chunk_rp_off.push_back((int64_t)crp.size());
      const int64_t cA = m->chunk_c[k], cB = m->chunk_c[k + 1];
      for (int64_t q = cA; q <= cB; ++q) crp.push_back((int32_t)(m->h_row_ptr[q] - m->h_row_ptr[cA]));
    }
    if (crp.empty()) crp.push_back(0);
    upload(m->chunk_rp, crp.data(), crp.size() * sizeof(int32_t));
  }
  m->ws_bytes = ws_layout(m->v, m->Ec, m->Nc, m->cap, n_local, n_total, !m->znum.empty(),
                          m->prec != ALLEGRO_PREC_FP32, m->rr_cfg != 0, 0, nullptr);
  m->arena.ensure(m->ws_bytes);
  ws_layout(m->v, m->Ec, m->Nc, m->cap, n_local, n_total, !m->znum.empty(), m->prec != ALLEGRO_PREC_FP32,
            m->rr_cfg != 0, (uintptr_t)m->arena.p, &m->ws);
  m->pos_ref.ensure(std::max<int64_t>(n_local, 1) * 3 * sizeof(double));
  if (n_local > 0)
    HIP_OK(hipMemcpyAsync(m->pos_ref.p, pos, n_local * 3 * sizeof(double), hipMemcpyDeviceToDevice, s));
  m->nbr_version++;
  if (n_edges) *n_edges = E;
}

// dev_count: the list may have been rebuilt on the device since the host
// last saw it (in-graph MD): launch over the edge capacity, with the live
// edge count and the row pointers read on the device (single-chunk lists).
void energy_forces_impl(AllegroModel* m, const Ws& w, const double* pos, const int32_t* species,
                        double* atom_energy, double* forces, double* virial, double* atom_virial, double* energy,
                        hipStream_t s, bool dev_count = false) {
  if (m->n_local < 0) throw Fail{ALLEGRO_E_STATE, "allegro_neighbors has not been called"};
  REQUIRE((pos && species && forces) || m->n_total == 0, "pos, species and forces must not be NULL");
  const Validated& v = m->v;
  const int d = v.d, n = v.n, LW = v.LW;
  double* aE = atom_energy ? atom_energy : w.atom_e;
  const int32_t* ei = ptr<int32_t>(m->ei);
  const int32_t* ej = ptr<int32_t>(m->ej);
  const int32_t* es = ptr<int32_t>(m->es);
  if (dev_count) REQUIRE(m->dev_rebuild && m->chunk_c.size() == 2, "device-side edge count needs a single chunk");
  for (size_t k = 0; k + 1 < m->chunk_c.size(); ++k) {
    const int64_t cA = m->chunk_c[k], cB = m->chunk_c[k + 1];
    const int64_t eA = dev_count ? 0 : m->h_row_ptr[cA], eB = dev_count ? m->cap : m->h_row_ptr[cB];
    const int E = (int)(eB - eA), nc = (int)(cB - cA);
    // row pointers of the chunk's centres, relative to its first edge (the
    // list's own row pointers for a device-side count: one chunk from 0)
    const int32_t* drp = dev_count ? ptr<int32_t>(m->row_ptr) : ptr<int32_t>(m->chunk_rp) + m->chunk_rp_off[k];
    const int32_t* E_dev = dev_count ? ptr<int32_t>(m->row_ptr) + m->n_local : nullptr;

    EdgeArgs ea;
    ea.E = E; ea.E_dev = E_dev; ea.pos = pos; ea.ei = ei + eA; ea.ej = ej + eA; ea.es = es + 3 * eA; ea.species = species;
    for (int ax = 0; ax < 3; ++ax) ea.L[ax] = m->L[ax];
    ea.r_cut = m->cfg.r_cut; ea.p = v.p; ea.n_bessel = v.nb; ea.l_max = v.lmax;
    ea.rc_pair = m->rc_pair.empty() ? nullptr : ptr<float>(m->rc_pair_f); ea.n_species = v.S;
    if (!m->znum.empty()) { ea.zbl = ptr<float>(m->zbl_tab); ea.e_pair = w.epair; }
    ea.eb = w.eb;
    timed(m, "edge_basis", s, [&] { return launch_edge_basis(ea, s); });

    MlpArgs base;
    base.E = E; base.E_dev = E_dev; base.d = d; base.n = n; base.l_max = v.lmax; base.n_species = v.S; base.n_bessel = v.nb;
    base.eb = w.eb; base.ei = ei + eA; base.ej = ej + eA; base.species = species;
    base.centre_base = (int)cA;

    MlpArgs m0 = base;
    m0.kind = kTwoBody; m0.w = m->twobody.view(); m0.head = m->head0.g; m0.head_bwd = m->head0T.g;
    m0.rr = rr_view(m->twobody, m->rr_cfg, &m->rr_head0, &m->rr_head0T);
    m0.x_out = w.x[0]; m0.head_out = w.head0o;
    m0.tm = m->tm_choice[0];
    // a chain whose forward and backward both take the register-resident
    // kernels keeps its activations for the backward instead of recomputing
    auto stores = [&](MlpArgs t, int kf, int kb, int prec) {
      t.tm = m->tm_choice[kf];
      const bool f = mlp_uses_rr(t, prec);
      t.tm = m->tm_choice[kb];
      return f && mlp_uses_rr(t, prec);
    };
    if (stores(m0, 0, 5, m->prec_two)) m0.act_store = w.zst[0];
    timed(m, "mlp_fwd_twobody", s, [&] { return launch_mlp_fwd(m0, m->prec_two, s); });

    TensorArgs tb;
    tb.E = E; tb.E_dev = E_dev; tb.n_centres = nc; tb.n = n; tb.l_max = v.lmax; tb.row_ptr = drp; tb.ei = ei + eA;
    tb.centre_base = (int)cA; tb.eb = w.eb; tb.c_norm = (float)m->c_norm;
    tb.channel_mix = m->cfg.channel_mix ? 1 : 0; tb.mix_scale = (float)(1.0 / std::sqrt((double)n));
    tb.mix_bf3 = m->prec != ALLEGRO_PREC_FP32 ? 1 : 0;   // BF16 modes: mixing as BF16 x 3
    tb.mix_stride = m->mix_stride;

    TensorArgs t1 = tb;
    t1.w_env = w.head0o + LW; t1.ld_w = 2 * LW; t1.gam = w.gam[0];
    timed(m, "env", s, [&] { return launch_env(t1, s); });

    const VSrc v_a0{w.head0o, 2 * LW, 1};
    MlpArgs mf = base;
    mf.kind = kLatentFinal; mf.we = ptr<float>(m->we); mf.g_const = ptr<float>(m->gconst);
    mf.rr = rr_view(m->latent[v.nl - 1], m->rr_cfg, nullptr, nullptr);
    mf.fold_v = m->rr_cfg ? ptr<float>(m->rr_fold_v) : nullptr;
    for (int k = 0; k < v.S && k < 16; ++k) mf.sigma[k] = m->sigma_f[k];
    for (int k = 0; k < 16; ++k) mf.tp_w[k] = m->tp_final[k];
    mf.eij = w.eij;
    // non-final layers: tensor product + mixing, then the latent MLP that
    // produces the next layer's scalars and environment weights
    MlpArgs ml[kMaxLayers];
    VSrc vin = v_a0;
    for (int L = 0; L + 1 < v.nl; ++L) {
      TensorArgs tl = tb;
      tl.in_kind = v.in_kind[L]; tl.out_kind = v.out_kind[L];
      tl.v = vin; tl.gam = w.gam[L]; tl.tile = m->tt_choice[0];
      tl.tpw = ptr<float>(m->tpw[L]); set_tpw(tl, m->tpw_host[L]); tl.mixB = m->mixF[L].p;
      tl.v_out = w.V[L];
      timed(m, "tp_mix", s, [&] { return launch_tp_mix(tl, false, s); });
      MlpArgs& mL = ml[L];
      mL = base;
      mL.kind = kLatent; mL.w = m->latent[L].view(); mL.head = m->envH[L].g; mL.head_bwd = m->envHT[L].g;
      mL.rr = rr_view(m->latent[L], m->rr_cfg, &m->rr_envH[L], &m->rr_envHT[L]);
      mL.x_prev = w.x[L]; mL.s_in = w.V[L]; mL.s_ld = v.w_out[L] * n;
      mL.x_out = w.x[L + 1]; mL.head_out = w.wenv[L + 1];
      mL.tm = m->tm_choice[1];
      if (stores(mL, 1, 4, m->prec_lat)) mL.act_store = w.zst[1 + L];
      timed(m, "mlp_fwd_latent", s, [&] { return launch_mlp_fwd(mL, m->prec_lat, s); });
      TensorArgs te = tb;
      te.w_env = w.wenv[L + 1]; te.ld_w = LW; te.gam = w.gam[L + 1];
      timed(m, "env", s, [&] { return launch_env(te, s); });
      vin = VSrc{w.V[L], v.w_out[L] * n, 0};
    }
    mf.w = m->latent[v.nl - 1].view(); mf.x_prev = w.x[v.nl - 1]; mf.tp_v = vin;
    mf.tp_gam = w.gam[v.nl - 1];
    mf.tm = m->tm_choice[2];
    mf.tp_out = w.gTf;   // the final scalars, read back by the backward pass
    if (stores(mf, 2, 3, m->prec_lat)) {
      mf.act_store = w.zst[v.nl];
      mf.av_store = w.av;
    }
    timed(m, "mlp_fwd_final", s, [&] { return launch_mlp_fwd(mf, m->prec_lat, s); });

    ReduceArgs ra;
    ra.n_centres = nc; ra.centre_base = (int)cA; ra.row_ptr = drp; ra.eij = w.eij;
    ra.e_pair = m->znum.empty() ? nullptr : w.epair;
    ra.species = species; ra.n_species = v.S;
    ra.scale = ptr<double>(m->scale); ra.shift = ptr<double>(m->shift); ra.atom_energy = aE;
    timed(m, "atom_energy", s, [&] { return launch_atom_energy(ra, s); });

    // ---- adjoint ----
    // the backward reads each row's stored scalars before overwriting them with dE/ds
    mf.tp_out = nullptr; mf.s_in = w.gTf; mf.s_ld = n;
    mf.g_xprev = w.gxa; mf.g_s = w.gTf; mf.g_u = w.gu; mf.gu_accum = 0;
    mf.g_store = mf.g_xprev; mf.act_scratch = w.zscr;
    mf.tm = m->tm_choice[3];
    timed(m, "mlp_bwd_final", s, [&] { return launch_mlp_bwd(mf, m->prec_lat, s); });

    TensorArgs tf = tb;
    tf.g_t = w.gTf; tf.g_Y = w.gY; tf.gy_accum = 0; tf.g_gam = w.ggam;
    tf.tpw = ptr<float>(m->tpw[v.nl - 1]);
    set_tpw(tf, m->tpw_host[v.nl - 1]);
    tf.v = vin; tf.gam = w.gam[v.nl - 1];
    if (v.nl >= 2) {
      tf.w_env = w.wenv[v.nl - 1]; tf.ld_w = LW; tf.g_w = w.gw2; tf.ld_gw = LW;
    } else {
      tf.w_env = w.head0o + LW; tf.ld_w = 2 * LW;
      tf.g_w = w.ghead0 + LW; tf.ld_gw = 2 * LW; tf.g_a0 = w.ghead0;
    }
    timed(m, "tp_env_adjoint_final", s, [&] { return launch_tp_env_adjoint(tf, true, s); });

    // non-final layers, last to first: latent-MLP adjoint (dE/dx of the layer's
    // input, dE/ds of its scalars), mixing adjoint (dE/dT from the next layer),
    // tensor-product / environment adjoint (dE/dw of its environment weights)
    float* gx_cur = w.gxa;     // dE/dx of the input of layer L+1
    float* gx_other = w.gxb;
    const float* gt_next = w.gTf;
    int slot = 0;
    for (int L = v.nl - 2; L >= 0; --L) {
      MlpArgs& mL = ml[L];
      mL.g_head = w.gw2; mL.g_x = gx_cur; mL.g_xprev = gx_other;
      mL.g_s = w.gs; mL.g_u = w.gu; mL.gu_accum = 1;
      mL.g_store = mL.g_xprev; mL.act_scratch = w.zscr;
      mL.tm = m->tm_choice[4];
      timed(m, "mlp_bwd_latent", s, [&] { return launch_mlp_bwd(mL, m->prec_lat, s); });
      std::swap(gx_cur, gx_other);
      TensorArgs tm = tb;
      tm.next_in = v.in_kind[L + 1]; tm.next_out = v.out_kind[L + 1];
      tm.g_tnext = gt_next; tm.gam_next = w.gam[L + 1];
      for (int k = 0; k < 16; ++k) tm.tp_wnext[k] = m->tp_final[k];
      tm.tpw = ptr<float>(m->tpw[L + 1]); set_tpw(tm, m->tpw_host[L + 1]);
      tm.g_s = w.gs; tm.tile = m->tt_choice[1]; tm.mixB = m->mixB[L].p;
      tm.g_tout = w.gT[slot];
      timed(m, "mix_adjoint", s, [&] { return launch_mix_adjoint(tm, s); });
      TensorArgs tl = tb;
      tl.in_kind = v.in_kind[L]; tl.out_kind = v.out_kind[L];
      tl.g_t = w.gT[slot]; tl.tpw = ptr<float>(m->tpw[L]); set_tpw(tl, m->tpw_host[L]);
      tl.g_Y = w.gY; tl.gy_accum = 1; tl.g_gam = w.ggam;
      tl.gam = w.gam[L];
      if (L == 0) {
        tl.v = v_a0; tl.w_env = w.head0o + LW; tl.ld_w = 2 * LW;
        tl.g_w = w.ghead0 + LW; tl.ld_gw = 2 * LW; tl.g_a0 = w.ghead0;
      } else {
        tl.v = VSrc{w.V[L - 1], v.w_out[L - 1] * n, 0};
        tl.w_env = w.wenv[L]; tl.ld_w = LW; tl.g_w = w.gw2; tl.ld_gw = LW;
      }
      timed(m, "tp_env_adjoint", s, [&] { return launch_tp_env_adjoint(tl, false, s); });
      gt_next = w.gT[slot];
      slot ^= 1;
    }
    float* gx_two = gx_cur;
    m0.g_head = w.ghead0; m0.g_x = gx_two; m0.g_u = w.gu; m0.gu_accum = 1;
    m0.g_R = w.gR;
    m0.g_store = gx_two; m0.act_scratch = w.zscr;   // the two-body backward reuses its g_x rows
    m0.tm = m->tm_choice[5];
    timed(m, "mlp_bwd_twobody", s, [&] { return launch_mlp_bwd(m0, m->prec_two, s); });

    ea.g_Y = w.gY; ea.g_R = w.gR; ea.g_u = w.gu;
    ea.g_e = w.g_e + 3 * eA;
    timed(m, "edge_adjoint", s, [&] { return launch_edge_adjoint(ea, s); });
  }
  ForceArgs fa;
  fa.n_total = m->n_total; fa.n_local = m->n_local; fa.pos = pos; fa.row_ptr = ptr<int32_t>(m->row_ptr);
  fa.rrow_ptr = ptr<int32_t>(m->rrow_ptr); fa.redge = ptr<int32_t>(m->redge); fa.ei = ei; fa.ej = ej; fa.es = es;
  for (int ax = 0; ax < 3; ++ax) fa.L[ax] = m->L[ax];
  fa.g_e = w.g_e; fa.forces = forces; fa.atom_virial = atom_virial;
  fa.partial = w.partial; fa.atom_energy = aE; fa.status = ptr<int>(m->status);
  int nb = 0;
  timed(m, "forces", s, [&] { return launch_forces(fa, &nb, s); });
  if (virial || energy) timed(m, "final_sums", s, [&] { return launch_final_sums(fa.partial, nb, virial, energy, s); });
}

// Synchronises `s`, reads and clears the sticky device status and turns it
// into a status code.
int take_status(AllegroModel* m, hipStream_t s) {
  int h = 0;
  HIP_OK(hipMemcpyAsync(&h, m->status.p, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  if (h == 0) return ALLEGRO_OK;
  HIP_OK(launch_fill_i32(ptr<int32_t>(m->status), 0, 1, s));
  HIP_OK(hipStreamSynchronize(s));
  if (h & kStatusNonFinite) {
    m->err = "a previous evaluation produced non-finite energies or forces";
    return ALLEGRO_E_NONFINITE;
  }
  return ALLEGRO_OK;
}

void release_graph(AllegroModel* m) {
  if (m->md_exec) (void)hipGraphExecDestroy(m->md_exec);
  if (m->md_graph) (void)hipGraphDestroy(m->md_graph);
  m->md_exec = nullptr;
  m->md_graph = nullptr;
  m->md_key.clear();
}

// Neighbour-list rebuild inside an MD step, on the device (single-chunk
// lists): every kernel runs only when some centre moved more than half the
// skin since the last build (flags[kFlagRebuild]).  The list keeps the cell
// grid and buffers of the last host build and holds at most m->cap edges; a
// rebuild that needs more sets kFlagHalt and clamps the row pointers to the
// capacity, so that the rest of the step stays in bounds (allegro_md_run then
// discards it).
void device_rebuild(AllegroModel* m, const double* pos, const int32_t* species, hipStream_t s) {
  int32_t* flags = ptr<int32_t>(m->md_flags);
  NbrArgs a = m->nbr;
  a.pos = pos;
  a.species = species;
  a.pred = flags + kFlagRebuild;
  const double half = 0.5 * m->cfg.neighbor_skin;
  HIP_OK(launch_fill_i32(flags + kFlagRebuild, 0, 1, s));
  HIP_OK(launch_disp_check(m->n_local, pos, ptr<double>(m->pos_ref), half * half, flags, s));
  HIP_OK(launch_fill_i32(a.cell_count, 0, m->n_cells, s));
  HIP_OK(launch_fill_i32(a.cell_cursor, 0, m->n_cells, s));
  HIP_OK(launch_fill_i32(a.rcount, 0, m->n_total, s));
  HIP_OK(launch_fill_i32(a.rcursor, 0, m->n_total, s));
  if (m->n_total > 0) HIP_OK(launch_bin_atoms_err(a, ptr<int>(m->err_flag), s));
  HIP_OK(launch_exclusive_scan(a.cell_count, a.cell_start, m->n_cells, a.scan_tmp, s, a.pred));
  if (m->n_total > 0) HIP_OK(launch_fill_cells(a, s));
  HIP_OK(launch_count_neighbors(a, s));
  HIP_OK(launch_exclusive_scan(a.count, a.row_ptr, m->n_local, a.scan_tmp, s, a.pred));
  HIP_OK(launch_capacity_check(a.row_ptr, m->n_local, m->cap, flags, ptr<int>(m->status), s));
  HIP_OK(launch_fill_neighbors(a, s));
  HIP_OK(launch_sort_neighbors(a, s));
  HIP_OK(launch_reverse_csr(a, m->cap, s));
  HIP_OK(launch_copy_f64_flag(ptr<double>(m->pos_ref), pos, m->n_local * 3, flags, kFlagRebuild, 1, s));
}

// The last host build's box and systems, for rebuilds at new positions.
void host_rebuild(AllegroModel* m, const double* pos, const int32_t* species, hipStream_t s) {
  const std::vector<int64_t> so = m->last_sys_off;
  double cl[9];
  int32_t pl[3];
  std::memcpy(cl, m->last_cell, sizeof(cl));
  std::memcpy(pl, m->last_pbc, sizeof(pl));
  neighbors_impl(m, m->n_local, m->n_total, pos, species, m->last_has_cell ? cl : nullptr, pl, s, nullptr,
                 so.empty() ? nullptr : so.data(), so.empty() ? 0 : (int)so.size() - 1);
}

// Lists evaluated in several chunks cannot be rebuilt on the device: the host
// checks the displacement and rebuilds (eager steps only).
void host_rebuild_if_needed(AllegroModel* m, const double* pos, const int32_t* species, hipStream_t s) {
  int nb = 0;
  HIP_OK(launch_max_disp(m->n_local, pos, ptr<double>(m->pos_ref), ptr<double>(m->md_part), &nb, s));
  std::vector<double> part(nb);
  HIP_OK(hipMemcpyAsync(part.data(), m->md_part.p, nb * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  double mx = 0.0;
  for (double v : part) mx = std::max(mx, v);
  const double half = 0.5 * m->cfg.neighbor_skin;
  if (!(mx <= half * half)) {
    host_rebuild(m, pos, species, s);
    m->last_run_rebuilds++;
  }
}

// One velocity-Verlet step; dev: the list is rebuilt on the device when needed
// and the state at the start of the step is kept until a rebuild overflows.
void md_step(AllegroModel* m, double dt, const double* masses, double* pos, double* vel, double* forces,
             const int32_t* species, bool dev, bool want_virial, hipStream_t s) {
  const int64_t nl = m->n_local, nt = m->n_total;
  int32_t* flags = ptr<int32_t>(m->md_flags);
  if (dev) {
    HIP_OK(launch_copy_f64_flag(ptr<double>(m->bak_pos), pos, nt * 3, flags, kFlagHalt, 0, s));
    HIP_OK(launch_copy_f64_flag(ptr<double>(m->bak_vel), vel, nl * 3, flags, kFlagHalt, 0, s));
    HIP_OK(launch_copy_f64_flag(ptr<double>(m->bak_f), forces, nt * 3, flags, kFlagHalt, 0, s));
  }
  HIP_OK(launch_kick_drift(nl, dt, masses, pos, vel, forces, s));
  if (m->n_ghost > 0)
    HIP_OK(launch_ghost_refresh(m->n_ghost, nl, ptr<int32_t>(m->g_owner), ptr<double>(m->g_offset), pos, s));
  if (dev) device_rebuild(m, pos, species, s);
  else host_rebuild_if_needed(m, pos, species, s);
  double* vir = want_virial ? ptr<double>(m->md_vir) : nullptr;
  energy_forces_impl(m, m->ws, pos, species, ptr<double>(m->md_atom_e), forces, vir, nullptr,
                     ptr<double>(m->md_epot), s, dev);
  if (m->n_ghost > 0) HIP_OK(launch_fold(nl, ptr<int32_t>(m->g_ptr), ptr<int32_t>(m->g_idx), forces, s));
  HIP_OK(launch_kick(nl, dt, masses, vel, forces, s));
  HIP_OK(launch_thermo(nl, masses, vel, ptr<double>(m->md_part), ptr<double>(m->md_epot), vir,
                       ptr<ThermoTarget>(m->md_counter), s));
  if (dev) HIP_OK(launch_step_done(flags, s));
}

void md_run_impl(AllegroModel* m, int n_steps, double dt, const double* masses, double* pos, double* vel,
                 double* forces, const int32_t* species, double* thermo, double* virial, int init_forces,
                 int use_graph,
                 hipStream_t s, double* max_disp, int32_t* steps_done) {
  if (steps_done) *steps_done = 0;
  if (m->n_local < 0) throw Fail{ALLEGRO_E_STATE, "allegro_neighbors has not been called"};
  REQUIRE(n_steps >= 0 && std::isfinite(dt) && dt > 0, "need n_steps >= 0 and dt > 0");
  REQUIRE(m->n_sys == 0 || m->n_ghost == 0, "ghost images are not used with batched systems");
  REQUIRE(m->n_ghost == 0 || (m->ghost_n_local == m->n_local && m->n_local + m->n_ghost == m->n_total),
          "ghost description does not match the neighbour list");
  REQUIRE((masses && pos && vel && forces && species) || m->n_total == 0, "NULL array");
  const int64_t nl = m->n_local, nt = m->n_total;
  const bool dev = m->dev_rebuild;
  m->md_epot.ensure(sizeof(double));
  m->md_counter.ensure(sizeof(ThermoTarget));
  m->md_vir.ensure(9 * sizeof(double));
  const bool want_virial = virial != nullptr;
  m->md_part.ensure(((std::max<int64_t>(nl, 1) + 255) / 256) * sizeof(double));
  m->md_atom_e.ensure(std::max<int64_t>(nl, 1) * sizeof(double));
  m->md_flags.ensure(kNumFlags * sizeof(int32_t));
  if (dev) {
    m->bak_pos.ensure(std::max<int64_t>(nt, 1) * 3 * sizeof(double));
    m->bak_vel.ensure(std::max<int64_t>(nl, 1) * 3 * sizeof(double));
    m->bak_f.ensure(std::max<int64_t>(nt, 1) * 3 * sizeof(double));
  }
  int32_t* flags = ptr<int32_t>(m->md_flags);
  const bool was_timing = m->timing;
  m->timing = false;
  m->last_run_rebuilds = 0;
  if (init_forces) {
    energy_forces_impl(m, m->ws, pos, species, ptr<double>(m->md_atom_e), forces, nullptr, nullptr, ptr<double>(m->md_epot), s);
    if (m->n_ghost > 0) HIP_OK(launch_fold(nl, ptr<int32_t>(m->g_ptr), ptr<int32_t>(m->g_idx), forces, s));
  }
  HIP_OK(launch_set_thermo(ptr<ThermoTarget>(m->md_counter), thermo, virial, n_steps, s));
  HIP_OK(launch_fill_i32(flags, 0, kNumFlags, s));
  if (use_graph && dev && n_steps > 0) {
    // one step, neighbour rebuild included, captured once per list layout and
    // state arrays and replayed n_steps times (the step count and the thermo
    // rows are read from device memory, so they do not enter the key)
    uint64_t dt_bits;
    std::memcpy(&dt_bits, &dt, sizeof(dt_bits));
    const std::vector<uintptr_t> key{(uintptr_t)pos, (uintptr_t)vel, (uintptr_t)forces, (uintptr_t)masses,
                                     (uintptr_t)species, (uintptr_t)m->nbr_version, (uintptr_t)dt_bits,
                                     (uintptr_t)m->md_flags.p, (uintptr_t)m->md_counter.p,
                                     (uintptr_t)m->bak_pos.p, (uintptr_t)m->bak_vel.p, (uintptr_t)m->bak_f.p,
                                     (uintptr_t)m->md_part.p, (uintptr_t)m->md_atom_e.p, (uintptr_t)m->md_vir.p,
                                     (uintptr_t)want_virial};
    if (!m->md_stream) HIP_OK(hipStreamCreateWithFlags(&m->md_stream, hipStreamNonBlocking));
    if (!m->md_ev[0]) {
      HIP_OK(hipEventCreateWithFlags(&m->md_ev[0], hipEventDisableTiming));
      HIP_OK(hipEventCreateWithFlags(&m->md_ev[1], hipEventDisableTiming));
    }
    HIP_OK(hipEventRecord(m->md_ev[0], s));
    HIP_OK(hipStreamWaitEvent(m->md_stream, m->md_ev[0], 0));
    if (!m->md_exec || m->md_key != key) {
      release_graph(m);
      HIP_OK(hipStreamBeginCapture(m->md_stream, hipStreamCaptureModeRelaxed));
      try {
        md_step(m, dt, masses, pos, vel, forces, species, true, want_virial, m->md_stream);
      } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(m->md_stream, &g);
        if (g) (void)hipGraphDestroy(g);
        m->timing = was_timing;
        throw;
      }
      HIP_OK(hipStreamEndCapture(m->md_stream, &m->md_graph));
      HIP_OK(hipGraphInstantiate(&m->md_exec, m->md_graph, nullptr, nullptr, 0));
      m->md_key = key;
      m->graph_captures++;
    }
    for (int k = 0; k < n_steps; ++k) HIP_OK(hipGraphLaunch(m->md_exec, m->md_stream));
    HIP_OK(hipEventRecord(m->md_ev[1], m->md_stream));
    HIP_OK(hipStreamWaitEvent(s, m->md_ev[1], 0));
  } else {
    for (int k = 0; k < n_steps; ++k) md_step(m, dt, masses, pos, vel, forces, species, dev, want_virial, s);
  }
  m->timing = was_timing;
  int32_t done = n_steps;
  if (dev) {
    int32_t hf[kNumFlags];
    HIP_OK(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (!hf[kFlagHalt] && n_steps > 0) {
      // the host's view of the list (edge count, the single chunk's row
      // pointers) follows the device-side rebuilds
      m->h_row_ptr.resize(nl + 1);
      HIP_OK(hipMemcpyAsync(m->h_row_ptr.data(), m->row_ptr.p, (nl + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
      if (nl > 0)
        HIP_OK(hipMemcpyAsync(m->chunk_rp.p, m->row_ptr.p, (nl + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
      HIP_OK(hipStreamSynchronize(s));
      m->E = m->h_row_ptr[nl];
    }
    m->last_run_rebuilds = hf[kFlagBuilds];
    if (hf[kFlagHalt]) {
      // a rebuild needed more edges than the capacity: back to the state at
      // the start of that step, a larger capacity, and a list built there
      done = hf[kFlagSteps];
      HIP_OK(launch_copy_f64_flag(pos, ptr<double>(m->bak_pos), nt * 3, flags, kFlagHalt, 1, s));
      HIP_OK(launch_copy_f64_flag(vel, ptr<double>(m->bak_vel), nl * 3, flags, kFlagHalt, 1, s));
      HIP_OK(launch_copy_f64_flag(forces, ptr<double>(m->bak_f), nt * 3, flags, kFlagHalt, 1, s));
      const int64_t need = hf[kFlagNeed];
      m->need_edges = std::max(m->need_edges, need);
      m->cap = std::max<int64_t>(m->cap, need + (need + 19) / 20);
      host_rebuild(m, pos, species, s);
      (void)take_status(m, s);   // the discarded steps' records
      // the next step rebuilds the list at its drifted positions, as the
      // overflowing step did, so that a resumed run follows the same lists
      if (nl > 0) {
        const std::vector<double> far(nl * 3, 1e30);
        HIP_OK(hipMemcpyAsync(m->pos_ref.p, far.data(), nl * 3 * sizeof(double), hipMemcpyHostToDevice, s));
        HIP_OK(hipStreamSynchronize(s));
      }
      if (steps_done) *steps_done = done;
      throw Fail{ALLEGRO_E_CAPACITY, "a neighbour rebuild needed " + std::to_string(need) +
                                         " edges, more than the capacity; regrown to " + std::to_string(m->cap) +
                                         " after " + std::to_string(done) + " steps"};
    }
  }
  if (steps_done) *steps_done = done;
  if (max_disp) {
    int nb = 0;
    HIP_OK(launch_max_disp(nl, pos, ptr<double>(m->pos_ref), ptr<double>(m->md_part), &nb, s));
    std::vector<double> part(nb);
    HIP_OK(hipMemcpyAsync(part.data(), m->md_part.p, nb * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    double mx = 0.0;
    for (double v : part) mx = std::max(mx, v);
    *max_disp = std::sqrt(mx);
  }
  const int st = take_status(m, s);
  if (st != ALLEGRO_OK) throw Fail{st, m->err};
}

const char* const kTuneNames[8] = {"mlp_fwd_twobody", "mlp_fwd_latent", "mlp_fwd_final", "mlp_bwd_final",
                                   "mlp_bwd_latent", "mlp_bwd_twobody", "tp_mix", "mix_adjoint"};

// Times every candidate tile shape on the current neighbour list and keeps the
// fastest per kernel kind.
void autotune_impl(AllegroModel* m, const double* pos, const int32_t* species, hipStream_t s, int32_t* choices) {
  if (m->n_local < 0) throw Fail{ALLEGRO_E_STATE, "allegro_neighbors has not been called"};
  REQUIRE((pos && species) || m->n_total == 0, "pos and species must not be NULL");
  // MLP tile rows: BF16 {256 (register-resident kernels, where compiled),
  // 128 (tall tiles), 64, 32}, FP32 {32, 16}; tensor tiles {32, 16} (tried
  // with the first two MLP candidates)
  int cand_tm[4], ntm = 0;
  if (m->prec && m->rr_cfg) cand_tm[ntm++] = kRRTile;
  if (m->prec) { cand_tm[ntm++] = 128; cand_tm[ntm++] = 64; cand_tm[ntm++] = 32; }
  else { cand_tm[ntm++] = 32; cand_tm[ntm++] = 16; }
  const int cand_tt[2] = {32, 16};
  m->tune_forces.ensure(std::max<int64_t>(m->n_total, 1) * 3 * sizeof(double));
  m->md_epot.ensure(sizeof(double));
  double tk[4][8];   // [candidate][kind]: summed kernel ms of two evaluations
  for (int c = 0; c < 4; ++c)
    for (int k = 0; k < 8; ++k) tk[c][k] = 1e300;
  const bool was = m->timing;
  for (int c = 0; c < ntm; ++c) {
    for (int k = 0; k < 6; ++k) m->tm_choice[k] = cand_tm[c];
    for (int k = 0; k < 2; ++k) m->tt_choice[k] = cand_tt[c < 2 ? c : 1];
    // warm-up, then two timed evaluations
    m->timing = false;
    energy_forces_impl(m, m->ws, pos, species, nullptr, ptr<double>(m->tune_forces), nullptr, nullptr,
                       ptr<double>(m->md_epot), s);
    collect_times(m);
    m->ktimes.clear();
    m->timing = true;
    for (int r = 0; r < 2; ++r)
      energy_forces_impl(m, m->ws, pos, species, nullptr, ptr<double>(m->tune_forces), nullptr, nullptr,
                         ptr<double>(m->md_epot), s);
    collect_times(m);
    for (int k = 0; k < 8; ++k)
      for (const auto& kt : m->ktimes)
        if (kt.name == kTuneNames[k] && (k < 6 || c < 2)) tk[c][k] = std::min(tk[c][k], kt.ms);
    m->ktimes.clear();
  }
  m->timing = was;
  int pick[8];
  // MLP chains as (forward, backward) pairs: register-resident in both
  // directions (the forward then stores the activations the backward reads;
  // that is how the register-resident candidate was timed), or the fastest
  // other tile in each direction
  const int pairs[3][2] = {{0, 5}, {1, 4}, {2, 3}};
  for (const auto& pr : pairs) {
    double rr_cost = 1e300, other[2] = {1e300, 1e300};
    int other_pick[2] = {0, 0};
    for (int c = 0; c < ntm; ++c) {
      if (cand_tm[c] == kRRTile) {
        rr_cost = tk[c][pr[0]] + tk[c][pr[1]];
        continue;
      }
      for (int d = 0; d < 2; ++d)
        if (tk[c][pr[d]] < other[d]) { other[d] = tk[c][pr[d]]; other_pick[d] = cand_tm[c]; }
    }
    const bool rr = rr_cost < 1e299 && rr_cost <= other[0] + other[1];
    for (int d = 0; d < 2; ++d) pick[pr[d]] = rr ? kRRTile : other_pick[d];
  }
  for (int k = 6; k < 8; ++k) {
    pick[k] = cand_tt[0];
    for (int c = 1; c < 2; ++c)
      if (tk[c][k] < tk[0][k]) pick[k] = cand_tt[c];
  }
  for (int k = 0; k < 6; ++k) m->tm_choice[k] = pick[k];
  for (int k = 0; k < 2; ++k) m->tt_choice[k] = pick[6 + k];
  release_graph(m);
  if (choices)
    for (int k = 0; k < 8; ++k) choices[k] = pick[k];
}

}  // namespace

extern "C" {

int allegro_set_tiles(AllegroModel* m, const int32_t* tiles) {
  if (!m) return ALLEGRO_E_INVAL;
  try {
    REQUIRE(tiles != nullptr, "tiles is NULL");
    for (int k = 0; k < 6; ++k) {
      const int t = tiles[k];
      const bool ok = t == 0 || (m->prec ? (t == 128 || t == 64 || t == 32 || (t == kRRTile && m->rr_cfg))
                                         : (t == 32 || t == 16));
      REQUIRE(ok, std::string("tile rows ") + std::to_string(t) + " not available for " + kTuneNames[k]);
    }
    for (int k = 6; k < 8; ++k)
      REQUIRE(tiles[k] == 0 || tiles[k] == 16 || tiles[k] == 32,
              std::string("tile rows ") + std::to_string(tiles[k]) + " not available for " + kTuneNames[k]);
    for (int k = 0; k < 6; ++k) m->tm_choice[k] = tiles[k];
    for (int k = 0; k < 2; ++k) m->tt_choice[k] = tiles[6 + k];
    release_graph(m);
    return ALLEGRO_OK;
  } catch (const Fail& f) {
    return fail(m, f);
  }
}

int allegro_autotune(AllegroModel* m, const double* pos, const int32_t* species, void* stream, int32_t* choices) {
  if (!m) return ALLEGRO_E_INVAL;
  try {
    autotune_impl(m, pos, species, (hipStream_t)stream, choices);
    return ALLEGRO_OK;
  } catch (const Fail& f) {
    return fail(m, f);
  } catch (...) {
    return fail(m, Fail{ALLEGRO_E_INVAL, "unexpected exception"});
  }
}

int allegro_set_ghosts(AllegroModel* m, int64_t n_local, int64_t n_ghost, const int32_t* owner,
                       const double* offset) {
  if (!m) return ALLEGRO_E_INVAL;
  try {
    REQUIRE(n_local >= 0 && n_ghost >= 0, "negative count");
    REQUIRE(n_ghost == 0 || (owner && offset), "owner and offset must not be NULL");
    std::vector<int32_t> gptr(n_local + 1, 0), gidx(std::max<int64_t>(n_ghost, 1), 0);
    for (int64_t g = 0; g < n_ghost; ++g) {
      REQUIRE(owner[g] >= 0 && owner[g] < n_local, "ghost owner out of range");
      REQUIRE(std::isfinite(offset[3 * g]) && std::isfinite(offset[3 * g + 1]) && std::isfinite(offset[3 * g + 2]),
              "non-finite ghost offset");
      gptr[owner[g] + 1]++;
    }
    for (int64_t o = 0; o < n_local; ++o) gptr[o + 1] += gptr[o];
    std::vector<int32_t> fill(gptr.begin(), gptr.end() - 1);
    for (int64_t g = 0; g < n_ghost; ++g) gidx[fill[owner[g]]++] = (int32_t)g;
    upload(m->g_ptr, gptr.data(), gptr.size() * sizeof(int32_t));
    upload(m->g_idx, gidx.data(), gidx.size() * sizeof(int32_t));
    if (n_ghost > 0) {
      upload(m->g_owner, owner, n_ghost * sizeof(int32_t));
      upload(m->g_offset, offset, n_ghost * 3 * sizeof(double));
    }
    m->n_ghost = n_ghost;
    m->ghost_n_local = n_local;
    release_graph(m);
    return ALLEGRO_OK;
  } catch (const Fail& f) {
    return fail(m, f);
  } catch (...) {
    return fail(m, Fail{ALLEGRO_E_INVAL, "unexpected exception"});
  }
}

int allegro_md_run(AllegroModel* m, int32_t n_steps, double dt_fs, const double* masses, double* pos, double* vel,
                   double* forces, const int32_t* species, double* thermo, double* virial, int32_t init_forces,
                   int32_t use_graph, void* stream, double* max_disp, int32_t* steps_done) {
  if (!m) return ALLEGRO_E_INVAL;
  try {
    md_run_impl(m, n_steps, dt_fs, masses, pos, vel, forces, species, thermo, virial, init_forces, use_graph,
                (hipStream_t)stream, max_disp, steps_done);
    return ALLEGRO_OK;
  } catch (const Fail& f) {
    return fail(m, f);
  } catch (...) {
    return fail(m, Fail{ALLEGRO_E_INVAL, "unexpected exception"});
  }
}


int allegro_md_stats(const AllegroModel* m, int64_t* graph_captures, int64_t* edge_capacity, int32_t* device_rebuild,
                     int64_t* last_run_rebuilds) {
  if (!m) return ALLEGRO_E_INVAL;
  if (last_run_rebuilds) *last_run_rebuilds = m->last_run_rebuilds;
  if (graph_captures) *graph_captures = m->graph_captures;
  if (edge_capacity) *edge_capacity = m->cap;
  if (device_rebuild) *device_rebuild = m->dev_rebuild ? 1 : 0;
  return ALLEGRO_OK;
}

int allegro_describe(const AllegroConfig* cfg, AllegroInfo* info) {
  try {
    const Validated v = validate(cfg);
    if (info) {
      info->n_weights = v.n_weights;
      info->dim = v.dim;
      info->latent = v.d;
      info->widest_row = (int32_t)widest_row(v);
      info->max_chunk_edges = max_chunk_edges(v);
      for (int L = 0; L < kMaxLayers; ++L) {
        info->n_paths[L] = 0;
        info->n_nonzero[L] = 0;
        info->width[L] = 0;
      }
      for (int L = 0; L < v.nl; ++L) {
        info->n_paths[L] = count_paths(v.lmax, v.in_kind[L], v.out_kind[L]);
        info->n_nonzero[L] = count_nonzeros(v.lmax, v.in_kind[L], v.out_kind[L]);
        info->width[L] = v.w_out[L];
      }
    }
    return ALLEGRO_OK;
  } catch (const Fail& f) {
    return fail(nullptr, f);
  } catch (...) {
    return fail(nullptr, Fail{ALLEGRO_E_INVAL, "unexpected exception"});
  }
}

int allegro_plan_chunks(const AllegroConfig* cfg, int64_t n_centres, const int32_t* edges_per_centre,
                        int64_t max_bounds, int64_t* bounds, int64_t* n_chunks) {
  try {
    const Validated v = validate(cfg);
    REQUIRE(n_centres >= 0 && (edges_per_centre || n_centres == 0), "need n_centres >= 0 and edge counts");
    std::vector<int64_t> rp((size_t)n_centres + 1, 0);
    for (int64_t c = 0; c < n_centres; ++c) {
      REQUIRE(edges_per_centre[c] >= 0, "negative edge count");
      rp[c + 1] = rp[c] + edges_per_centre[c];
    }
    const std::vector<int64_t> b = plan_chunks(rp.data(), n_centres, chunk_cap(v, cfg->edge_chunk));
    const int64_t nch = (int64_t)b.size() - 1;
    if (n_chunks) *n_chunks = nch;
    if (bounds) {
      REQUIRE(max_bounds >= nch + 1, "bounds holds fewer than n_chunks + 1 entries");
      for (int64_t k = 0; k <= nch; ++k) bounds[k] = b[k];
    }
    return ALLEGRO_OK;
  } catch (const Fail& f) {
    return fail(nullptr, f);
  } catch (const std::bad_alloc&) {
    return fail(nullptr, Fail{ALLEGRO_E_NOMEM, "host allocation failed"});
  } catch (...) {
    return fail(nullptr, Fail{ALLEGRO_E_INVAL, "unexpected exception"});
  }
}

int allegro_create(const AllegroConfig* cfg, const float* weights, int64_t n_weights, const double* species_scale,
                   const double* species_shift, AllegroModel** out) {
  if (out) *out = nullptr;
  AllegroModel* m = nullptr;
  try {
    REQUIRE(out != nullptr, "out is NULL");
    const Validated v = validate(cfg);
    m = new (std::nothrow) AllegroModel();
    if (!m) throw Fail{ALLEGRO_E_NOMEM, "host allocation failed"};
    m->cfg = *cfg;
    m->v = v;
    m->prec = cfg->precision;
    if (cfg->r_cut_pair) m->rc_pair.assign(cfg->r_cut_pair, cfg->r_cut_pair + v.S * v.S);
    if (cfg->atomic_numbers) m->znum.assign(cfg->atomic_numbers, cfg->atomic_numbers + v.S);
    m->cfg.r_cut_pair = nullptr;   // the caller's tables are not kept
    m->cfg.atomic_numbers = nullptr;
    switch (m->prec) {
      case ALLEGRO_PREC_FP32: m->prec_two = m->prec_lat = m->prec_lat_first = m->prec_lat_rest = 0; break;
      case ALLEGRO_PREC_BF16: m->prec_two = m->prec_lat = m->prec_lat_first = m->prec_lat_rest = 1; break;
      case ALLEGRO_PREC_BF16_SINGLE: m->prec_two = m->prec_lat = m->prec_lat_first = m->prec_lat_rest = 2; break;
      default:   // BF16_MIXED: pairs in the two-body MLP and the later MLPs' first layers
        m->prec_two = m->prec_lat = m->prec_lat_first = 1;
        m->prec_lat_rest = 2;
    }
    create_impl(m, weights, n_weights, species_scale, species_shift);
    *out = m;
    return ALLEGRO_OK;
  } catch (const Fail& f) {
    delete m;
    return fail(nullptr, f);
  } catch (const std::bad_alloc&) {
    delete m;
    return fail(nullptr, Fail{ALLEGRO_E_NOMEM, "host allocation failed"});
  } catch (...) {
    delete m;
    return fail(nullptr, Fail{ALLEGRO_E_INVAL, "unexpected exception"});
  }
}

int allegro_neighbors(AllegroModel* m, int64_t n_local, int64_t n_total, const double* pos, const int32_t* species,
                      const double* cell, const int32_t* pbc, void* stream, int64_t* n_edges) {
  if (!m) return ALLEGRO_E_INVAL;
  try {
    neighbors_impl(m, n_local, n_total, pos, species, cell, pbc, (hipStream_t)stream, n_edges);
    return ALLEGRO_OK;
  } catch (const Fail& f) {
    m->n_local = -1;
    return fail(m, f);
  } catch (const std::bad_alloc&) {
    m->n_local = -1;
    return fail(m, Fail{ALLEGRO_E_NOMEM, "host allocation failed"});
  } catch (...) {
    m->n_local = -1;
    return fail(m, Fail{ALLEGRO_E_INVAL, "unexpected exception"});
  }
}

int allegro_neighbors_batched(AllegroModel* m, int32_t n_systems, const int64_t* atom_offsets, const double* pos,
                              const int32_t* species, void* stream, int64_t* n_edges) {
  if (!m) return ALLEGRO_E_INVAL;
  try {
    REQUIRE(n_systems >= 1 && atom_offsets != nullptr, "need n_systems >= 1 and atom_offsets");
    REQUIRE(atom_offsets[0] == 0, "atom_offsets[0] must be 0");
    for (int k = 0; k < n_systems; ++k) REQUIRE(atom_offsets[k + 1] >= atom_offsets[k], "atom_offsets must ascend");
    const int64_t n = atom_offsets[n_systems];
    const int32_t pbc[3] = {0, 0, 0};
    neighbors_impl(m, n, n, pos, species, nullptr, pbc, (hipStream_t)stream, n_edges, atom_offsets, n_systems);
    return ALLEGRO_OK;
  } catch (const Fail& f) {
    m->n_local = -1;
    return fail(m, f);
  } catch (const std::bad_alloc&) {
    m->n_local = -1;
    return fail(m, Fail{ALLEGRO_E_NOMEM, "host allocation failed"});
  } catch (...) {
    m->n_local = -1;
    return fail(m, Fail{ALLEGRO_E_INVAL, "unexpected exception"});
  }
}

int allegro_system_energies(AllegroModel* m, const double* atom_energy, double* system_energy, void* stream) {
  if (!m) return ALLEGRO_E_INVAL;
  try {
    if (m->n_local < 0 || m->n_sys <= 0) throw Fail{ALLEGRO_E_STATE, "no batched neighbour list"};
    REQUIRE(atom_energy && system_energy, "atom_energy and system_energy must not be NULL");
    HIP_OK(launch_system_sums(atom_energy, ptr<int64_t>(m->sys_off), m->n_sys, system_energy, (hipStream_t)stream));
    return ALLEGRO_OK;
  } catch (const Fail& f) {
    return fail(m, f);
  }
}

int allegro_energy_forces(AllegroModel* m, const double* pos, const int32_t* species, double* atom_energy,
                          double* forces, double* virial, double* atom_virial, double* energy, void* stream) {
  if (!m) return ALLEGRO_E_INVAL;
  try {
    energy_forces_impl(m, m->ws, pos, species, atom_energy, forces, virial, atom_virial, energy, (hipStream_t)stream);
    return ALLEGRO_OK;
  } catch (const Fail& f) {
    return fail(m, f);
  } catch (const std::bad_alloc&) {
    return fail(m, Fail{ALLEGRO_E_NOMEM, "host allocation failed"});
  } catch (...) {
    return fail(m, Fail{ALLEGRO_E_INVAL, "unexpected exception"});
  }
}

int allegro_energy_forces_noalloc(AllegroModel* m, const double* pos, const int32_t* species,
                                  double* atom_energy, double* forces, double* virial, double* atom_virial,
                                  double* energy, void* stream) {
  if (!m) return ALLEGRO_E_INVAL;
  try {
    if (m->n_local < 0) throw Fail{ALLEGRO_E_STATE, "allegro_neighbors has not been called"};
    int dev = -1;
    HIP_OK(hipGetDevice(&dev));
    REQUIRE(dev == m->device, "the current device is not the model's device");
    const bool zbl = !m->znum.empty(), tall = m->prec != ALLEGRO_PREC_FP32, rr = m->rr_cfg != 0;
    const size_t need = ws_layout(m->v, m->Ec, m->Nc, m->cap, m->n_local, m->n_total, zbl, tall, rr, 0, nullptr);
    REQUIRE(need <= (size_t)ALLEGRO_NOALLOC_SCRATCH_BYTES,
            "the neighbour list needs " + std::to_string(need) + " bytes of workspace, the static workspace holds " +
                std::to_string((size_t)ALLEGRO_NOALLOC_SCRATCH_BYTES) +
                "; build the list with a smaller edge_chunk");
    void* base = g_scratch_ptr[dev];
    if (!base) throw Fail{ALLEGRO_E_STATE, "static workspace address not resolved on this device"};
    Ws w;
    ws_layout(m->v, m->Ec, m->Nc, m->cap, m->n_local, m->n_total, zbl, tall, rr, (uintptr_t)base, &w);
    // no per-kernel timing here: recording it creates events
    const bool timing = m->timing;
    m->timing = false;
    try {
      energy_forces_impl(m, w, pos, species, atom_energy, forces, virial, atom_virial, energy,
                         (hipStream_t)stream);
    } catch (...) {
      m->timing = timing;
      throw;
    }
    m->timing = timing;
    return ALLEGRO_OK;
  } catch (const Fail& f) {
    return fail(m, f);
  } catch (...) {
    return fail(m, Fail{ALLEGRO_E_INVAL, "unexpected exception"});
  }
}

int allegro_check(AllegroModel* m, void* stream) {
  if (!m) return ALLEGRO_E_INVAL;
  try {
    return take_status(m, (hipStream_t)stream);
  } catch (const Fail& f) {
    return fail(m, f);
  }
}

int allegro_copy_edges(AllegroModel* m, int32_t* centre, int32_t* neighbor, int32_t* shift, void* stream) {
  if (!m) return ALLEGRO_E_INVAL;
  try {
    if (m->n_local < 0) throw Fail{ALLEGRO_E_STATE, "allegro_neighbors has not been called"};
    hipStream_t s = (hipStream_t)stream;
    if (m->E > 0) {
      if (centre) HIP_OK(hipMemcpyAsync(centre, m->ei.p, m->E * 4, hipMemcpyDeviceToDevice, s));
      if (neighbor) HIP_OK(hipMemcpyAsync(neighbor, m->ej.p, m->E * 4, hipMemcpyDeviceToDevice, s));
      if (shift) HIP_OK(hipMemcpyAsync(shift, m->es.p, m->E * 12, hipMemcpyDeviceToDevice, s));
    }
    return ALLEGRO_OK;
  } catch (const Fail& f) {
    return fail(m, f);
  }
}

int64_t allegro_num_edges(const AllegroModel* m) { return m ? m->E : -1; }

int allegro_set_timing(AllegroModel* m, int32_t enable) {
  if (!m) return ALLEGRO_E_INVAL;
  try {
    collect_times(m);
    m->ktimes.clear();
    m->timing = enable != 0;
    return ALLEGRO_OK;
  } catch (const Fail& f) {
    return fail(m, f);
  }
}

int allegro_kernel_times(AllegroModel* m, int32_t max_entries, char* names, double* total_ms, int64_t* launches,
                         int32_t* n_entries) {
  if (!m) return ALLEGRO_E_INVAL;
  try {
    collect_times(m);
    const int n = (int)m->ktimes.size();
    if (n_entries) *n_entries = n;
    for (int k = 0; k < n && k < max_entries; ++k) {
      if (names) {
        std::memset(names + 48 * k, 0, 48);
        std::strncpy(names + 48 * k, m->ktimes[k].name.c_str(), 47);
      }
      if (total_ms) total_ms[k] = m->ktimes[k].ms;
      if (launches) launches[k] = m->ktimes[k].launches;
    }
    return ALLEGRO_OK;
  } catch (const Fail& f) {
    return fail(m, f);
  }
}

int64_t allegro_workspace_bytes(const AllegroModel* m) {
  if (!m) return -1;
  const DevBuf* bufs[] = {&m->ei, &m->ej, &m->es, &m->row_ptr, &m->rrow_ptr, &m->redge, &m->keys, &m->cell_of,
                          &m->img, &m->cell_count, &m->cell_start, &m->cell_cursor, &m->cell_atoms, &m->count,
                          &m->rcount, &m->rcursor, &m->bbox, &m->scan_tmp, &m->arena, &m->chunk_rp};
  int64_t s = 0;
  for (const DevBuf* b : bufs) s += (int64_t)b->bytes;
  return s;
}

void allegro_destroy(AllegroModel* m) {
  if (!m) return;
  release_graph(m);
  if (m->md_stream) (void)hipStreamSynchronize(m->md_stream);
  if (m->md_stream) (void)hipStreamDestroy(m->md_stream);
  for (hipEvent_t e : m->md_ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& p : m->pending) {
    (void)hipEventDestroy(p.second.first);
    (void)hipEventDestroy(p.second.second);
  }
  delete m;
}

const char* allegro_last_error(const AllegroModel* m) {
  if (m) return m->err.c_str();
  return g_create_error.c_str();
}

const char* allegro_status_string(int status) {
  switch (status) {
    case ALLEGRO_OK: return "ALLEGRO_OK";
    case ALLEGRO_E_INVAL: return "ALLEGRO_E_INVAL";
    case ALLEGRO_E_NOMEM: return "ALLEGRO_E_NOMEM";
    case ALLEGRO_E_CAPACITY: return "ALLEGRO_E_CAPACITY";
    case ALLEGRO_E_DEVICE: return "ALLEGRO_E_DEVICE";
    case ALLEGRO_E_NONFINITE: return "ALLEGRO_E_NONFINITE";
    case ALLEGRO_E_STATE: return "ALLEGRO_E_STATE";
    default: return "unknown status";
  }
}

}  // extern "C"
