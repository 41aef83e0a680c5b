// internal.h - data layouts and kernel entry points shared by the host runtime
// (abi.cpp) and the gfx950 kernels (*.hip).  Not part of the public interface.
//
// Edge-major layouts in HBM (E = edges of the current chunk, rows ordered by
// centre, each centre's neighbours sorted by (j, shift)):
//   eb      [E][kEB]     float  edge record: Y[0..8], u, d, rhat[3], Z_i, Z_j, R[16..31];
//                               with l_max = 3 (at most 8 radial functions) the
//                               l = 3 harmonics Y[9..15] sit in slots 24..30
//   x^L     [E][d]       float  latent (scalar-track) features, the residual stream
//   head    [E][H]       float  outputs of the linear map that follows an MLP
//                               (after the two-body MLP: [a0 | w^1], each
//                               (l_max+1) n wide, column l n + u)
//   V^L     [E][w][n]    float  tensor features, component-major: the n channels
//                               of one strided component are contiguous; w = dim
//                               (natural parity only) or 2 dim (both parities)
//   Gamma^L [N][dim][n]  float  per-centre environment sums
// dim = (l_max+1)^2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace allegro {

constexpr int kEB = 32;     // floats per edge record
constexpr int kEB_U = 9;
constexpr int kEB_D = 10;
constexpr int kEB_RHAT = 11;
constexpr int kEB_ZI = 14;  // species of the centre and of the neighbour (small integers held
constexpr int kEB_ZJ = 15;  // exactly as floats), so that edge-row readers need no index chase
constexpr int kEB_R = 16;   // radial basis R_n = B_n u, n < 16 (n < 8 with l_max = 3)
constexpr int kEB_Y3 = 24;  // Y[9..15] when l_max = 3

// Record slot of harmonic component c.
__host__ __device__ constexpr int eb_y(int c) { return c < 9 ? c : kEB_Y3 + (c - 9); }
// Row stride of the dE/dY buffers.
__host__ __device__ constexpr int gy_width(int l_max) { return l_max >= 3 ? 16 : 9; }

// Bits of the model's sticky device status word: set by kernels, read and
// cleared by the host at its next check.
constexpr int kStatusNonFinite = 1;   // a force or atom energy was not finite
constexpr int kStatusCapacity = 2;    // an in-graph neighbour rebuild exceeded the edge capacity

// Slots of the MD flag array (int32) of the in-graph neighbour rebuild.
constexpr int kFlagRebuild = 0;   // this step rebuilds the list
constexpr int kFlagHalt = 1;      // a rebuild overflowed: later steps are discarded
constexpr int kFlagSteps = 2;     // steps completed before a halt
constexpr int kFlagNeed = 3;      // edges the overflowing rebuild needed
constexpr int kFlagBuilds = 4;    // completed steps that rebuilt the list
constexpr int kNumFlags = 5;

// Edge-wise kernels launched over a capacity take the live edge count from
// the device (E_dev, the last row pointer of the list) when it is set.
//
// The argument struct itself is never modified: a kernel that wrote to it
// would get a private copy of the whole struct (scratch memory).
template <class A>
__device__ __forceinline__ int live_edges(const A& a) {
  if (a.E_dev) {
    const int e = *a.E_dev;
    return e < a.E ? e : a.E;
  }
  return a.E;
}

constexpr int kMaxLayers = 4;
constexpr int kTpwArgs = 83;  // fused-table non-zeros passed by value (larger tables are read from memory)

constexpr int kMaxMlpLayers = 3;

// Packed MFMA B operand of a K x N matrix (y = x @ W): fragments
// [Np/16][Kp/32][64 lanes][8 elements]; lane l of fragment (nt, kb) holds
// rows k = 32 kb + 8 (l / 16) + 0..7 of column n = 16 nt + l % 16 (zero padded).
struct GemmB {
  const void* p = nullptr;
  int K = 0, N = 0, Kp = 0, Np = 0;
  int split = 0;   // BF16 hi fragments followed by lo fragments (w = hi + lo)
};

struct MlpW {
  int nl = 0;
  GemmB fwd[kMaxMlpLayers];
  GemmB bwd[kMaxMlpLayers];   // packed W^T (for input gradients)
};

// Weights of the register-resident BF16 chain kernels (mlp_rr.h): each GEMM
// out = in @ M packed as A fragments of the 32x32x16 instruction,
// [pass][K step][block of the pass][hi, lo][64 lanes][8]; lane l of fragment
// (block mb, K step s) holds M[f][32 mb + l % 32] for input features
// f = 16 s + 4 (l / 32) + j (j < 4) and 16 s + 8 + 4 (l / 32) + (j - 4) (j >= 4).
// A pass covers rr_nbp(MB) consecutive blocks of 32 output features.
__host__ __device__ constexpr int rr_nbp(int mb) { return mb % 2 == 0 ? 2 : 1; }
constexpr int kRRTile = 256;   // tile value selecting these kernels (edges per block)
struct RRW {
  int cfg = 0;                 // 0: not packed; 1: d 256, n 64, 3-layer MLPs; 2: d 128, n 32, 2-layer MLPs
  const void* fwd[kMaxMlpLayers] = {};
  const void* bwd[kMaxMlpLayers] = {};   // packed W^T
  const void* head = nullptr;
  const void* head_bwd = nullptr;
};

enum MlpKind { kTwoBody = 0, kLatent = 1, kLatentFinal = 2 };

// Where a tensor-product input V[e][a][u] comes from.
struct VSrc {
  const float* p = nullptr;   // stored V [E][dim][n]  or  a0 (head columns 0..(l_max+1)n)
  int ld = 0;                 // row stride (floats)
  int from_a0 = 0;            // V[a][u] = a0[l(a) n + u] * Y[a]
};

struct MlpArgs {
  int E = 0;                  // rows of this launch
  const int32_t* E_dev = nullptr;  // live rows on the device (launch over E = a capacity), or null
  int kind = 0;
  int tm = 0;                 // edge-tile rows (0 = largest that fits LDS)
  int d = 0, n = 0, l_max = 0, n_species = 0, n_bessel = 0;
  MlpW w;
  GemmB head;                 // forward head (none when head.p == nullptr)
  GemmB head_bwd;             // its transpose (backward)
  const float* eb = nullptr;
  const int32_t* ei = nullptr;  // centre of each edge (global atom index)
  int centre_base = 0;          // first centre of the chunk (Gamma rows are chunk-local)
  const int32_t* ej = nullptr;  // neighbour of each edge (global atom index)
  const int32_t* species = nullptr;  // [n_total]
  // latent inputs
  const float* x_prev = nullptr;  // [E][d]
  const float* s_in = nullptr;    // non-final: V^L (component 0 = first n floats), row stride s_ld;
                                  // final: the stored tensor-product scalars, or null to recompute them
  int s_ld = 0;
  // final layer: scalar tensor-product outputs computed in the prologue
  VSrc tp_v;
  const float* tp_gam = nullptr;  // Gamma [centres][dim][n]
  float* tp_out = nullptr;        // forward: receives those scalars [E][n] (optional); the
                                  // backward reads them back through s_in (s_ld = n)
  float tp_w[16] = {0};           // diagonal coupling weight of each component
  float res_scale = 0.70710678118654752f;
  // forward outputs
  float* x_out = nullptr;         // [E][d]
  float* head_out = nullptr;      // [E][head.N]
  float* eij = nullptr;           // final: [E]
  const float* we = nullptr;      // final: folded edge-energy vector [d]
  // backward inputs / outputs
  const float* g_head = nullptr;  // [E][head.N]
  const float* g_x = nullptr;     // [E][d] gradient w.r.t. x_out (partial)
  const float* g_const = nullptr; // final: [n_species][d] = sigma_Z * we
  float* g_xprev = nullptr;       // [E][d]
  float* g_s = nullptr;           // [E][n]
  float* g_u = nullptr;           // [E]
  int gu_accum = 0;
  float* g_R = nullptr;           // two-body: [E][n_bessel]
  // tall-tile backward only
  float* g_store = nullptr;       // [E][d] receives dE/dx_out (g_xprev, or g_x itself for two-body)
  void* act_scratch = nullptr;    // hidden pre-activations of the recomputation (fragment order)
  // Register-resident kernels: activations the forward pass stores and the
  // backward pass reads instead of recomputing the chain (both directions
  // must run the register-resident kernels on the same edges and tiles):
  // hidden pre-activations and h (two-body, latent), or the last hidden
  // pre-activations plus a . v per edge in av_store (final layer).
  void* act_store = nullptr;
  float* av_store = nullptr;
  RRW rr;                         // register-resident kernels' weights (rr.cfg = 0: unavailable)
  const float* fold_v = nullptr;  // final layer, register-resident kernels: v = W_last w_e [d]
  float sigma[16] = {0};          // species scales sigma_Z (final layer, register-resident backward)
};

struct EdgeArgs {
  int64_t E = 0;
  const int32_t* E_dev = nullptr;  // live edges on the device (launch over E = a capacity), or null
  const double* pos = nullptr;
  const int32_t* ei = nullptr;    // global centre index
  const int32_t* ej = nullptr;
  const int32_t* es = nullptr;    // [E][3]
  const int32_t* species = nullptr;  // [n_total]
  double L[3] = {0, 0, 0};        // periodic lengths (0 = open axis)
  double r_cut = 0;
  const float* rc_pair = nullptr; // [S][S] cutoff of each ordered species pair, or null (r_cut)
  int n_species = 1;
  const float* zbl = nullptr;     // [2][S] atomic number and its 0.23 power per species, or null (no ZBL)
  float* e_pair = nullptr;        // [E] ZBL share of each ordered edge (written when zbl is set)
  int p = 6, n_bessel = 8, l_max = 2;
  float* eb = nullptr;
  // backward
  const float* g_Y = nullptr;     // [E][gy_width(l_max)]
  const float* g_R = nullptr;     // [E][n_bessel]
  const float* g_u = nullptr;     // [E]
  float* g_e = nullptr;           // [E][3]
};

struct TensorArgs {
  int E = 0;                      // edges of the chunk
  const int32_t* E_dev = nullptr; // live edges on the device (launch over E = a capacity), or null
  int tile = 0;                   // edges per tile of the edge-tile kernels (16 or 32; 0 = 32)
  int n_centres = 0;
  int n = 0, l_max = 0;
  int in_kind = 1, out_kind = 1;  // irrep kinds (TpKind) of this layer's input and output features
  int next_in = 1, next_out = 0;  // kinds of the next layer (channel-mixing adjoint)
  const int32_t* row_ptr = nullptr;  // [n_centres+1], chunk-relative
  const int32_t* ei = nullptr;       // centre per edge (global atom index)
  int centre_base = 0;               // first centre of the chunk
  const float* eb = nullptr;
  const float* w_env = nullptr;   // [E][(l_max+1) n] at row stride ld_w
  int ld_w = 0;
  float c_norm = 1.0f;
  float* gam = nullptr;           // [n_centres][dim][n]
  VSrc v;                         // tensor-product input
  const float* tpw = nullptr;     // device: non-zero weights of the fused table (for the
                                  // mixing adjoint: those of the next layer)
  float tpw_v[kTpwArgs] = {0};    // the same values, passed by value (kernel argument)
  const void* mixB = nullptr;     // packed FP32 mixing matrices, one GemmB block per irrep slot
                                  // (natural l = 0..l_max, then unnatural l = 0..l_max)
  int mix_stride = 0;             // floats between consecutive blocks
  int channel_mix = 1;
  int mix_bf3 = 0;                // mixing as three BF16 MFMAs per product (BF16 modes)
  float mix_scale = 1.0f;         // 1/sqrt(n)
  float* v_out = nullptr;         // [E][w_out][n]
  // backward
  const float* g_t = nullptr;     // [E][dout][n]
  const float* g_s = nullptr;     // [E][n] gradient w.r.t. scalar outputs (component 0)
  const float* gam_next = nullptr;  // next layer's Gamma (to rebuild dE/dV)
  const float* g_tnext = nullptr;   // next layer's dE/dT [E][w_next_out][n]
  float tp_wnext[16] = {0};         // final next layer: its diagonal weights
  float* g_tout = nullptr;        // [E][w_out][n]
  float* g_w = nullptr;           // [E][(l_max+1) n] at row stride ld_gw
  int ld_gw = 0;
  float* g_a0 = nullptr;          // [E][(l_max+1) n] at row stride ld_gw (layer 1 only)
  float* g_Y = nullptr;           // [E][gy_width(l_max)]
  int gy_accum = 0;
  float* g_gam = nullptr;         // [n_centres][dim][n] dE/dGamma (without the factor c)
};

// Kernel launchers (each returns hipSuccess or the launch error).
hipError_t launch_edge_basis(const EdgeArgs& a, hipStream_t s);
hipError_t launch_edge_adjoint(const EdgeArgs& a, hipStream_t s);
hipError_t launch_mlp_fwd(const MlpArgs& a, int prec, hipStream_t s);
hipError_t launch_mlp_bwd(const MlpArgs& a, int prec, hipStream_t s);
size_t mlp_lds_bytes(const MlpArgs& a, int prec, bool bwd);
bool mlp_tile_fits(const MlpArgs& a, int prec, bool bwd, int tm);
size_t mlp_tall_scratch_bytes(int64_t E, int d);   // scratch of the 128-row backward kernels
size_t mlp_rr_scratch_bytes(int64_t E, int d, int nl);   // activation array of the register-resident kernels
bool mlp_uses_rr(const MlpArgs& a, int prec);             // whether a launch takes the register-resident kernels
hipError_t launch_mlp_rr(const MlpArgs& a, bool bwd, hipStream_t s);   // mlp_rr*.hip
hipError_t launch_env(const TensorArgs& a, hipStream_t s);
hipError_t launch_tp_mix(const TensorArgs& a, bool final_layer, hipStream_t s);
hipError_t launch_mix_adjoint(const TensorArgs& a, hipStream_t s);
hipError_t launch_tp_env_adjoint(const TensorArgs& a, bool final_layer, hipStream_t s);

struct ReduceArgs {
  int n_centres = 0;              // centres of the chunk
  int centre_base = 0;            // global index of the chunk's first centre
  const int32_t* row_ptr = nullptr;  // chunk-relative [n_centres+1]
  const float* eij = nullptr;
  const float* e_pair = nullptr;  // [E] unscaled pair-term shares, or null
  const int32_t* species = nullptr;
  int n_species = 1;
  const double* scale = nullptr;
  const double* shift = nullptr;
  double* atom_energy = nullptr;  // global [n_local]
};
hipError_t launch_atom_energy(const ReduceArgs& a, hipStream_t s);

struct ForceArgs {
  int64_t n_total = 0, n_local = 0;
  const double* pos = nullptr;
  const int32_t* row_ptr = nullptr;   // [n_local+1]
  const int32_t* rrow_ptr = nullptr;  // [n_total+1] reverse CSR (edges by neighbour)
  const int32_t* redge = nullptr;     // [E] edge ids grouped by neighbour, ascending
  const int32_t* ei = nullptr;
  const int32_t* ej = nullptr;
  const int32_t* es = nullptr;
  double L[3] = {0, 0, 0};
  const float* g_e = nullptr;
  double* forces = nullptr;
  double* atom_virial = nullptr;      // may be null
  double* partial = nullptr;          // [n_blocks][10]  (virial 9 + energy 1)
  const double* atom_energy = nullptr;
  int* status = nullptr;              // sticky device status bits (kStatus*), or null
};
hipError_t launch_forces(const ForceArgs& a, int* n_blocks, hipStream_t s);
hipError_t launch_final_sums(const double* partial, int n_blocks, double* virial, double* energy,
                             hipStream_t s);

struct NbrArgs {
  int64_t n_local = 0, n_total = 0;
  const double* pos = nullptr;
  const int32_t* species = nullptr;
  int n_species = 0;
  double L[3] = {0, 0, 0};
  int pbc[3] = {0, 0, 0};
  double lo[3] = {0, 0, 0};       // grid origin (open axes)
  double h[3] = {1, 1, 1};        // cell size
  int nc[3] = {1, 1, 1};          // cells per axis
  int R[3] = {1, 1, 1};           // stencil half-width per axis
  double r_cut2 = 0;
  const double* rc2_pair = nullptr;  // [S][S] squared list radius of each ordered species pair, or null (r_cut2)
  int32_t* cell_of = nullptr;     // [n_total]
  int32_t* img = nullptr;         // [n_total][3] image index q (x = x_wrapped + q L)
  int32_t* cell_count = nullptr;  // [n_cells]
  int32_t* cell_start = nullptr;  // [n_cells+1]
  int32_t* cell_cursor = nullptr; // [n_cells]
  int32_t* cell_atoms = nullptr;  // [n_total]
  int32_t* count = nullptr;       // [n_local]
  int32_t* row_ptr = nullptr;     // [n_local+1]
  unsigned long long* keys = nullptr;  // [E] unsorted candidate keys
  int32_t* ei = nullptr;
  int32_t* ej = nullptr;
  int32_t* es = nullptr;
  int32_t* rcount = nullptr;      // [n_total]
  int32_t* rrow_ptr = nullptr;    // [n_total+1]
  int32_t* rcursor = nullptr;     // [n_total]
  int32_t* redge = nullptr;       // [E]
  double* bbox = nullptr;         // [n_blocks][6] partial min/max
  void* scan_tmp = nullptr;       // exclusive_scan_tmp_bytes(max(n_total, n_cells))
  // batched independent systems (null otherwise): system of each atom and the
  // offset added to its coordinates for binning only
  const int32_t* sys = nullptr;
  const double* sys_shift = nullptr;  // [n_systems][3]
  // in-graph rebuild: the kernels run only when *pred != 0 (null: always);
  // the edge count comes from row_ptr[n_local]
  const int32_t* pred = nullptr;
};
hipError_t launch_bbox(const NbrArgs& a, int* n_blocks, hipStream_t s);
hipError_t launch_system_bbox(const double* pos, const int64_t* offsets, int n_sys, double* out, hipStream_t s);
hipError_t launch_system_sums(const double* atom_value, const int64_t* offsets, int n_sys, double* out,
                              hipStream_t s);
hipError_t launch_bin_atoms_err(const NbrArgs& a, int* err, hipStream_t s);
hipError_t launch_fill_cells(const NbrArgs& a, hipStream_t s);
hipError_t launch_count_neighbors(const NbrArgs& a, hipStream_t s);
hipError_t launch_exclusive_scan(const int32_t* in, int32_t* out, int64_t n, void* tmp, hipStream_t s,
                                 const int32_t* pred = nullptr);
size_t exclusive_scan_tmp_bytes(int64_t n);
hipError_t launch_fill_neighbors(const NbrArgs& a, hipStream_t s);
hipError_t launch_sort_neighbors(const NbrArgs& a, hipStream_t s);
hipError_t launch_reverse_csr(const NbrArgs& a, int64_t E, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);

// velocity Verlet (md.hip)
hipError_t launch_kick_drift(int64_t n, double dt, const double* m, double* x, double* v, const double* f,
                             hipStream_t s);
hipError_t launch_kick(int64_t n, double dt, const double* m, double* v, const double* f, hipStream_t s);
hipError_t launch_ghost_refresh(int64_t n_ghost, int64_t n_local, const int32_t* owner, const double* offset,
                                double* x, hipStream_t s);
hipError_t launch_fold(int64_t n_local, const int32_t* gptr, const int32_t* gidx, double* f, hipStream_t s);
// Where MD steps write their energies: rows [cap][2], the next row `counter`.
// Per-step virial rows [cap][9] too, when set.
struct ThermoTarget {
  double* rows;
  int64_t cap;
  int64_t counter;
  double* vrows;
};
hipError_t launch_thermo(int64_t n, const double* m, const double* v, double* part, const double* epot,
                         const double* vir, ThermoTarget* target, hipStream_t s);
hipError_t launch_set_thermo(ThermoTarget* target, double* rows, double* vrows, int64_t cap, hipStream_t s);
hipError_t launch_disp_check(int64_t n, const double* x, const double* x0, double r2, int32_t* flags,
                             hipStream_t s);
hipError_t launch_copy_f64_flag(double* dst, const double* src, int64_t n, const int32_t* flags, int slot, int want,
                                hipStream_t s);
hipError_t launch_capacity_check(int32_t* row_ptr, int64_t n_local, int64_t cap, int32_t* flags, int* status,
                                 hipStream_t s);
hipError_t launch_step_done(int32_t* flags, hipStream_t s);
hipError_t launch_max_disp(int64_t n, const double* x, const double* x0, double* part, int* n_blocks,
                           hipStream_t s);

}  // namespace allegro
