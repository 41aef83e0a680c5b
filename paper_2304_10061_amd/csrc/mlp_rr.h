// mlp_rr.h - BF16 MLP chains with the edges as the MFMA N dimension.
//
// Same operations as the LDS-staged chain kernels of mlp_kernels.h (the
// scalar track of section "Allegro: Scalable Equivariant Deep Learning"; the
// matrix products dominate the cost, section "Mixed-precision calculations"),
// arranged for the 32x32x16 BF16 matrix instruction with the edges as its N
// dimension: each wave owns 32 kNE consecutive edges and runs their whole
// chain on its own.  For out^T = M^T in^T the A operand is a block of 32
// output features of the weights and the B operand 16 input features of 32
// edges, held in registers.  The K order inside a 16-wide step is permuted
// (feature 16 s + 4 g + j for slot 8 g + j, j < 4, and 16 s + 8 + 4 g + (j - 4)
// for j >= 4, g = lane / 32), which is exactly the order in which a 32 x 32
// accumulator block holds its features: slots 8 h .. 8 h + 7 of an output
// block are the B operand of K step 2 (block) + h of the next layer, so a
// layer's output becomes the next layer's operand without any reshuffling;
// it passes through a per-wave LDS area (private to the wave, no barrier) so
// that the loop over output blocks can stay a loop.  Weights are packed in
// that order at model creation (one 1 KB fragment per (32 output features,
// 16 input features)) and stream from L2 through buffer loads, several K
// steps ahead of their use; each fragment feeds the wave's kNE N blocks.
// Rows beyond E only compute on clamped copies and are never stored.
//
// Backward kernels recompute the chain (no stored activations) and keep the
// hidden pre-activations of the recomputation in a global scratch array in
// register order; dE/dx_out is staged in the output rows it is added to.
//
// Final layer: its MLP's last matrix W is followed only by the folded
// edge-energy vector w_e (no nonlinearity between them), so
// E_ij = rs (x_prev . w_e + u a . v) with v = W w_e (folded at model creation)
// and a the last hidden activation: the forward pass needs a dot product
// instead of that GEMM, and the backward pass starts from
// dE/da = rs u sigma_Z v without recomputing or differentiating it.
#pragma once

#include <type_traits>

#include "mlp_kernels.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace allegro {

// Forward kernels: 64 edges per wave, one wave per SIMD (the accumulators in
// the accumulation registers, the activations of two N blocks in the others).
namespace rr_fwd {
constexpr int kNE = 2, kOcc = 1, kWaves = 4, kPD = 4;
constexpr bool kNonTemporalOut = true;
#include "mlp_rr_body.h"
}  // namespace rr_fwd

// Backward kernels: the same shape (their extra live arrays, the staged
// dE/dx_out and the pre-activation reads, fit the accumulation registers).
namespace rr_bwd {
constexpr int kNE = 2, kOcc = 1, kWaves = 4, kPD = 4;
constexpr bool kNonTemporalOut = false;
#include "mlp_rr_body.h"
}  // namespace rr_bwd

namespace rr {

// The forward kernels store activations in the tile layout the backward
// kernels read.
static_assert(rr_fwd::kNE == rr_bwd::kNE && rr_fwd::kWaves == rr_bwd::kWaves, "tile shapes must agree");

inline size_t scratch_bytes(int64_t E, int D, int NL) { return rr_bwd::scratch_bytes(E, D, NL); }

template <bool FWD, int KIND, int D, int NT, int HN, int NL, bool SF, bool SR>
hipError_t launch(const MlpArgs& a, hipStream_t s) {
  if constexpr (FWD) return rr_fwd::launch_fwd<KIND, D, NT, HN, NL, SF, SR>(a, s);
  else return rr_bwd::launch_bwd<KIND, D, NT, HN, NL, SF, SR>(a, s);
}

// Kernel for the chain of `a` with the configuration's widths; the weight-pair
// pattern (first layer, other layers and head) is read from the packed
// matrices.
template <bool FWD, int D, int NT, int LW, int NL>
hipError_t dispatch(const MlpArgs& a, hipStream_t s) {
  const bool sf = a.w.fwd[0].split != 0, sr = a.w.fwd[a.w.nl - 1].split != 0;
  if (a.w.nl != NL) return hipErrorInvalidValue;
  switch (a.kind) {
    case kTwoBody:
      if (sf && sr) return launch<FWD, kTwoBody, D, NT, 2 * LW, NL, true, true>(a, s);
      if (!sf && !sr) return launch<FWD, kTwoBody, D, NT, 2 * LW, NL, false, false>(a, s);
      break;
    case kLatent:
      if (sf && sr) return launch<FWD, kLatent, D, NT, LW, NL, true, true>(a, s);
      if (sf && !sr) return launch<FWD, kLatent, D, NT, LW, NL, true, false>(a, s);
      if (!sf && !sr) return launch<FWD, kLatent, D, NT, LW, NL, false, false>(a, s);
      break;
    case kLatentFinal:
      if (sf && sr) return launch<FWD, kLatentFinal, D, NT, LW, NL, true, true>(a, s);
      if (sf && !sr) return launch<FWD, kLatentFinal, D, NT, LW, NL, true, false>(a, s);
      if (!sf && !sr) return launch<FWD, kLatentFinal, D, NT, LW, NL, false, false>(a, s);
      break;
  }
  return hipErrorInvalidValue;
}

}  // namespace rr
}  // namespace allegro
