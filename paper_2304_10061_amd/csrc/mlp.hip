// mlp.hip - host-side tile selection for the MLP chain kernels
// (mlp_kernels.h; instantiated per precision in mlp_fp32.hip, mlp_bf16.hip
// and mlp_bf16s.hip).
#include "mlp_kernels.h"

namespace allegro {

using namespace mlpk;

namespace {

template <int PREC>
int pick_tm(const MlpArgs& a, bool bwd) {
  for (int t : kTileRows<PREC>) {
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

bool tall_fits(const MlpArgs& a, int prec, bool bwd) {
  if (!tall_ok(a, prec, bwd)) return false;
  int ldx;
  size_t bytes;
  tall_dims(a, bwd, &ldx, &bytes);
  return bytes <= kLdsLimit;
}

hipError_t launch(const MlpArgs& a, int prec, bool bwd, hipStream_t s) {
  if (a.E <= 0) return hipSuccess;
  // the final layer's backward reads the scalars its forward pass stored
  if (bwd && a.kind == kLatentFinal && a.s_in == nullptr) return hipErrorInvalidValue;
  if (prec == 1 || prec == 2) {
    // tall tiles on request (autotuner or allegro_set_tiles), where they fit
    if (a.tm == kTallRows && tall_fits(a, prec, bwd))
      return prec == 1 ? launch_prec<1>(a, kTallRows, bwd, s) : launch_prec<2>(a, kTallRows, bwd, s);
    const int tm = (a.tm == 64 || a.tm == 32) && fits<1>(a, bwd, a.tm) ? a.tm : pick_tm<1>(a, bwd);
    if (tm == 0) return hipErrorInvalidValue;
    return prec == 1 ? launch_prec<1>(a, tm, bwd, s) : launch_prec<2>(a, tm, bwd, s);
  } else {
    const int tm = (a.tm == 32 || a.tm == 16) && fits<0>(a, bwd, a.tm) ? a.tm : pick_tm<0>(a, bwd);
    if (tm == 0) return hipErrorInvalidValue;
    return launch_prec<0>(a, tm, bwd, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

size_t mlp_lds_bytes(const MlpArgs& a, int prec, bool bwd) {
  int ldx, ldh;
  size_t bytes;
  const int tm = prec ? pick_tm<1>(a, bwd) : pick_tm<0>(a, bwd);
  if (tm == 0 || max_ct(a) > 2) return (size_t)-1;
  if (prec) lds_dims<1>(a, tm, bwd, &ldx, &ldh, &bytes);
  else lds_dims<0>(a, tm, bwd, &ldx, &ldh, &bytes);
  return bytes;
}

bool mlp_tile_fits(const MlpArgs& a, int prec, bool bwd, int tm) {
  if (prec && tm == kTallRows) return tall_fits(a, prec, bwd);
  if (prec) return (tm == 64 || tm == 32) && fits<1>(a, bwd, tm);
  return (tm == 32 || tm == 16) && fits<0>(a, bwd, tm);
}

size_t mlp_tall_scratch_bytes(int64_t E, int d) { return tall_scratch_bytes(E, d); }

hipError_t launch_mlp_fwd(const MlpArgs& a, int prec, hipStream_t s) { return launch(a, prec, false, s); }
hipError_t launch_mlp_bwd(const MlpArgs& a, int prec, hipStream_t s) { return launch(a, prec, true, s); }

}  // namespace allegro
