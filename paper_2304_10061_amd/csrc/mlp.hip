// mlp.hip - host-side tile selection for the MLP chain kernels
// (mlp_kernels.h; instantiated per precision in mlp_fp32.hip, mlp_bf16.hip
// and mlp_bf16s.hip).
#include "mlp_kernels.h"
#include "mlp_rr.h"

namespace allegro {

// register-resident kernels, one source file per latent width and direction
hipError_t launch_mlp_rr_256_fwd(const MlpArgs& a, hipStream_t s);   // mlp_rr1f.hip
hipError_t launch_mlp_rr_256_bwd(const MlpArgs& a, hipStream_t s);   // mlp_rr1b.hip
hipError_t launch_mlp_rr_128_fwd(const MlpArgs& a, hipStream_t s);   // mlp_rr2f.hip
hipError_t launch_mlp_rr_128_bwd(const MlpArgs& a, hipStream_t s);   // mlp_rr2b.hip

hipError_t launch_mlp_rr(const MlpArgs& a, bool bwd, hipStream_t s) {
  if (a.E <= 0) return hipSuccess;
  if (a.kind == kLatentFinal && (a.fold_v == nullptr || a.we == nullptr)) return hipErrorInvalidValue;
  if (a.kind == kLatentFinal && a.act_store != nullptr && a.av_store == nullptr) return hipErrorInvalidValue;
  if (bwd && ((a.act_scratch == nullptr && a.act_store == nullptr) ||
              (a.kind != kLatentFinal && a.g_store == nullptr)))
    return hipErrorInvalidValue;
  if (a.rr.cfg == 1) return bwd ? launch_mlp_rr_256_bwd(a, s) : launch_mlp_rr_256_fwd(a, s);
  if (a.rr.cfg == 2) return bwd ? launch_mlp_rr_128_bwd(a, s) : launch_mlp_rr_128_fwd(a, s);
  return hipErrorInvalidValue;
}

size_t mlp_rr_scratch_bytes(int64_t E, int d, int nl) { return rr::scratch_bytes(E, d, nl); }

bool mlp_uses_rr(const MlpArgs& a, int prec) {
  return (prec == 1 || prec == 2) && a.rr.cfg != 0 && (a.tm == kRRTile || a.tm == 0);
}

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
    // register-resident kernels by default where the model has them
    if (mlp_uses_rr(a, prec)) return launch_mlp_rr(a, bwd, s);
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
  if (tm == kRRTile) return prec != 0 && a.rr.cfg != 0;
  if (prec && tm == kTallRows) return tall_fits(a, prec, bwd);
  if (prec) return (tm == 64 || tm == 32) && fits<1>(a, bwd, tm);
  return (tm == 32 || tm == 16) && fits<0>(a, bwd, tm);
}

size_t mlp_tall_scratch_bytes(int64_t E, int d) { return tall_scratch_bytes(E, d); }

hipError_t launch_mlp_fwd(const MlpArgs& a, int prec, hipStream_t s) { return launch(a, prec, false, s); }
hipError_t launch_mlp_bwd(const MlpArgs& a, int prec, hipStream_t s) { return launch(a, prec, true, s); }

}  // namespace allegro
