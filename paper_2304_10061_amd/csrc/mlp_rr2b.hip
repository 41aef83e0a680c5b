// mlp_rr2b.hip - register-resident BF16 chain kernels, backward, latent width 128.
#include "mlp_rr.h"

namespace allegro {
hipError_t launch_mlp_rr_128_bwd(const MlpArgs& a, hipStream_t s) { return rr::dispatch<false, 128, 32, 96, 2>(a, s); }
}  // namespace allegro
