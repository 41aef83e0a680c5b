// mlp_rr1b.hip - register-resident BF16 chain kernels, backward, latent width 256.
#include "mlp_rr.h"

namespace allegro {
hipError_t launch_mlp_rr_256_bwd(const MlpArgs& a, hipStream_t s) { return rr::dispatch<false, 256, 64, 192, 3>(a, s); }
}  // namespace allegro
