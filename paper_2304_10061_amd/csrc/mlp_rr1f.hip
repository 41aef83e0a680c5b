// mlp_rr1f.hip - register-resident BF16 chain kernels, forward, latent width 256.
#include "mlp_rr.h"

namespace allegro {
hipError_t launch_mlp_rr_256_fwd(const MlpArgs& a, hipStream_t s) { return rr::dispatch<true, 256, 64, 192, 3>(a, s); }
}  // namespace allegro
