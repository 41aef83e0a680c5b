// mlp_rr2f.hip - register-resident BF16 chain kernels, forward, latent width 128.
#include "mlp_rr.h"

namespace allegro {
hipError_t launch_mlp_rr_128_fwd(const MlpArgs& a, hipStream_t s) { return rr::dispatch<true, 128, 32, 96, 2>(a, s); }
}  // namespace allegro
