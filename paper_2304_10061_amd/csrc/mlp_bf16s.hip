// mlp_bf16s.hip - MLP chain kernels, BF16 operands with single-rounded weights.
#include "mlp_kernels.h"

namespace allegro {
namespace mlpk {
template hipError_t launch_prec<2>(const MlpArgs&, int, bool, hipStream_t);
}  // namespace mlpk
}  // namespace allegro
