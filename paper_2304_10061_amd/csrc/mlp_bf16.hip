// mlp_bf16.hip - MLP chain kernels, BF16 operands with hi+lo weight pairs.
#include "mlp_kernels.h"

namespace allegro {
namespace mlpk {
template hipError_t launch_prec<1>(const MlpArgs&, int, bool, hipStream_t);
}  // namespace mlpk
}  // namespace allegro
