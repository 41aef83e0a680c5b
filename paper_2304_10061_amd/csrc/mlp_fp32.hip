// mlp_fp32.hip - MLP chain kernels, FP32 operands.
#include "mlp_kernels.h"

namespace allegro {
namespace mlpk {
template hipError_t launch_prec<0>(const MlpArgs&, int, bool, hipStream_t);
}  // namespace mlpk
}  // namespace allegro
