// Stencil kernels for K = 17 and K = 19 (both storage types).
#include "launch.cuh"
namespace maid {
MAID_INSTANTIATE_K(17)
MAID_INSTANTIATE_K(19)
}  // namespace maid
