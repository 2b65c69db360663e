// Stencil kernels for K = 1 and K = 3 (both storage types).
#include "launch.cuh"
namespace maid {
MAID_INSTANTIATE_K(1)
MAID_INSTANTIATE_K(3)
}  // namespace maid
