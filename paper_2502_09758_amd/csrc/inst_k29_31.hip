// Stencil kernels for K = 29 and K = 31 (both storage types).
#include "launch.cuh"
namespace maid {
MAID_INSTANTIATE_K(29)
MAID_INSTANTIATE_K(31)
}  // namespace maid
