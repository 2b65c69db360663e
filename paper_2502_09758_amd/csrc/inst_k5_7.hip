// Stencil kernels for K = 5 and K = 7 (both storage types).
#include "launch.cuh"
namespace maid {
MAID_INSTANTIATE_K(5)
MAID_INSTANTIATE_K(7)
}  // namespace maid
