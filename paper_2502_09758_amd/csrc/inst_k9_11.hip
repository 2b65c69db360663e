// Stencil kernels for K = 9 and K = 11 (both storage types).
#include "launch.cuh"
namespace maid {
MAID_INSTANTIATE_K(9)
MAID_INSTANTIATE_K(11)
}  // namespace maid
