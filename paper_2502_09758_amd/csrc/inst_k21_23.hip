// Stencil kernels for K = 21 and K = 23 (both storage types).
#include "launch.cuh"
namespace maid {
MAID_INSTANTIATE_K(21)
MAID_INSTANTIATE_K(23)
}  // namespace maid
