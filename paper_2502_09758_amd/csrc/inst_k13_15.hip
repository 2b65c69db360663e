// Stencil kernels for K = 13 and K = 15 (both storage types).
#include "launch.cuh"
namespace maid {
MAID_INSTANTIATE_K(13)
MAID_INSTANTIATE_K(15)
}  // namespace maid
