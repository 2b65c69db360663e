// Stencil kernels for K = 25 and K = 27 (both storage types).
#include "launch.cuh"
namespace maid {
MAID_INSTANTIATE_K(25)
MAID_INSTANTIATE_K(27)
}  // namespace maid
