// stencil_decl.h -- per-K stencil launchers (defined in launch.cuh and
// explicitly instantiated, a few kernel sizes per translation unit, so the
// build parallelises).
#pragma once
#include "ops.h"

namespace maid {
template <typename T, int K>
hipError_t conv_k(const Shape& d, int R, const T* ker, const T* in, const T* sub, T* out, double* part, hipStream_t s);
template <typename T, int K>
hipError_t apg_grad_k(const Shape& d, int R, const Params& p, const ApgState* sin, ApgState* sout, const ApgBufs<T>& b,
                      hipStream_t s);
template <typename T, int K>
hipError_t apg_trial_k(const Shape& d, int R, const Params& p, const ApgState* sin, ApgState* sout, const ApgBufs<T>& b,
                       hipStream_t s);
template <typename T, int K>
hipError_t cg_dir_k(const Shape& d, int R, const Params& p, const CgState* sin, CgState* sout, const CgBufs<T>& b, int init,
                    hipStream_t s);
template <typename T, int K>
hipError_t cg_hvp_k(const Shape& d, int R, const Params& p, const CgState* sin, CgState* sout, const CgBufs<T>& b, int init,
                    hipStream_t s);
}  // namespace maid
