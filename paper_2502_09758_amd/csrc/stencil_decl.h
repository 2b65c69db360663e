// stencil_decl.h -- per-K stencil launchers (defined in launch.cuh and
// explicitly instantiated, a few kernel sizes per translation unit, so the
// build parallelises).
#pragma once
#include "ops.h"

namespace maid {
template <typename T, int K>
hipError_t conv_k(const Shape& d, int R, DevCtx* c, const T* ker, const T* in, const T* sub, T* out, int slot,
                  double* partials, unsigned* counter, hipStream_t s);
template <typename T, int K>
hipError_t apg_grad_k(const Shape& d, int R, DevCtx* c, const ApgBufs<T>& b, hipStream_t s);
template <typename T, int K>
hipError_t apg_trial_k(const Shape& d, int R, DevCtx* c, const ApgBufs<T>& b, hipStream_t s);
template <typename T, int K>
hipError_t cg_dir_k(const Shape& d, int R, DevCtx* c, const CgBufs<T>& b, hipStream_t s);
template <typename T, int K>
hipError_t cg_hvp_k(const Shape& d, int R, DevCtx* c, const CgBufs<T>& b, int init, hipStream_t s);
}  // namespace maid
