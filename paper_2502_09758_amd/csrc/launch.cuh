// launch.cuh -- definitions of Ops<T>: K / R dispatch to the kernel
// templates of kernels.cuh.  Included by one translation unit per storage
// type.
#pragma once
#include "kernels.cuh"
#include "ops.h"

namespace maid {

#define MAID_FOR_EACH_K(X) X(1) X(3) X(5) X(7) X(9) X(11) X(13) X(15) X(17) X(19) X(21) X(23) X(25) X(27) X(29) X(31)


// Raise the dynamic-LDS limit of a kernel once if it needs more than 64 KiB.
template <typename Kern>
static inline hipError_t ensure_lds(Kern kern, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <typename T, int K, int R>
static hipError_t conv_kr(const Shape& d, DevCtx* c, const T* ker, const T* in, const T* sub, T* out, int slot, double* partials,
                          unsigned* counter, hipStream_t s) {
    const size_t lds = sizeof(T) * lds_conv(K, R);
    auto kern = k_conv<T, K, R>;
    hipError_t e = ensure_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(stencil_blocks(d, R)), dim3(kNT), lds, s, c, ker, in, sub, out, slot, partials, counter);
    return hipGetLastError();
}

template <typename T, int K, int R>
static hipError_t apg_grad_kr(const Shape& d, DevCtx* c, const ApgBufs<T>& b, hipStream_t s) {
    const int nw = d.reg == 1 ? d.C : 1;
    const size_t lds = sizeof(T) * lds_apg_grad(K, R, d.C, nw);
    auto kern = k_apg_grad<T, K, R>;
    hipError_t e = ensure_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(stencil_blocks(d, R)), dim3(kNT), lds, s, c, b);
    return hipGetLastError();
}

template <typename T, int K, int R>
static hipError_t apg_trial_kr(const Shape& d, DevCtx* c, const ApgBufs<T>& b, hipStream_t s) {
    const size_t lds = sizeof(T) * lds_apg_trial(K, R, d.C);
    auto kern = k_apg_trial<T, K, R>;
    hipError_t e = ensure_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(stencil_blocks(d, R)), dim3(kNT), lds, s, c, b);
    return hipGetLastError();
}

template <typename T, int K, int R>
static hipError_t cg_dir_kr(const Shape& d, DevCtx* c, const CgBufs<T>& b, hipStream_t s) {
    const size_t lds = sizeof(T) * lds_conv(K, R);
    auto kern = k_cg_dir<T, K, R>;
    hipError_t e = ensure_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(stencil_blocks(d, R)), dim3(kNT), lds, s, c, b);
    return hipGetLastError();
}

template <typename T, int K, int R>
static hipError_t cg_hvp_kr(const Shape& d, DevCtx* c, const CgBufs<T>& b, int init, hipStream_t s) {
    const int nw = d.reg == 1 ? d.C : 1;
    const size_t lds = sizeof(T) * lds_cg_hvp(K, R, d.C, nw);
    auto kern = k_cg_hvp<T, K, R>;
    hipError_t e = ensure_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(stencil_blocks(d, R)), dim3(kNT), lds, s, c, b, init);
    return hipGetLastError();
}

#define MAID_R_DISPATCH(FN, ...)                                   \
    switch (R) {                                                   \
        case 1: return FN<T, K, 1>(__VA_ARGS__);                   \
        case 2: return FN<T, K, 2>(__VA_ARGS__);                   \
        case 4: return FN<T, K, 4>(__VA_ARGS__);                   \
        default: return hipErrorInvalidValue;                      \
    }

template <typename T, int K>
hipError_t conv_k(const Shape& d, int R, DevCtx* c, const T* ker, const T* in, const T* sub, T* out, int slot,
                  double* partials, unsigned* counter, hipStream_t s) {
    MAID_R_DISPATCH(conv_kr, d, c, ker, in, sub, out, slot, partials, counter, s)
}
template <typename T, int K>
hipError_t apg_grad_k(const Shape& d, int R, DevCtx* c, const ApgBufs<T>& b, hipStream_t s) {
    MAID_R_DISPATCH(apg_grad_kr, d, c, b, s)
}
template <typename T, int K>
hipError_t apg_trial_k(const Shape& d, int R, DevCtx* c, const ApgBufs<T>& b, hipStream_t s) {
    MAID_R_DISPATCH(apg_trial_kr, d, c, b, s)
}
template <typename T, int K>
hipError_t cg_dir_k(const Shape& d, int R, DevCtx* c, const CgBufs<T>& b, hipStream_t s) {
    MAID_R_DISPATCH(cg_dir_kr, d, c, b, s)
}
template <typename T, int K>
hipError_t cg_hvp_k(const Shape& d, int R, DevCtx* c, const CgBufs<T>& b, int init, hipStream_t s) {
    MAID_R_DISPATCH(cg_hvp_kr, d, c, b, init, s)
}

// Instantiate every stencil launcher of both storage types for one K.
#define MAID_INSTANTIATE_K(KV)                                                                                           \
    template hipError_t conv_k<float, KV>(const Shape&, int, DevCtx*, const float*, const float*, const float*, float*,  \
                                          int, double*, unsigned*, hipStream_t);                                       \
    template hipError_t conv_k<double, KV>(const Shape&, int, DevCtx*, const double*, const double*, const double*,     \
                                           double*, int, double*, unsigned*, hipStream_t);                             \
    template hipError_t apg_grad_k<float, KV>(const Shape&, int, DevCtx*, const ApgBufs<float>&, hipStream_t);          \
    template hipError_t apg_grad_k<double, KV>(const Shape&, int, DevCtx*, const ApgBufs<double>&, hipStream_t);        \
    template hipError_t apg_trial_k<float, KV>(const Shape&, int, DevCtx*, const ApgBufs<float>&, hipStream_t);         \
    template hipError_t apg_trial_k<double, KV>(const Shape&, int, DevCtx*, const ApgBufs<double>&, hipStream_t);       \
    template hipError_t cg_dir_k<float, KV>(const Shape&, int, DevCtx*, const CgBufs<float>&, hipStream_t);             \
    template hipError_t cg_dir_k<double, KV>(const Shape&, int, DevCtx*, const CgBufs<double>&, hipStream_t);           \
    template hipError_t cg_hvp_k<float, KV>(const Shape&, int, DevCtx*, const CgBufs<float>&, int, hipStream_t);        \
    template hipError_t cg_hvp_k<double, KV>(const Shape&, int, DevCtx*, const CgBufs<double>&, int, hipStream_t);

}  // namespace maid
