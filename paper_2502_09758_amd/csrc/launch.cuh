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
static hipError_t conv_kr(const Shape& d, const T* ker, const T* in, const T* sub, T* out, double* part, hipStream_t s) {
    const size_t lds = sizeof(T) * lds_conv(K, R);
    auto kern = k_conv<T, K, R>;
    hipError_t e = ensure_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(stencil_blocks(d, R)), dim3(kNT), lds, s, d.C, d.H, d.W, ker, in, sub, out, part);
    return hipGetLastError();
}

template <typename T, int K, int R>
static hipError_t apg_grad_kr(const Shape& d, const Params& p, const ApgState* sin, ApgState* sout, const ApgBufs<T>& b,
                              hipStream_t s) {
    const int nw = d.reg == 1 ? d.C : 1;
    const size_t lds = sizeof(T) * lds_apg_grad(K, R, d.C, nw);
    auto kern = k_apg_grad<T, K, R>;
    hipError_t e = ensure_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(stencil_blocks(d, R)), dim3(kNT), lds, s, p, sin, sout, b);
    return hipGetLastError();
}

template <typename T, int K, int R>
static hipError_t apg_trial_kr(const Shape& d, const Params& p, const ApgState* sin, ApgState* sout, const ApgBufs<T>& b,
                               hipStream_t s) {
    const size_t lds = sizeof(T) * lds_apg_trial(K, R, d.C);
    auto kern = k_apg_trial<T, K, R>;
    hipError_t e = ensure_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(stencil_blocks(d, R)), dim3(kNT), lds, s, p, sin, sout, b);
    return hipGetLastError();
}

template <typename T, int K, int R>
static hipError_t cg_dir_kr(const Shape& d, const Params& p, const CgState* sin, CgState* sout, const CgBufs<T>& b, int init,
                            hipStream_t s) {
    const size_t lds = sizeof(T) * lds_conv(K, R);
    auto kern = k_cg_dir<T, K, R>;
    hipError_t e = ensure_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(stencil_blocks(d, R)), dim3(kNT), lds, s, p, sin, sout, b, init);
    return hipGetLastError();
}

template <typename T, int K, int R>
static hipError_t cg_hvp_kr(const Shape& d, const Params& p, const CgState* sin, CgState* sout, const CgBufs<T>& b, int init,
                            hipStream_t s) {
    const int nw = d.reg == 1 ? d.C : 1;
    const size_t lds = sizeof(T) * lds_cg_hvp(K, R, d.C, nw);
    auto kern = k_cg_hvp<T, K, R>;
    hipError_t e = ensure_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(stencil_blocks(d, R)), dim3(kNT), lds, s, p, sin, sout, b, init);
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
hipError_t conv_k(const Shape& d, int R, const T* ker, const T* in, const T* sub, T* out, double* part, hipStream_t s) {
    MAID_R_DISPATCH(conv_kr, d, ker, in, sub, out, part, s)
}
template <typename T, int K>
hipError_t apg_grad_k(const Shape& d, int R, const Params& p, const ApgState* sin, ApgState* sout, const ApgBufs<T>& b,
                      hipStream_t s) {
    MAID_R_DISPATCH(apg_grad_kr, d, p, sin, sout, b, s)
}
template <typename T, int K>
hipError_t apg_trial_k(const Shape& d, int R, const Params& p, const ApgState* sin, ApgState* sout, const ApgBufs<T>& b,
                       hipStream_t s) {
    MAID_R_DISPATCH(apg_trial_kr, d, p, sin, sout, b, s)
}
template <typename T, int K>
hipError_t cg_dir_k(const Shape& d, int R, const Params& p, const CgState* sin, CgState* sout, const CgBufs<T>& b, int init,
                    hipStream_t s) {
    MAID_R_DISPATCH(cg_dir_kr, d, p, sin, sout, b, init, s)
}
template <typename T, int K>
hipError_t cg_hvp_k(const Shape& d, int R, const Params& p, const CgState* sin, CgState* sout, const CgBufs<T>& b, int init,
                    hipStream_t s) {
    MAID_R_DISPATCH(cg_hvp_kr, d, p, sin, sout, b, init, s)
}

// Instantiate every stencil launcher of both storage types for one K.
#define MAID_INSTANTIATE_T(T, KV)                                                                                        \
    template hipError_t conv_k<T, KV>(const Shape&, int, const T*, const T*, const T*, T*, double*, hipStream_t);       \
    template hipError_t apg_grad_k<T, KV>(const Shape&, int, const Params&, const ApgState*, ApgState*,                \
                                          const ApgBufs<T>&, hipStream_t);                                             \
    template hipError_t apg_trial_k<T, KV>(const Shape&, int, const Params&, const ApgState*, ApgState*,               \
                                           const ApgBufs<T>&, hipStream_t);                                            \
    template hipError_t cg_dir_k<T, KV>(const Shape&, int, const Params&, const CgState*, CgState*, const CgBufs<T>&,  \
                                        int, hipStream_t);                                                             \
    template hipError_t cg_hvp_k<T, KV>(const Shape&, int, const Params&, const CgState*, CgState*, const CgBufs<T>&,  \
                                        int, hipStream_t);

// Instantiate every stencil launcher of both storage types for one K.
#define MAID_INSTANTIATE_K(KV) MAID_INSTANTIATE_T(float, KV) MAID_INSTANTIATE_T(double, KV)

}  // namespace maid
