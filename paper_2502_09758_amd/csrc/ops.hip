// ops.hip -- Ops<T>: runtime dispatch of K to the per-K launchers, and the
// kernels that do not depend on K.
#include "kernels.cuh"
#include "stencil_decl.h"

namespace maid {

// out = th - s z  (double, K*K)
__global__ void k_theta_step(const double* __restrict__ th, const double* __restrict__ z, double s, double* __restrict__ out, int KK) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < KK) out[t] = th[t] - s * z[t];
}

// Sobolev term on the KxK grid (Neumann forward differences):
// value r = beta (w0 sum e^2 + sum (D_h e)^2 + sum (D_v e)^2), e = theta - a,
// gradient 2 beta (w0 e + D^T D e).  One block of 1024 threads.
__device__ __forceinline__ double sob_e(const double* s_e, int K, int u, int v) { return s_e[u * K + v]; }

__global__ __launch_bounds__(1024) void k_sobolev(double beta, double h1_w0, const double* __restrict__ th,
                                                  const double* __restrict__ a, int K, double* __restrict__ out) {
    __shared__ double s_e[1024];
    __shared__ double s_r[1024];
    const int t = threadIdx.x, KK = K * K;
    if (t < KK) s_e[t] = th[t] - a[t];
    __syncthreads();
    double val = 0.0;
    if (t < KK) {
        const int u = t / K, v = t - u * K;
        const double e = s_e[t];
        const double dh = (v < K - 1) ? sob_e(s_e, K, u, v + 1) - e : 0.0;
        const double dv = (u < K - 1) ? sob_e(s_e, K, u + 1, v) - e : 0.0;
        val = h1_w0 * e * e + dh * dh + dv * dv;
    }
    s_r[t] = val;
    __syncthreads();
    if (t == 0) {
        double s = 0.0;
        for (int i = 0; i < KK; ++i) s += s_r[i];
        *out = beta * s;
    }
}


// *out = sum of nb partials (one block)
__global__ __launch_bounds__(kNT) void k_reduce(const double* __restrict__ part, int nb, double* __restrict__ out) {
    const double s = reduce_partials(part, nb);
    if (threadIdx.x == 0) *out = s;
}

#define MAID_FOR_EACH_K(X) X(1) X(3) X(5) X(7) X(9) X(11) X(13) X(15) X(17) X(19) X(21) X(23) X(25) X(27) X(29) X(31)

template <typename T>
hipError_t Ops<T>::prep_kernel(double* L_io, double* abs_out, const double* th, T* out, T* outf, int K, hipStream_t s) {
    hipLaunchKernelGGL(k_prep_kernel<T>, dim3(1), dim3(1024), 0, s, L_io, abs_out, th, out, outf, K);
    return hipGetLastError();
}

template <typename T>
hipError_t Ops<T>::conv(const Shape& d, int R, const T* ker, const T* in, const T* sub, T* out, double* part, hipStream_t s) {
    switch (d.K) {
#define MAID_CASE(KV) \
    case KV: return conv_k<T, KV>(d, R, ker, in, sub, out, part, s);
        MAID_FOR_EACH_K(MAID_CASE)
#undef MAID_CASE
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t Ops<T>::apg_grad(const Shape& d, int R, const Params& p, const ApgState* sin, ApgState* sout, const ApgBufs<T>& b,
                            hipStream_t s) {
    switch (d.K) {
#define MAID_CASE(KV) \
    case KV: return apg_grad_k<T, KV>(d, R, p, sin, sout, b, s);
        MAID_FOR_EACH_K(MAID_CASE)
#undef MAID_CASE
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t Ops<T>::apg_trial(const Shape& d, int R, const Params& p, const ApgState* sin, ApgState* sout, const ApgBufs<T>& b,
                             hipStream_t s) {
    switch (d.K) {
#define MAID_CASE(KV) \
    case KV: return apg_trial_k<T, KV>(d, R, p, sin, sout, b, s);
        MAID_FOR_EACH_K(MAID_CASE)
#undef MAID_CASE
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t Ops<T>::cg_dir(const Shape& d, int R, const Params& p, const CgState* sin, CgState* sout, const CgBufs<T>& b,
                          int init, hipStream_t s) {
    switch (d.K) {
#define MAID_CASE(KV) \
    case KV: return cg_dir_k<T, KV>(d, R, p, sin, sout, b, init, s);
        MAID_FOR_EACH_K(MAID_CASE)
#undef MAID_CASE
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t Ops<T>::cg_hvp(const Shape& d, int R, const Params& p, const CgState* sin, CgState* sout, const CgBufs<T>& b,
                          int init, hipStream_t s) {
    switch (d.K) {
#define MAID_CASE(KV) \
    case KV: return cg_hvp_k<T, KV>(d, R, p, sin, sout, b, init, s);
        MAID_FOR_EACH_K(MAID_CASE)
#undef MAID_CASE
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t Ops<T>::apg_final(const ApgState* sin, const ApgBufs<T>& b, T* out, int64_t n, hipStream_t s) {
    int64_t nb = (n + kNT - 1) / kNT;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_apg_final<T>, dim3((unsigned)nb), dim3(kNT), 0, s, sin, b.X[0], b.X[1], b.X[2], out, n);
    return hipGetLastError();
}

template <typename T>
hipError_t Ops<T>::cg_update(const CgState* sin, CgState* sout, const CgBufs<T>& b, int64_t n, int nblk, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_update<T>, dim3(nblk), dim3(kNT), 0, s, sin, sout, b, n);
    return hipGetLastError();
}

template <typename T>
hipError_t Ops<T>::cg_init(const CgBufs<T>& b, int64_t n, int nblk, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_init<T>, dim3(nblk), dim3(kNT), 0, s, b, n);
    return hipGetLastError();
}

template <typename T>
hipError_t Ops<T>::hg_corr(const Shape& d, const T* rho, const T* q, const T* w, const T* xt, double* part, int nblk,
                           hipStream_t s) {
    if (d.K <= 16)
        hipLaunchKernelGGL((k_hg_corr<T, 16>), dim3(nblk), dim3(kNT), 0, s, d.C, d.H, d.W, d.K, rho, q, w, xt, part);
    else
        hipLaunchKernelGGL((k_hg_corr<T, 32>), dim3(nblk), dim3(kNT), 0, s, d.C, d.H, d.W, d.K, rho, q, w, xt, part);
    return hipGetLastError();
}

template struct Ops<float>;
template struct Ops<double>;

hipError_t launch_reduce(const double* part, int nb, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kNT), 0, s, part, nb, out);
    return hipGetLastError();
}

int hg_items(const Shape& d) {
    return ((d.W + kHgTJ - 1) / kHgTJ) * ((d.H + kHgTI - 1) / kHgTI) * d.C * 2;
}

hipError_t launch_hg_final(const Shape& d, double beta, double h1_w0, const double* part, int nblk, const double* th,
                           const double* a, int with_r, double* z, double* znorm2, hipStream_t s) {
    if (d.K <= 16)
        hipLaunchKernelGGL(k_hg_final<16>, dim3(1), dim3(1024), 0, s, beta, h1_w0, part, nblk, d.K, th, a, with_r, z, znorm2);
    else
        hipLaunchKernelGGL(k_hg_final<32>, dim3(1), dim3(1024), 0, s, beta, h1_w0, part, nblk, d.K, th, a, with_r, z, znorm2);
    return hipGetLastError();
}

hipError_t launch_theta_step(const double* th, const double* z, double step, double* out, int KK, hipStream_t s) {
    hipLaunchKernelGGL(k_theta_step, dim3((KK + 255) / 256), dim3(256), 0, s, th, z, step, out, KK);
    return hipGetLastError();
}

hipError_t launch_sobolev(double beta, double h1_w0, const double* th, const double* a, int K, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_sobolev, dim3(1), dim3(1024), 0, s, beta, h1_w0, th, a, K, out);
    return hipGetLastError();
}

}  // namespace maid
