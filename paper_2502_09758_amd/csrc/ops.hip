// ops.hip -- Ops<T>: runtime dispatch of K to the per-K launchers, and the
// kernels that do not depend on K.
#include <algorithm>

#include "kernels.cuh"
#include "stencil_decl.h"

namespace maid {

// x += alpha d over n elements, with per-block FP64 partial sums of d^2
// (part[2b]) and of the new x^2 (part[2b+1]); grid-stride, kNT threads.
template <typename T>
__global__ __launch_bounds__(kNT) void k_axpy_norms(T* __restrict__ x, const T* __restrict__ d, T alpha, int64_t n,
                                                    double* __restrict__ part) {
    double dd = 0.0, xx = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kNT) {
        const T di = d[i];
        const T xi = x[i] + alpha * di;
        x[i] = xi;
        dd += (double)di * (double)di;
        xx += (double)xi * (double)xi;
    }
    block_sum2<4>(dd, xx);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = dd;
        part[2 * blockIdx.x + 1] = xx;
    }
}

template <typename T>
hipError_t launch_axpy_norms(T* x, const T* d, T alpha, int64_t n, double* part, int blocks, hipStream_t s) {
    return launch(k_axpy_norms<T>, dim3(blocks), dim3(kNT), 0, s, x, d, alpha, n, part);
}
template hipError_t launch_axpy_norms<float>(float*, const float*, float, int64_t, double*, int, hipStream_t);
template hipError_t launch_axpy_norms<double>(double*, const double*, double, int64_t, double*, int, hipStream_t);

// dst[i] = (D) src[i] over n elements (grid-stride, kNT threads).
template <typename S, typename D>
__global__ __launch_bounds__(kNT) void k_cast(const S* __restrict__ src, D* __restrict__ dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kNT) dst[i] = (D)src[i];
}

template <typename S, typename D>
hipError_t launch_cast(const S* src, D* dst, int64_t n, hipStream_t s) {
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((n + kNT - 1) / kNT, 2048));
    return launch(k_cast<S, D>, dim3(blocks), dim3(kNT), 0, s, src, dst, n);
}
template hipError_t launch_cast<float, double>(const float*, double*, int64_t, hipStream_t);
template hipError_t launch_cast<double, float>(const double*, float*, int64_t, hipStream_t);

// x64 += alpha d (d in FP32, the sum in FP64), x32 = x64 rounded, per-block
// FP64 partials of d^2 (part[2b]) and x64^2 (part[2b+1]).
__global__ __launch_bounds__(kNT) void k_axpy_mixed(double* __restrict__ x64, const float* __restrict__ d, double alpha,
                                                    int64_t n, float* __restrict__ x32, double* __restrict__ part) {
    double dd = 0.0, xx = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kNT) {
        const double di = (double)d[i];
        const double xi = x64[i] + alpha * di;
        x64[i] = xi;
        x32[i] = (float)xi;
        dd += di * di;
        xx += xi * xi;
    }
    block_sum2<4>(dd, xx);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = dd;
        part[2 * blockIdx.x + 1] = xx;
    }
}

hipError_t launch_axpy_mixed(double* x64, const float* d, double alpha, int64_t n, float* x32, double* part, int blocks,
                             hipStream_t s) {
    return launch(k_axpy_mixed, dim3(blocks), dim3(kNT), 0, s, x64, d, alpha, n, x32, part);
}

// out = th - s z  (double, K*K)
__global__ void k_theta_step(const double* __restrict__ th, const double* __restrict__ z, double s, double* __restrict__ out, int KK) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < KK) out[t] = th[t] - s * z[t];
}

// Sobolev term on the KxK grid of each of kp kernel planes (Neumann forward
// differences, none across planes):
// value r = beta (w0 sum e^2 + sum (D_h e)^2 + sum (D_v e)^2), e = theta - a.
// One block of 1024 threads; thread t takes taps t, t + 1024, ... and thread
// 0 adds the threads' sums in order.
__global__ __launch_bounds__(1024) void k_sobolev(double beta, double h1_w0, const double* __restrict__ th,
                                                  const double* __restrict__ a, int K, int kp, double* __restrict__ out) {
    __shared__ double s_r[1024];
    const int KK = K * K;
    double val = 0.0;
    for (int t = threadIdx.x; t < kp * KK; t += 1024) {
        const int tp = t % KK, u = tp / K, v = tp - u * K;
        const double e = th[t] - a[t];
        const double dh = (v < K - 1) ? (th[t + 1] - a[t + 1]) - e : 0.0;
        const double dv = (u < K - 1) ? (th[t + K] - a[t + K]) - e : 0.0;
        val += h1_w0 * e * e + dh * dh + dv * dv;
    }
    s_r[threadIdx.x] = val;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < 1024; ++i) s += s_r[i];
        *out = beta * s;
    }
}


#define MAID_FOR_EACH_K(X) X(1) X(3) X(5) X(7) X(9) X(11) X(13) X(15) X(17) X(19) X(21) X(23) X(25) X(27) X(29) X(31)

#define MAID_K_SWITCH(CALL)                                  \
    switch (g.K) {                                           \
        MAID_FOR_EACH_K(CALL)                                \
        default: return hipErrorInvalidValue;                \
    }

template <typename T>
hipError_t Ops<T>::prep_kernel(const Inst<T>* insts, int n, ApgState* Lst, CgState* Cst, int slot_abs,
                               hipStream_t s) {
    return launch(k_prep_kernel<T>, dim3(n), dim3(1024), 0, s, insts, Lst, Cst, slot_abs, (const unsigned*)nullptr,
                  (unsigned*)nullptr, 0);
}
template <typename T>
hipError_t Ops<T>::prep_upload(const void* src_host, void* dst, int roles, int n, ApgState* Lst, CgState* Cst,
                               int slot_abs, hipStream_t s) {
    return launch(k_prep_kernel<T>, dim3(n), dim3(1024), 0, s, (const Inst<T>*)dst, Lst, Cst, slot_abs,
                  (const unsigned*)src_host, (unsigned*)dst, roles);
}

template <typename T>
hipError_t Ops<T>::finish(const Inst<T>* insts, int n, int slot, int sob_slot, hipStream_t s) {
    return launch(k_finish<T>, dim3(n), dim3(kNT), 0, s, insts, slot, sob_slot);
}

template <typename T>
hipError_t Ops<T>::conv(const Group& g, const Inst<T>* insts, hipStream_t s) {
#define MAID_CASE(KV) \
    case KV: return conv_k<T, KV>(g, insts, s);
    MAID_K_SWITCH(MAID_CASE)
#undef MAID_CASE
}

template <typename T>
hipError_t Ops<T>::apg_grad(const Group& g, const Inst<T>* insts, const ApgState* sin, ApgState* sout, hipStream_t s) {
#define MAID_CASE(KV) \
    case KV: return apg_grad_k<T, KV>(g, insts, sin, sout, s);
    MAID_K_SWITCH(MAID_CASE)
#undef MAID_CASE
}

template <typename T>
hipError_t Ops<T>::apg_trial(const Group& g, const Inst<T>* insts, const ApgState* sin, ApgState* sout, hipStream_t s) {
#define MAID_CASE(KV) \
    case KV: return apg_trial_k<T, KV>(g, insts, sin, sout, s);
    MAID_K_SWITCH(MAID_CASE)
#undef MAID_CASE
}

template <typename T>
hipError_t Ops<T>::cg_dir(const Group& g, const Inst<T>* insts, const CgState* sin, CgState* sout, int init, hipStream_t s) {
#define MAID_CASE(KV) \
    case KV: return cg_dir_k<T, KV>(g, insts, sin, sout, init, s);
    MAID_K_SWITCH(MAID_CASE)
#undef MAID_CASE
}

template <typename T>
hipError_t Ops<T>::cg_hvp(const Group& g, const Inst<T>* insts, const CgState* sin, CgState* sout, int init, hipStream_t s) {
#define MAID_CASE(KV) \
    case KV: return cg_hvp_k<T, KV>(g, insts, sin, sout, init, s);
    MAID_K_SWITCH(MAID_CASE)
#undef MAID_CASE
}

template <typename T>
hipError_t Ops<T>::apg_step(const Group& g, const Inst<T>* insts, const ApgState* sin, ApgState* sout, hipStream_t s) {
#define MAID_CASE(KV) \
    case KV: return apg_step_k<T, KV>(g, insts, sin, sout, s);
    MAID_K_SWITCH(MAID_CASE)
#undef MAID_CASE
}

template <typename T>
hipError_t Ops<T>::cg_step(const Group& g, const Inst<T>* insts, const CgState* sin, CgState* sout, hipStream_t s) {
#define MAID_CASE(KV) \
    case KV: return cg_step_k<T, KV>(g, insts, sin, sout, s);
    MAID_K_SWITCH(MAID_CASE)
#undef MAID_CASE
}

template <typename T>
hipError_t Ops<T>::apg_team(const Group& g, const Inst<T>* insts, const int* list, int nlist, ApgState* st,
                            const TeamCtl& ctl, long max_slots, hipStream_t s) {
#define MAID_CASE(KV) \
    case KV: return apg_team_k<T, KV>(g, insts, list, nlist, st, ctl, max_slots, s);
    MAID_K_SWITCH(MAID_CASE)
#undef MAID_CASE
}

template <typename T>
hipError_t Ops<T>::cg_team(const Group& g, const Inst<T>* insts, const int* list, int nlist, CgState* st, int n,
                           const TeamCtl& ctl, long max_slots, hipStream_t s) {
#define MAID_CASE(KV) \
    case KV: return cg_team_k<T, KV>(g, insts, list, nlist, st, n, ctl, max_slots, s);
    MAID_K_SWITCH(MAID_CASE)
#undef MAID_CASE
}

template <typename T>
hipError_t Ops<T>::team_occupancy(const Group& g, int* blocks_per_cu) {
#define MAID_CASE(KV) \
    case KV: return team_occupancy_k<T, KV>(g, blocks_per_cu);
    MAID_K_SWITCH(MAID_CASE)
#undef MAID_CASE
}

template <typename T>
hipError_t Ops<T>::apg_final(int grid_e, const int* blk_e, int only, const Inst<T>* insts, const ApgState* sin,
                             hipStream_t s) {
    return launch(k_apg_final<T>, dim3(grid_e), dim3(kNT), 0, s, insts, blk_e, only, sin);
}

template <typename T>
hipError_t Ops<T>::cg_update(int grid_e, const int* blk_e, int only, const Inst<T>* insts, const CgState* sin,
                             CgState* sout, hipStream_t s) {
    return launch(k_cg_update<T>, dim3(grid_e), dim3(kNT), 0, s, insts, blk_e, only, sin, sout);
}

template <typename T>
hipError_t Ops<T>::cg_init(int grid_e, const int* blk_e, int only, const Inst<T>* insts, const CgState* sin,
                           hipStream_t s) {
    return launch(k_cg_init<T>, dim3(grid_e), dim3(kNT), 0, s, insts, blk_e, only, sin);
}

template <typename T>
hipError_t Ops<T>::hg_corr_batch(int kt, int blocks, const Inst<T>* insts, int n, hipStream_t s) {
    if (kt == 16) return launch((k_hg_corr_batch<T, 16>), dim3(blocks), dim3(kNT), 0, s, insts, n);
    return launch((k_hg_corr_batch<T, 32>), dim3(blocks), dim3(kNT), 0, s, insts, n);
}

template <typename T>
hipError_t Ops<T>::hg_final_batch(int kt, const Inst<T>* insts, int n, hipStream_t s) {
    if (kt == 16) return launch((k_hg_final_batch<T, 16>), dim3(n), dim3(1024), 0, s, insts);
    return launch((k_hg_final_batch<T, 32>), dim3(n), dim3(1024), 0, s, insts);
}

// dst[i] = src[i] for `words` 32-bit words, src in host memory mapped for the
// device: the instance tables' upload as a kernel (no copy-engine call).
__global__ __launch_bounds__(kNT) void k_upload(const unsigned* __restrict__ src, int words, unsigned* __restrict__ dst) {
    const int stride = (int)gridDim.x * kNT * 4;
    for (int i0 = ((int)blockIdx.x * kNT + (int)threadIdx.x) * 4; i0 < words; i0 += stride) {
        unsigned v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = i0 + k < words ? src[i0 + k] : 0u;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (i0 + k < words) dst[i0 + k] = v[k];
    }
}

hipError_t launch_upload(const void* src_host, size_t bytes, void* dst, hipStream_t s) {
    const int words = (int)(bytes / 4);
    const int blocks = std::max(1, std::min(64, (words + 4 * kNT - 1) / (4 * kNT)));
    return launch(k_upload, dim3(blocks), dim3(kNT), 0, s, (const unsigned*)src_host, words, (unsigned*)dst);
}

// XCD (hardware XCC_ID) of every block of the grid.
__global__ __launch_bounds__(64) void k_team_map(int* out) {
    if (threadIdx.x == 0) out[blockIdx.x] = (int)(__builtin_amdgcn_s_getreg(20 | (0 << 6) | (3 << 11)) & 7u);
}

hipError_t launch_team_map(int* out, hipStream_t s) {
    return launch(k_team_map, dim3(kTeamXcd * kTeamMax), dim3(64), 0, s, out);
}

// Copy `words` 32-bit words of solver state into host-visible memory and
// then raise *flag: every thread's stores are made visible system-wide before
// the flag is written, so a host that sees the flag reads complete state.
__global__ __launch_bounds__(kNT) void k_publish(const unsigned* __restrict__ src, int words, unsigned* dst,
                                                 unsigned* flag) {
    for (int i = threadIdx.x; i < words; i += kNT) dst[i] = src[i];
    __threadfence_system();
    __syncthreads();
    if (threadIdx.x == 0) *(volatile unsigned*)flag = 1u;
}

hipError_t launch_publish(const void* src, size_t bytes, void* dst_host, unsigned* flag_host, hipStream_t s) {
    return launch(k_publish, dim3(1), dim3(kNT), 0, s, (const unsigned*)src, (int)(bytes / 4), (unsigned*)dst_host,
                  flag_host);
}

template struct Ops<float>;
template struct Ops<double>;

LaunchTiming& launch_timing() {
    static thread_local LaunchTiming t;
    return t;
}

int hg_items(const Shape& d) {
    return ((d.W + kHgTJ - 1) / kHgTJ) * ((d.H + kHgTI - 1) / kHgTI) * d.C * 2;
}

hipError_t launch_theta_step(const double* th, const double* z, double step, double* out, int KK, hipStream_t s) {
    return launch(k_theta_step, dim3((KK + 255) / 256), dim3(256), 0, s, th, z, step, out, KK);
}

hipError_t launch_sobolev(double beta, double h1_w0, const double* th, const double* a, int K, int kp, double* out,
                          hipStream_t s) {
    return launch(k_sobolev, dim3(1), dim3(1024), 0, s, beta, h1_w0, th, a, K, kp, out);
}

}  // namespace maid
