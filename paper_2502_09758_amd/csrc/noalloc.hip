// noalloc.hip -- the upper-level value and gradient without any allocation.
//
// maid_upper_value_grad_noalloc runs the kernels of maid_upper_value_grad
// (preparation of the kernel a, rho = a*x - y with its squared-norm
// partials, grad = a.rho with its partials, the finishing sums) on one
// instance described by a maid_desc, with no context: everything those
// kernels need beyond the caller's inputs and outputs -- the instance
// table, the kernel in the storage type, the per-block partial sums, the
// reduction slots and the residual image -- lives in `scratch`, a
// file-scope device array of kScratchBytes that every device the library
// runs on holds until the process ends.  The host takes its device address
// once per device with hipGetSymbolAddress and passes that address (never
// the array's host-side name) to the kernels; the instance table entries
// (laid out by host code in engine.cpp) go up as kernel arguments.  No call
// of this file allocates device or host memory.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "engine.h"
#include "maid.h"
#include "ops.h"

namespace maid {

constexpr size_t kScratchBytes = size_t(64) << 20;   // per device

// The workspace of maid_upper_value_grad_noalloc.  In host code this name
// is a stand-in, not a device address: host code uses the address that
// scratch_address() took with hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

// the two instance-table entries of the evaluation, written from kernel
// arguments (two entries stay well inside the 4 KiB of kernel arguments)
template <int NW>
__global__ void k_put_words(Words<NW> a, Words<NW> b, unsigned* dst) {
    for (int w = threadIdx.x; w < NW; w += blockDim.x) {
        dst[w] = a.w[w];
        dst[NW + w] = b.w[w];
    }
}

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// device address of `scratch` on the current device (taken once per device)
hipError_t scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

// Errors are reported through static strings: no path of the entry point
// allocates host memory either.
int reject(const char** why, int code, const char* msg) {
    if (why) *why = msg;
    return code;
}

template <typename T>
int upper_noalloc(const maid_desc* d, const double* a, const T* y, const T* x, T* grad_out, double* g_out,
                  double* gn_out, const char** why, hipStream_t s) {
    void* base = nullptr;
    hipError_t e = scratch_address(&base);
    if (e != hipSuccess) return reject(why, MAID_EHIP, "upper_value_grad_noalloc: the workspace address is unavailable");
    // the table entries, launch group and workspace layout (host code)
    NoallocUpper<T> job;
    if (int rc = noalloc_upper_setup<T>(d, a, y, x, grad_out, static_cast<char*>(base), kScratchBytes, &job, why))
        return rc;
    Inst<T>* tab = reinterpret_cast<Inst<T>*>(job.tab_dev);
    hipLaunchKernelGGL(k_put_words<kInstWords<T>>, dim3(1), dim3(64), 0, s, job.words[0], job.words[1],
                       reinterpret_cast<unsigned*>(job.tab_dev));
    e = hipGetLastError();
    if (e == hipSuccess) e = Ops<T>::prep_kernel(tab, 1, nullptr, nullptr, kRedAbs, s);
    if (e == hipSuccess) e = Ops<T>::conv(job.g, tab, s);
    if (e == hipSuccess) e = Ops<T>::conv(job.g, tab + 1, s);
    if (e == hipSuccess) e = Ops<T>::finish(tab + 1, 1, kRedGrad, kRedSob, s);
    double r[kRedSlots];
    if (e == hipSuccess) e = hipMemcpyAsync(r, job.red_dev, sizeof(r), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return reject(why, MAID_EHIP, "upper_value_grad_noalloc: a HIP call failed");
    if (!std::isfinite(r[kRedG]) || !std::isfinite(r[kRedGrad]))
        return reject(why, MAID_NONFINITE, "upper_value_grad_noalloc: non-finite value");
    if (g_out) *g_out = 0.5 * r[kRedG];
    if (gn_out) *gn_out = std::sqrt(r[kRedGrad]);
    return MAID_OK;
}

}  // namespace
}  // namespace maid

extern "C" int maid_upper_value_grad_noalloc(const maid_desc* desc, const void* a, const void* y, const void* x,
                                             void* grad_out, double* g_out, double* gradnorm_out, const char** why,
                                             hipStream_t stream) {
    using namespace maid;
    if (why) *why = "";
    if (const char* p = desc_problem(desc)) return reject(why, MAID_EINVAL, p);
    if (!a || !y || !x) return reject(why, MAID_EINVAL, "upper_value_grad_noalloc: NULL argument");
    if (desc->dtype == MAID_F64)
        return upper_noalloc<double>(desc, (const double*)a, (const double*)y, (const double*)x, (double*)grad_out, g_out,
                                     gradnorm_out, why, stream);
    return upper_noalloc<float>(desc, (const double*)a, (const float*)y, (const float*)x, (float*)grad_out, g_out,
                                gradnorm_out, why, stream);
}
