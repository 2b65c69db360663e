// ops.h -- host-side launchers of the libmaid kernels, one set per storage
// type.  Each dispatches the runtime kernel size K (odd, 1..31) and the
// rows-per-thread tile parameter R (1, 2, 4) to the matching template
// instantiation.  All launches are asynchronous on `s`.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "devctx.h"

namespace maid {

struct Shape {
    int C, H, W, K, reg;
};

inline int stencil_blocks(const Shape& d, int R) {
    return ((d.W + kTW - 1) / kTW) * ((d.H + tile_h(R) - 1) / tile_h(R));
}

inline bool valid_rows(int R) { return R == 1 || R == 2 || R == 4; }

template <typename T> struct Ops {
    static hipError_t prep_kernel(double* L_io, double* abs_out, const double* th, T* out, T* outf, int K, hipStream_t s);
    static hipError_t conv(const Shape& d, int R, const T* ker, const T* in, const T* sub, T* out, double* part,
                           hipStream_t s);
    static hipError_t apg_grad(const Shape& d, int R, const Params& p, const ApgState* sin, ApgState* sout,
                               const ApgBufs<T>& b, hipStream_t s);
    static hipError_t apg_trial(const Shape& d, int R, const Params& p, const ApgState* sin, ApgState* sout,
                                const ApgBufs<T>& b, hipStream_t s);
    static hipError_t apg_final(const ApgState* sin, const ApgBufs<T>& b, T* out, int64_t n, hipStream_t s);
    static hipError_t cg_dir(const Shape& d, int R, const Params& p, const CgState* sin, CgState* sout, const CgBufs<T>& b,
                             int init, hipStream_t s);
    static hipError_t cg_hvp(const Shape& d, int R, const Params& p, const CgState* sin, CgState* sout, const CgBufs<T>& b,
                             int init, hipStream_t s);
    static hipError_t cg_update(const CgState* sin, CgState* sout, const CgBufs<T>& b, int64_t n, int nblk, hipStream_t s);
    static hipError_t cg_init(const CgBufs<T>& b, int64_t n, int nblk, hipStream_t s);
    static hipError_t hg_corr(const Shape& d, const T* rho, const T* q, const T* w, const T* xt, double* part, int nblk,
                              hipStream_t s);
};

hipError_t launch_reduce(const double* part, int nb, double* out, hipStream_t s);
hipError_t launch_hg_final(const Shape& d, double beta, double h1_w0, const double* part, int nblk, const double* th,
                           const double* a, int with_r, double* z, double* znorm2, hipStream_t s);
hipError_t launch_theta_step(const double* th, const double* z, double step, double* out, int KK, hipStream_t s);
hipError_t launch_sobolev(double beta, double h1_w0, const double* th, const double* a, int K, double* out, hipStream_t s);
int hg_items(const Shape& d);

extern template struct Ops<float>;
extern template struct Ops<double>;

}  // namespace maid
