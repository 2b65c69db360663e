// adp.cpp -- the two ADP baselines of Section 4.1 (ADP-IFT and ADP-LISTA)
// on the library's kernels, beside MAID: the fixed-step lower-level
// iteration they share, Proposition 1's Hessian applied to a vector, and one
// upper-level iteration of each.
//
// Both baselines run the proximal-gradient iteration of Section 4.1 with a
// fixed step lambda_x on the lower level; with the smooth TV regulariser of
// the 2D problem its proximal map is the identity, so an iteration is
//   x_{k+1} = x_k - lambda_x grad_x h(x_k; theta),
// run here by the FISTA passes with the momentum off and every step accepted
// (L = 1/lambda_x).
//   ADP-IFT: a fixed number of those iterations (warm-started), the
//     implicit-function hypergradient (CG on the Hessian system, Eq. 3.2),
//     a gradient step on theta.
//   ADP-LISTA: a fixed number of iterations whose iterates are kept, the
//     gradient of g(x_n(theta)) + r(theta) through them in reverse
//       w_n = grad g(x_n),  dtheta += lambda_x * z(x_k, w_{k+1}),
//       w_k = w_{k+1} - lambda_x H(x_k) w_{k+1},
//     with z(x, w) = -(d grad_x h / d theta)^T w the hypergradient's
//     correlation, then a gradient step on theta.  Here w carries the factor
//     lambda_x from the start (the recursion is linear), so every
//     correlation gives lambda_x z directly and the Sobolev gradient of r
//     joins the first one.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "engine.h"
#include "maid.h"
#include "ops.h"

namespace maid {

namespace {

#define ADP_HIP(expr)                                                                                        \
    do {                                                                                                     \
        hipError_t e_ = (expr);                                                                              \
        if (e_ != hipSuccess)                                                                                \
            return fail(c, MAID_EHIP, std::string("HIP error in ") + #expr + ": " + hipGetErrorString(e_)); \
    } while (0)

#define ADP_TRY(expr)           \
    do {                        \
        int rc_ = (expr);       \
        if (rc_ < 0) return rc_; \
    } while (0)

template <typename P> std::vector<P> one(P p) { return std::vector<P>(1, p); }

// the fixed-step mode of the lower-level passes for one call
struct FixedStep {
    maid_ctx* c;
    FixedStep(maid_ctx* cc, void* hist) : c(cc) {
        c->lower_fixed = true;
        c->lower_hist = hist;
    }
    ~FixedStep() {
        c->lower_fixed = false;
        c->lower_hist = nullptr;
    }
};

// the baselines' workspace, grown to `bytes`
int adp_workspace(maid_ctx* c, size_t bytes) {
    if (c->adp_ws_bytes >= bytes) return MAID_OK;
    if (c->adp_ws) {
        ADP_HIP(hipDeviceSynchronize());
        ADP_HIP(hipFree(c->adp_ws));
        c->adp_ws = nullptr;
        c->adp_ws_bytes = 0;
    }
    hipError_t e = hipMalloc((void**)&c->adp_ws, bytes);
    if (e == hipErrorOutOfMemory) return fail(c, MAID_ENOMEM, "ADP baselines: workspace allocation failed");
    ADP_HIP(e);
    c->adp_ws_bytes = bytes;
    return MAID_OK;
}

size_t al256(size_t b) { return (b + 255) / 256 * 256; }

// the upper-level loss g(x) + r(theta) and ||grad g|| (FP64 scalars), grad g
// into grad
template <typename T>
int upper_loss(maid_ctx* c, const double* theta, const double* a, const T* y, const T* x, T* grad, double* loss,
               double* gn, hipStream_t s) {
    double g = 0.0, r = 0.0;
    ADP_TRY(upper_batch<T>(c, one<char>(1), one<const double*>(a), one<const T*>(y), one<const T*>(x), one<T*>(grad),
                           &g, gn, s));
    ADP_TRY(sobolev_batch(c, one<char>(1), one<const double*>(theta), one<const double*>(a), &r, s));
    *loss = g + r;
    return MAID_OK;
}

}  // namespace

template <typename T>
int gd_one(maid_ctx* c, const double* theta, const T* y, T* x, double step, int n_iter, double tol, T* hist,
           maid_solve_info* info, hipStream_t s) {
    if (hist && c->m[0].nbf > 0)
        return fail(c, MAID_EINVAL,
                    "gd_solve: keeping the iterates needs the two-pass lower-level form (maid_set_one_pass(ctx, 0))");
    FixedStep fs(c, hist);
    double L = 1.0 / step;
    int code = MAID_OK;
    maid_solve_info inf{};
    ADP_TRY(lower_batch<T>(c, one<char>(1), one<const double*>(theta), one<const T*>(y), one<T*>(x), one<double>(tol),
                           n_iter, &L, &inf, &code, nullptr, s));
    if (info) *info = inf;
    if (code < 0) return fail(c, code, "gd_solve: non-finite values met");
    return code;
}

template <typename T>
int ift_step_one(maid_ctx* c, const double* a, const T* y, maid_state* st, int n_lower, double lambda_x,
                 double cg_tol, int max_cg, maid_step_info* info, hipStream_t s) {
    const Member& M = c->m[0];
    double* theta = (double*)st->theta;
    T* x = (T*)st->x;
    T* q = (T*)st->q;
    T* grad = (T*)M.gradg;
    maid_step_info I{};
    // lower level: n_lower fixed-step iterations from the warm start
    maid_solve_info li{};
    const int lc = gd_one<T>(c, theta, y, x, lambda_x, n_lower, 0.0, nullptr, &li, s);
    if (lc < 0) return lc;
    I.lower_iters = li.iters;
    // upper level at x: the loss and grad g, the CG right-hand side
    double loss = 0.0, gn = 0.0;
    ADP_TRY(upper_loss<T>(c, theta, a, y, x, grad, &loss, &gn, s));
    // adjoint: H(x) q = grad g to cg_tol relative, from the previous q
    maid_solve_info ci{};
    int code = MAID_OK;
    ADP_TRY(adjoint_batch<T>(c, one<char>(1), one<const double*>(theta), one<const T*>(x), one<const T*>(grad),
                             one<T*>(q), one<double>(cg_tol * gn), max_cg, &ci, &code, s));
    if (code < 0) return fail(c, code, "ift_step: adjoint solve failed");
    I.cg_iters = ci.iters;
    I.cg_status = code;
    // hypergradient and the step on theta
    double* z = M.zbuf;
    double zn = 0.0;
    ADP_TRY(hypergrad_batch<T>(c, one<char>(1), one<const double*>(theta), one<const double*>(a), one<const T*>(y),
                               one<const T*>(x), one<const T*>(q), 1, one<double*>(z), &zn, s));
    ADP_HIP(launch_theta_step(theta, z, st->step, theta, kplanes(M.d) * M.d.K * M.d.K, s));
    ADP_HIP(hipStreamSynchronize(s));
    st->k += 1;
    I.accepted = 1;
    I.trials = 1;
    I.ell_k = loss;
    I.znorm = zn;
    I.status = code == MAID_MAXITER ? MAID_MAXITER : MAID_OK;
    if (info) *info = I;
    return I.status;
}

template <typename T>
int lista_step_one(maid_ctx* c, const double* a, const T* y, maid_state* st, int n_unroll, double lambda_x,
                   maid_step_info* info, hipStream_t s) {
    const Member& M = c->m[0];
    if (M.nbf > 0)
        return fail(c, MAID_EINVAL,
                    "lista_step: the unrolled iterates need the two-pass lower-level form (maid_set_one_pass(ctx, 0))");
    const size_t N = (size_t)M.N;
    const int KK = kplanes(M.d) * M.d.K * M.d.K;
    // workspace: x_0 .. x_n (dense, x_k at xs + k N: the passes write x_{k+1}
    // at hist + k N), w, H w, the accumulated gradient, one z, partials
    const size_t img = al256(N * sizeof(T));
    const size_t hist_bytes = al256((size_t)(n_unroll + 1) * N * sizeof(T));
    const size_t need = hist_bytes + 2 * img + 2 * al256(KK * sizeof(double)) + al256(2 * 512 * sizeof(double));
    ADP_TRY(adp_workspace(c, need));
    char* p = c->adp_ws;
    T* xs = (T*)p;
    const size_t stride = N;
    p += hist_bytes;
    T* w = (T*)p;
    p += img;
    T* hw = (T*)p;
    p += img;
    double* acc = (double*)p;
    p += al256(KK * sizeof(double));
    double* z = (double*)p;
    p += al256(KK * sizeof(double));
    double* part = (double*)p;
    double* theta = (double*)st->theta;
    T* x = (T*)st->x;
    maid_step_info I{};
    // forward: x_0 kept, x_1 .. x_n written by the passes
    ADP_HIP(hipMemcpyAsync(xs, x, N * sizeof(T), hipMemcpyDeviceToDevice, s));
    maid_solve_info li{};
    const int lc = gd_one<T>(c, theta, y, x, lambda_x, n_unroll, 0.0, xs + stride, &li, s);
    if (lc < 0) return lc;
    if (li.iters != n_unroll) return fail(c, MAID_EHIP, "lista_step: the forward iteration stopped early");
    I.lower_iters = li.iters;
    // loss and w_n = lambda_x grad g(x_n)
    double loss = 0.0, gn = 0.0;
    T* grad = (T*)M.gradg;
    ADP_TRY(upper_loss<T>(c, theta, a, y, x, grad, &loss, &gn, s));
    ADP_HIP(hipMemsetAsync(w, 0, N * sizeof(T), s));
    ADP_HIP(launch_axpy_norms<T>(w, grad, (T)lambda_x, (int64_t)N, part, 512, s));
    // reverse sweep
    ADP_HIP(hipMemsetAsync(acc, 0, KK * sizeof(double), s));
    for (int k = n_unroll - 1; k >= 0; --k) {
        const T* xk = xs + (size_t)k * stride;
        double zn = 0.0;
        ADP_TRY(hypergrad_batch<T>(c, one<char>(1), one<const double*>(theta), one<const double*>(a), one<const T*>(y),
                                   one<const T*>(xk), one<const T*>(w), k == n_unroll - 1 ? 1 : 0, one<double*>(z),
                                   &zn, s));
        ADP_HIP(launch_theta_step(acc, z, -1.0, acc, KK, s));
        if (k == 0) break;
        ADP_TRY(hessian_one<T>(c, theta, xk, w, hw, s));
        ADP_HIP(launch_axpy_norms<T>(w, hw, (T)(-lambda_x), (int64_t)N, part, 512, s));
        I.cg_iters += 1;
    }
    // theta <- theta - step * dtheta; ||dtheta|| from the host copy
    std::vector<double> acc_h(KK);
    ADP_HIP(hipMemcpyAsync(acc_h.data(), acc, KK * sizeof(double), hipMemcpyDeviceToHost, s));
    ADP_HIP(launch_theta_step(theta, acc, st->step, theta, KK, s));
    ADP_HIP(hipStreamSynchronize(s));
    double zz = 0.0;
    for (double v : acc_h) zz += v * v;
    st->k += 1;
    I.accepted = 1;
    I.trials = 1;
    I.ell_k = loss;
    I.znorm = std::sqrt(zz);
    I.status = MAID_OK;
    if (info) *info = I;
    return MAID_OK;
}

#define MAID_ADP_INSTANTIATE(T)                                                                                   \
    template int gd_one<T>(maid_ctx*, const double*, const T*, T*, double, int, double, T*, maid_solve_info*,     \
                           hipStream_t);                                                                          \
    template int ift_step_one<T>(maid_ctx*, const double*, const T*, maid_state*, int, double, double, int,       \
                                 maid_step_info*, hipStream_t);                                                   \
    template int lista_step_one<T>(maid_ctx*, const double*, const T*, maid_state*, int, double, maid_step_info*, \
                                   hipStream_t);

MAID_ADP_INSTANTIATE(float)
MAID_ADP_INSTANTIATE(double)

}  // namespace maid
