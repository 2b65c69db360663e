// d1.cpp -- host side of the 1D problem of Section 4.1 (maid1d.h): the
// context and its workspace, the batched solver loops over the kernels of
// d1.hip (per-instance states on the device, decided by the kernels; the
// host reads them back once per chunk of iterations), and Algorithm 2 in
// lockstep over the batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "d1.h"
#include "maid1d.h"

using namespace maid::d1;

struct maid1d_ctx {
    int n = 0, nb = 0;
    double a1 = 0.0, a2 = 0.0;
    char* ws = nullptr;
    // [nb][n] vectors
    double *X0 = nullptr, *X1 = nullptr, *r = nullptr, *u = nullptr, *hq = nullptr, *grad = nullptr;
    double *cq = nullptr, *cr = nullptr, *cp = nullptr, *chp = nullptr, *xs = nullptr;
    // [nb][n][n]: the trial matrix and z
    double *Bt = nullptr, *z = nullptr;
    // per-block partials: two vector-sized sets and the outer product's
    double *pa = nullptr, *pb = nullptr, *pz = nullptr;
    double* steps = nullptr;           // per-instance trial steps (device)
    ProxState* pst = nullptr;
    CgState1* cst = nullptr;
    int *done_p = nullptr, *cur = nullptr, *done_c = nullptr, *skip = nullptr;
    // pinned host mirrors
    char* host = nullptr;
    ProxState* pst_h = nullptr;
    CgState1* cst_h = nullptr;
    int* ints_h = nullptr;             // 4 nb: done_p, cur, done_c, skip
    double* steps_h = nullptr;
    double* part_h = nullptr;
    size_t part_cap = 0;               // doubles per partial buffer
    std::string err;
};

namespace {

thread_local std::string g_err1d;

int fail(maid1d_ctx* c, int code, const std::string& m) {
    if (c) c->err = m;
    return code;
}

#define D1_HIP(expr)                                                                                         \
    do {                                                                                                     \
        hipError_t e_ = (expr);                                                                              \
        if (e_ != hipSuccess)                                                                                \
            return fail(c, MAID_EHIP, std::string("HIP error in ") + #expr + ": " + hipGetErrorString(e_)); \
    } while (0)

#define D1_TRY(expr)          \
    do {                      \
        int rc_ = (expr);     \
        if (rc_ < 0) return rc_; \
    } while (0)

size_t al(size_t b) { return (b + 255) / 256 * 256; }

constexpr int kChunk = 16;   // iterations between read-backs of the solver states

// upload the int arrays (done_p, cur, done_c, skip) from their host mirror
int put_ints(maid1d_ctx* c, hipStream_t s) {
    D1_HIP(hipMemcpyAsync(c->done_p, c->ints_h, 4 * c->nb * sizeof(int), hipMemcpyHostToDevice, s));
    return MAID_OK;
}

// sum of `per` partials of each instance, in block order
void sum_parts(const double* h, int nb, int per, std::vector<double>& out) {
    out.assign(nb, 0.0);
    for (int b = 0; b < nb; ++b) {
        double s = 0.0;
        for (int k = 0; k < per; ++k) s += h[(size_t)b * per + k];
        out[b] = s;
    }
}

int read_parts(maid1d_ctx* c, const double* dev, int per, std::vector<double>& out, hipStream_t s) {
    D1_HIP(hipMemcpyAsync(c->part_h, dev, (size_t)c->nb * per * sizeof(double), hipMemcpyDeviceToHost, s));
    D1_HIP(hipStreamSynchronize(s));
    sum_parts(c->part_h, c->nb, per, out);
    return MAID_OK;
}

// ------------------------------------------------------------------ solvers
int lower(maid1d_ctx* c, const double* B, const double* y, double* x, double step, const double* tol, int max_iter,
          const std::vector<char>& act, maid_solve_info* info, hipStream_t s) {
    const int n = c->n, nb = c->nb;
    for (int b = 0; b < nb; ++b) {
        ProxState& p = c->pst_h[b];
        std::memset(&p, 0, sizeof(p));
        p.tol = tol[b];
        p.lam = step;
        p.max = max_iter;
        p.done = act[b] ? 0 : 1;
        c->ints_h[b] = p.done;          // done_p
        c->ints_h[nb + b] = 0;          // cur
        c->ints_h[3 * nb + b] = act[b] ? 0 : 1;
    }
    D1_HIP(hipMemcpyAsync(c->pst, c->pst_h, nb * sizeof(ProxState), hipMemcpyHostToDevice, s));
    D1_TRY(put_ints(c, s));
    D1_HIP(hipMemcpyAsync(c->X0, x, (size_t)nb * n * sizeof(double), hipMemcpyDeviceToDevice, s));
    Epi e{};
    e.mode = kProx;
    e.alpha1 = c->a1;
    e.alpha2 = c->a2;
    e.lam = step;
    e.xa = c->X0;
    e.xb = c->X1;
    e.cur = c->cur;
    const int64_t nn = (int64_t)n * n;
    long done_iters = 0;
    for (;;) {
        for (int k = 0; k < kChunk; ++k) {
            D1_HIP(gemv(B, nn, c->X0, c->X1, c->cur, n, nb, y, c->r, nullptr, c->done_p, s));
            D1_HIP(gemvt(B, nn, c->r, n, nb, e, nullptr, c->pa, c->done_p, s));
            D1_HIP(prox_decide(c->pst, c->pa, col_blocks(n), nb, c->done_p, c->cur, s));
        }
        done_iters += kChunk;
        D1_HIP(hipMemcpyAsync(c->pst_h, c->pst, nb * sizeof(ProxState), hipMemcpyDeviceToHost, s));
        D1_HIP(hipStreamSynchronize(s));
        bool all = true;
        for (int b = 0; b < nb; ++b) all = all && c->pst_h[b].done;
        if (all) break;
        if (done_iters > (long)max_iter + 2 * kChunk) return fail(c, MAID_EHIP, "lower_solve: iteration count lost");
    }
    D1_HIP(pick(c->X0, c->X1, c->cur, n, nb, x, c->skip, s));
    D1_HIP(hipStreamSynchronize(s));
    for (int b = 0; b < nb; ++b)
        if (info && act[b]) {
            const ProxState& p = c->pst_h[b];
            info[b] = maid_solve_info{p.iters, 0, p.status, p.res, 0.0, 1.0 / step};
        }
    return MAID_OK;
}

int adjoint(maid1d_ctx* c, const double* B, const double* x, const double* rhs, double* q, const double* tol,
            int max_iter, const std::vector<char>& act, maid_solve_info* info, hipStream_t s) {
    const int n = c->n, nb = c->nb;
    for (int b = 0; b < nb; ++b) {
        CgState1& p = c->cst_h[b];
        std::memset(&p, 0, sizeof(p));
        p.tol = tol[b];
        p.max = max_iter;
        p.first = 1;
        p.done = act[b] ? 0 : 1;
        c->ints_h[2 * nb + b] = p.done;
        c->ints_h[3 * nb + b] = act[b] ? 0 : 1;
    }
    D1_HIP(hipMemcpyAsync(c->cst, c->cst_h, nb * sizeof(CgState1), hipMemcpyHostToDevice, s));
    D1_TRY(put_ints(c, s));
    const int64_t nn = (int64_t)n * n;
    // q0 restricted to the support, then H q0 and the first residual
    D1_HIP(hipMemcpyAsync(c->cq, q, (size_t)nb * n * sizeof(double), hipMemcpyDeviceToDevice, s));
    D1_HIP(cg_setup(x, rhs, rhs, c->cq, c->cr, c->cp, n, nb, c->pa, c->done_c, s));   // masks q (r, p overwritten below)
    Epi e{};
    e.mode = kHvp;
    e.alpha2 = c->a2;
    e.p = c->cq;
    e.xsup = x;
    D1_HIP(gemv(B, nn, c->cq, c->cq, nullptr, n, nb, nullptr, c->u, nullptr, c->done_c, s));
    D1_HIP(gemvt(B, nn, c->u, n, nb, e, c->hq, nullptr, c->done_c, s));
    D1_HIP(cg_setup(x, rhs, c->hq, c->cq, c->cr, c->cp, n, nb, c->pa, c->done_c, s));
    e.p = c->cp;
    long done_iters = 0;
    for (;;) {
        for (int k = 0; k < kChunk; ++k) {
            D1_HIP(cg_gamma(c->cst, c->pa, ew_blocks(n), nb, c->done_c, s));
            D1_HIP(cg_dir(c->cst, c->cr, c->cp, n, nb, s));
            D1_HIP(gemv(B, nn, c->cp, c->cp, nullptr, n, nb, nullptr, c->u, nullptr, c->done_c, s));
            D1_HIP(gemvt(B, nn, c->u, n, nb, e, c->chp, c->pb, c->done_c, s));
            D1_HIP(cg_alpha(c->cst, c->pb, col_blocks(n), nb, c->done_c, s));
            D1_HIP(cg_update(c->cst, c->cp, c->chp, c->cq, c->cr, n, nb, c->pa, s));
        }
        done_iters += kChunk;
        D1_HIP(hipMemcpyAsync(c->cst_h, c->cst, nb * sizeof(CgState1), hipMemcpyDeviceToHost, s));
        D1_HIP(hipStreamSynchronize(s));
        bool all = true;
        for (int b = 0; b < nb; ++b) all = all && c->cst_h[b].done;
        if (all) break;
        if (done_iters > (long)max_iter + 2 * kChunk) return fail(c, MAID_EHIP, "adjoint_solve: iteration count lost");
    }
    // the solution of every active instance that did not fail
    for (int b = 0; b < nb; ++b)
        c->ints_h[3 * nb + b] = (act[b] && c->cst_h[b].status >= 0) ? 0 : 1;
    D1_TRY(put_ints(c, s));
    D1_HIP(pick(c->cq, c->cq, c->cur, n, nb, q, c->skip, s));
    D1_HIP(hipStreamSynchronize(s));
    for (int b = 0; b < nb; ++b)
        if (info && act[b]) {
            const CgState1& p = c->cst_h[b];
            info[b] = maid_solve_info{p.iters, 0, p.status, p.res, 0.0, 0.0};
        }
    return MAID_OK;
}

int upper(maid1d_ctx* c, const double* A, const double* y, const double* x, double* grad, double* g, double* gn,
          const std::vector<char>& act, hipStream_t s) {
    const int n = c->n, nb = c->nb;
    for (int b = 0; b < nb; ++b) c->ints_h[3 * nb + b] = act[b] ? 0 : 1;
    D1_TRY(put_ints(c, s));
    D1_HIP(gemv(A, 0, x, x, nullptr, n, nb, y, c->r, c->pa, c->skip, s));
    Epi e{};
    e.mode = kGrad;
    D1_HIP(gemvt(A, 0, c->r, n, nb, e, grad ? grad : c->grad, c->pb, c->skip, s));
    std::vector<double> sg, sn;
    D1_TRY(read_parts(c, c->pa, row_blocks(n), sg, s));
    D1_TRY(read_parts(c, c->pb, col_blocks(n), sn, s));
    for (int b = 0; b < nb; ++b)
        if (act[b]) {
            if (g) g[b] = 0.5 * sg[b];
            if (gn) gn[b] = std::sqrt(sn[b]);
        }
    return MAID_OK;
}

int hyper(maid1d_ctx* c, const double* B, const double* y, const double* x, const double* q, double* z, double* zn,
          const std::vector<char>& act, hipStream_t s) {
    const int n = c->n, nb = c->nb;
    for (int b = 0; b < nb; ++b) c->ints_h[3 * nb + b] = act[b] ? 0 : 1;
    D1_TRY(put_ints(c, s));
    const int64_t nn = (int64_t)n * n;
    D1_HIP(gemv(B, nn, x, x, nullptr, n, nb, y, c->r, nullptr, c->skip, s));
    D1_HIP(gemv(B, nn, q, q, nullptr, n, nb, nullptr, c->u, nullptr, c->skip, s));
    D1_HIP(outer(c->r, q, c->u, x, n, nb, z, c->pz, c->skip, s));
    std::vector<double> sz;
    D1_TRY(read_parts(c, c->pz, n * ew_blocks(n), sz, s));
    for (int b = 0; b < nb; ++b)
        if (act[b] && zn) zn[b] = std::sqrt(sz[b]);
    return MAID_OK;
}

bool bad_tol(double t) { return !(t >= 0.0) || !std::isfinite(t); }

}  // namespace

// ====================================================================== C ABI
extern "C" {

int maid1d_create(const maid1d_desc* d, maid1d_ctx** out) {
    if (!out) {
        g_err1d = "out is NULL";
        return MAID_EINVAL;
    }
    *out = nullptr;
    if (!d) {
        g_err1d = "desc is NULL";
        return MAID_EINVAL;
    }
    if (d->n < 1 || d->n > kMaxN) {
        g_err1d = "n must be in 1.." + std::to_string(kMaxN);
        return MAID_EINVAL;
    }
    if (d->batch < 1) {
        g_err1d = "batch must be >= 1";
        return MAID_EINVAL;
    }
    if (!(d->alpha1 >= 0.0) || !std::isfinite(d->alpha1) || !(d->alpha2 > 0.0) || !std::isfinite(d->alpha2)) {
        g_err1d = "need alpha1 >= 0 and alpha2 > 0 (finite)";
        return MAID_EINVAL;
    }
    auto* c = new maid1d_ctx;
    c->n = d->n;
    c->nb = d->batch;
    c->a1 = d->alpha1;
    c->a2 = d->alpha2;
    const size_t n = (size_t)c->n, nb = (size_t)c->nb;
    const size_t vec = al(nb * n * sizeof(double)), mat = al(nb * n * n * sizeof(double));
    c->part_cap = std::max<size_t>(nb * n * ew_blocks(c->n), nb * (size_t)std::max(row_blocks(c->n), ew_blocks(c->n)));
    const size_t part = al(c->part_cap * sizeof(double));
    const size_t bytes = 11 * vec + 2 * mat + 3 * part + al(nb * sizeof(double)) + al(nb * sizeof(ProxState)) +
                         al(nb * sizeof(CgState1)) + al(4 * nb * sizeof(int));
    hipError_t e = hipMalloc((void**)&c->ws, bytes);
    if (e != hipSuccess) {
        delete c;
        g_err1d = std::string("allocation failed: ") + hipGetErrorString(e);
        return e == hipErrorOutOfMemory ? MAID_ENOMEM : MAID_EHIP;
    }
    char* p = c->ws;
    auto take = [&](size_t b) { char* r = p; p += b; return (void*)r; };
    double** vecs[] = {&c->X0, &c->X1, &c->r, &c->u, &c->hq, &c->grad, &c->cq, &c->cr, &c->cp, &c->chp, &c->xs};
    for (double** v : vecs) *v = (double*)take(vec);
    c->Bt = (double*)take(mat);
    c->z = (double*)take(mat);
    c->pa = (double*)take(part);
    c->pb = (double*)take(part);
    c->pz = (double*)take(part);
    c->steps = (double*)take(al(nb * sizeof(double)));
    c->pst = (ProxState*)take(al(nb * sizeof(ProxState)));
    c->cst = (CgState1*)take(al(nb * sizeof(CgState1)));
    int* ints = (int*)take(al(4 * nb * sizeof(int)));
    c->done_p = ints;
    c->cur = ints + nb;
    c->done_c = ints + 2 * nb;
    c->skip = ints + 3 * nb;
    const size_t hbytes = al(nb * sizeof(ProxState)) + al(nb * sizeof(CgState1)) + al(4 * nb * sizeof(int)) +
                          al(nb * sizeof(double)) + part;
    e = hipHostMalloc((void**)&c->host, hbytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMemset(c->ws, 0, bytes);
    if (e != hipSuccess) {
        maid1d_destroy(c);
        g_err1d = std::string("allocation failed: ") + hipGetErrorString(e);
        return MAID_EHIP;
    }
    std::memset(c->host, 0, hbytes);
    char* h = c->host;
    c->pst_h = (ProxState*)h;
    h += al(nb * sizeof(ProxState));
    c->cst_h = (CgState1*)h;
    h += al(nb * sizeof(CgState1));
    c->ints_h = (int*)h;
    h += al(4 * nb * sizeof(int));
    c->steps_h = (double*)h;
    h += al(nb * sizeof(double));
    c->part_h = (double*)h;
    *out = c;
    return MAID_OK;
}

void maid1d_destroy(maid1d_ctx* c) {
    if (!c) return;
    if (c->ws) (void)hipFree(c->ws);
    if (c->host) (void)hipHostFree(c->host);
    delete c;
}

const char* maid1d_last_error(const maid1d_ctx* c) { return c ? c->err.c_str() : g_err1d.c_str(); }

int maid1d_lower_solve(maid1d_ctx* c, const double* B, const double* y, double* x, double step, const double* tol,
                       int32_t max_iter, maid_solve_info* info, hipStream_t s) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    if (!B || !y || !x || !tol) return fail(c, MAID_EINVAL, "lower_solve: NULL argument");
    if (!(step > 0.0) || !std::isfinite(step)) return fail(c, MAID_EINVAL, "lower_solve: step must be finite and > 0");
    if (max_iter < 0) return fail(c, MAID_EINVAL, "lower_solve: max_iter must be >= 0");
    for (int b = 0; b < c->nb; ++b)
        if (bad_tol(tol[b])) return fail(c, MAID_EINVAL, "lower_solve: tolerances must be finite and >= 0");
    std::vector<maid_solve_info> inf(c->nb);
    D1_TRY(lower(c, B, y, x, step, tol, max_iter, std::vector<char>(c->nb, 1), inf.data(), s));
    int code = MAID_OK;
    for (int b = 0; b < c->nb; ++b) {
        if (info) info[b] = inf[b];
        if (code == MAID_OK && inf[b].status != MAID_OK) code = inf[b].status;
    }
    if (code < 0) return fail(c, code, "lower_solve: non-finite values met");
    return code;
}

int maid1d_upper_value_grad(maid1d_ctx* c, const double* A, const double* y, const double* x, double* grad_out,
                            double* g_out, double* gradnorm_out, hipStream_t s) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    if (!A || !y || !x) return fail(c, MAID_EINVAL, "upper_value_grad: NULL argument");
    return upper(c, A, y, x, grad_out, g_out, gradnorm_out, std::vector<char>(c->nb, 1), s);
}

int maid1d_adjoint_solve(maid1d_ctx* c, const double* B, const double* x, const double* rhs, double* q, const double* tol,
                         int32_t max_iter, maid_solve_info* info, hipStream_t s) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    if (!B || !x || !rhs || !q || !tol) return fail(c, MAID_EINVAL, "adjoint_solve: NULL argument");
    if (max_iter < 0) return fail(c, MAID_EINVAL, "adjoint_solve: max_iter must be >= 0");
    for (int b = 0; b < c->nb; ++b)
        if (bad_tol(tol[b])) return fail(c, MAID_EINVAL, "adjoint_solve: tolerances must be finite and >= 0");
    std::vector<maid_solve_info> inf(c->nb);
    D1_TRY(adjoint(c, B, x, rhs, q, tol, max_iter, std::vector<char>(c->nb, 1), inf.data(), s));
    int code = MAID_OK;
    for (int b = 0; b < c->nb; ++b) {
        if (info) info[b] = inf[b];
        if (code == MAID_OK && inf[b].status != MAID_OK) code = inf[b].status;
    }
    if (code == MAID_NOT_SPD) return fail(c, code, "adjoint_solve: curvature <p,Hp> <= 0");
    if (code < 0) return fail(c, code, "adjoint_solve: non-finite values met");
    return code;
}

int maid1d_hypergrad(maid1d_ctx* c, const double* B, const double* y, const double* x, const double* q, double* z,
                     double* znorm_out, hipStream_t s) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    if (!B || !y || !x || !q || !z) return fail(c, MAID_EINVAL, "hypergrad: NULL argument");
    return hyper(c, B, y, x, q, z, znorm_out, std::vector<char>(c->nb, 1), s);
}

int maid1d_step(maid1d_ctx* c, const double* A, const double* y, double* B, double* x, double* q, maid1d_sched* sc,
                const maid_hparams* hp, double lam_x, maid_step_info* infos, hipStream_t s) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    if (!A || !y || !B || !x || !q || !sc || !hp) return fail(c, MAID_EINVAL, "step: NULL argument");
    if (!(hp->rho_lo > 0 && hp->rho_lo < 1) || !(hp->nu_lo > 0 && hp->nu_lo < 1) || !(hp->rho_hi > 1) || !(hp->nu_hi > 1) ||
        hp->max_bt < 1 || hp->max_lower_iter < 0 || hp->max_cg_iter < 0 || !(hp->lambda > 0) || !(hp->mu > 0) ||
        !(hp->eps_min > 0))
        return fail(c, MAID_EINVAL, "step: bad hyperparameters");
    if (!(lam_x > 0.0) || !std::isfinite(lam_x)) return fail(c, MAID_EINVAL, "step: lam_x must be finite and > 0");
    const int n = c->n, nb = c->nb;
    for (int b = 0; b < nb; ++b)
        if (!(sc[b].eps > 0) || !(sc[b].delta > 0) || !(sc[b].step > 0))
            return fail(c, MAID_EINVAL, "step: eps, delta, step must be > 0");
    // L_g: the caller's, else ||A||_1 ||A||_inf from a host copy of A
    double Lg = hp->L_g;
    if (!(Lg > 0)) {
        std::vector<double> Ah((size_t)n * n);
        D1_HIP(hipMemcpyAsync(Ah.data(), A, Ah.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        D1_HIP(hipStreamSynchronize(s));
        double c1 = 0.0, ci = 0.0;
        for (int j = 0; j < n; ++j) {
            double sc1 = 0.0;
            for (int i = 0; i < n; ++i) sc1 += std::fabs(Ah[(size_t)i * n + j]);
            c1 = std::max(c1, sc1);
        }
        for (int i = 0; i < n; ++i) {
            double si = 0.0;
            for (int j = 0; j < n; ++j) si += std::fabs(Ah[(size_t)i * n + j]);
            ci = std::max(ci, si);
        }
        Lg = c1 * ci;
    }
    const size_t nn = (size_t)n * n;
    std::vector<maid_step_info> I(nb);
    std::memset(I.data(), 0, nb * sizeof(maid_step_info));
    std::vector<int> codes(nb, MAID_OK), j(nb, hp->max_bt);
    std::vector<char> need(nb, 1);
    std::vector<double> tol(nb), g_k(nb), n_k(nb), zn(nb), g_n(nb), n_n(nb);
    std::vector<maid_solve_info> li(nb), ci(nb);
    auto any = [](const std::vector<char>& v) {
        for (char a : v)
            if (a) return true;
        return false;
    };
    while (any(need)) {
        // InexactGradient(B_k, eps_k, delta_k)
        for (int b = 0; b < nb; ++b) tol[b] = sc[b].eps * hp->mu;
        D1_TRY(lower(c, B, y, x, lam_x, tol.data(), hp->max_lower_iter, need, li.data(), s));
        for (int b = 0; b < nb; ++b)
            if (need[b]) {
                I[b].lower_iters += li[b].iters;
                if (li[b].status < 0) {
                    codes[b] = li[b].status;
                    need[b] = 0;
                } else if (li[b].status == MAID_MAXITER) {
                    I[b].lower_status = MAID_MAXITER;
                }
            }
        D1_TRY(upper(c, A, y, x, c->grad, g_k.data(), n_k.data(), need, s));
        for (int b = 0; b < nb; ++b) tol[b] = sc[b].delta;
        D1_TRY(adjoint(c, B, x, c->grad, q, tol.data(), hp->max_cg_iter, need, ci.data(), s));
        for (int b = 0; b < nb; ++b)
            if (need[b]) {
                I[b].cg_iters += ci[b].iters;
                if (ci[b].status < 0) {
                    codes[b] = ci[b].status;
                    need[b] = 0;
                } else if (ci[b].status == MAID_MAXITER) {
                    I[b].cg_status = MAID_MAXITER;
                }
            }
        D1_TRY(hyper(c, B, y, x, q, c->z, zn.data(), need, s));
        for (int b = 0; b < nb; ++b)
            if (need[b]) {
                I[b].ell_k = g_k[b];
                I[b].znorm = zn[b];
            }
        // backtracking on the step size: instances try in lockstep
        std::vector<char> trying = need;
        std::vector<int> t(nb, 0);
        for (int b = 0; b < nb; ++b) tol[b] = sc[b].eps * hp->mu;
        while (any(trying)) {
            for (int b = 0; b < nb; ++b) {
                c->steps_h[b] = sc[b].step;
                c->ints_h[3 * nb + b] = trying[b] ? 0 : 1;
            }
            D1_HIP(hipMemcpyAsync(c->steps, c->steps_h, nb * sizeof(double), hipMemcpyHostToDevice, s));
            D1_TRY(put_ints(c, s));
            D1_HIP(mat_step(B, c->z, c->steps, n, nb, c->Bt, c->skip, s));
            D1_HIP(hipMemcpyAsync(c->xs, x, (size_t)nb * n * sizeof(double), hipMemcpyDeviceToDevice, s));
            D1_TRY(lower(c, c->Bt, y, c->xs, lam_x, tol.data(), hp->max_lower_iter, trying, li.data(), s));
            D1_TRY(upper(c, A, y, c->xs, nullptr, g_n.data(), n_n.data(), trying, s));
            for (int b = 0; b < nb; ++b) {
                if (!trying[b]) continue;
                I[b].lower_iters += li[b].iters;
                if (li[b].status == MAID_MAXITER) I[b].lower_status = MAID_MAXITER;
                const double e = sc[b].eps;
                const double psi = g_n[b] + n_n[b] * e + 0.5 * Lg * e * e - g_k[b] + n_k[b] * e +
                                   hp->lambda * sc[b].step * zn[b] * zn[b];
                I[b].trials += 1;
                I[b].psi = psi;
                I[b].ell_next = g_n[b];
                if (li[b].status < 0) {
                    codes[b] = li[b].status;
                    trying[b] = 0;
                    need[b] = 0;
                    continue;
                }
                if (psi <= 0.0) {
                    D1_HIP(hipMemcpyAsync(B + b * nn, c->Bt + b * nn, nn * sizeof(double), hipMemcpyDeviceToDevice, s));
                    D1_HIP(hipMemcpyAsync(x + (size_t)b * n, c->xs + (size_t)b * n, n * sizeof(double),
                                          hipMemcpyDeviceToDevice, s));
                    sc[b].eps *= hp->nu_hi;
                    sc[b].delta *= hp->nu_hi;
                    sc[b].step *= hp->rho_hi;
                    sc[b].k += 1;
                    trying[b] = 0;
                    need[b] = 0;
                    I[b].accepted = 1;
                } else {
                    sc[b].step *= hp->rho_lo;
                    if (++t[b] >= j[b]) trying[b] = 0;
                }
            }
        }
        for (int b = 0; b < nb; ++b) {
            if (!need[b]) continue;
            sc[b].eps *= hp->nu_lo;
            sc[b].delta *= hp->nu_lo;
            j[b] += 1;
            I[b].retries += 1;
            if (sc[b].eps < hp->eps_min) {
                codes[b] = MAID_ACCURACY_FLOOR;
                need[b] = 0;
            }
        }
    }
    D1_HIP(hipStreamSynchronize(s));
    int code = MAID_OK;
    for (int b = 0; b < nb; ++b) {
        if (codes[b] == MAID_OK && (I[b].lower_status == MAID_MAXITER || I[b].cg_status == MAID_MAXITER))
            codes[b] = MAID_MAXITER;
        I[b].status = codes[b];
        if (infos) infos[b] = I[b];
        if (code == MAID_OK && codes[b] != MAID_OK) code = codes[b];
    }
    if (code < 0) return fail(c, code, "step: a solve failed");
    return code;
}

}  // extern "C"
