// api.cpp -- the C ABI of libmaid (include/maid.h): context and workspace
// management, argument checking, and the host side of the solvers.
//
// The host side only enqueues kernels and polls: every arithmetic step runs
// on the GPU, and every solver decision (stop tests, backtracking, CG
// coefficients) is taken on the GPU by the pass that consumes the
// reduction, and kept in the device-resident DevCtx.  Solver passes are
// replayed in chunks from captured HIP graphs; the host copies the small
// solver state back once per chunk to learn whether the solve has finished.
// MAID's outer loop (Algorithm 2) runs on the host over scalars that the
// kernels computed in FP64.  Setting MAID_GRAPHS=0 in the environment
// launches the passes directly instead of through graphs.
#include "maid.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "devctx.h"
#include "ops.h"

using namespace maid;

struct maid_ctx {
    maid_desc d;
    Shape shape;
    int64_t N = 0;
    size_t esz = 0;
    int R_auto = 1, R_override = 0;
    DevCtx* dev = nullptr;    // device-resident solver state
    DevCtx* host = nullptr;   // pinned host mirror
    char* ws = nullptr;       // one device allocation for all scratch
    size_t ws_bytes = 0;
    void* X[3] = {};
    void* KX[3] = {};
    void* G = nullptr;
    void* cq = nullptr;
    void* cr = nullptr;
    void* cP[2] = {};
    void* cKp = nullptr;
    void* cHp = nullptr;
    void* tmp0 = nullptr;
    void* tmp1 = nullptr;
    void* xtrial = nullptr;
    void* gradg = nullptr;
    void* th_c = nullptr;
    void* thf_c = nullptr;
    void* a_c = nullptr;
    void* af_c = nullptr;
    double* th_trial = nullptr;
    double* zbuf = nullptr;
    double* pA = nullptr;      // per-block partials: gradient pass
    double* pB = nullptr;      //                     trial pass
    double* pR = nullptr;      //                     CG residual
    double* pK = nullptr;      //                     CG curvature
    double* pC = nullptr;      //                     convolution passes
    double* hg_part = nullptr;
    int ew_blocks = 0;
    hipStream_t cap = nullptr; // private stream for graph capture
    bool use_graphs = true;
    struct Graph { int kind; const void* k1; const void* k2; int chunk; int R; hipGraphExec_t exec; };
    std::vector<Graph> graphs;
    int* trace = nullptr;
    int trace_cap = 0;
    std::string err;
    std::string cfg;
    // per-launch timing with HIP events on the launch stream
    bool prof_on = false;
    struct Rec { int kind; hipEvent_t a, b; };
    std::vector<Rec> prof_pending;
    std::vector<hipEvent_t> prof_pool;
    int64_t prof_launches[MAID_PROF_KINDS] = {};
    double prof_ms[MAID_PROF_KINDS] = {};

    int R() const { return R_override ? R_override : R_auto; }
    Params params() const { return Params{d.C, d.H, d.W, d.reg, d.alpha, d.eps_tv}; }
    double* red(int k) const { return &dev->red[k]; }
};

namespace {

thread_local std::string g_create_error;

constexpr int kTraceCap = 1 << 16;
constexpr int kHgMaxBlocks = 512;
constexpr int kRedG = 0, kRedGrad = 1, kRedZ = 2, kRedSob = 3, kRedAbs = 4;

int fail(maid_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                               \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            return fail(c, MAID_EHIP, std::string("HIP error in ") + #expr + ": " + hipGetErrorString(e_)); \
    } while (0)

int auto_rows(const Shape& d) {
    // the largest tile height that still gives every CU (256) four blocks
    if (stencil_blocks(d, 4) >= 1024) return 4;
    if (stencil_blocks(d, 2) >= 1024) return 2;
    return 1;
}

bool finite(double v) { return std::isfinite(v); }

int validate_desc(const maid_desc* d, std::string& why) {
    if (!d) { why = "desc is NULL"; return MAID_EINVAL; }
    if (d->H < 1 || d->W < 1) { why = "H and W must be >= 1"; return MAID_EINVAL; }
    if (d->C < 1 || d->C > kMaxC) { why = "C must be 1, 2 or 3"; return MAID_EINVAL; }
    if (d->K < 1 || d->K > kMaxK || (d->K % 2) == 0) { why = "K must be odd, 1 <= K <= 31"; return MAID_EINVAL; }
    if (d->K > d->H || d->K > d->W) { why = "K must not exceed H or W"; return MAID_EINVAL; }
    if (d->dtype != MAID_F32 && d->dtype != MAID_F64) { why = "dtype must be MAID_F32 or MAID_F64"; return MAID_EINVAL; }
    if (d->reg < 0 || d->reg > 2) { why = "reg must be 0, 1 or 2"; return MAID_EINVAL; }
    if (!finite(d->alpha) || d->alpha < 0) { why = "alpha must be finite and >= 0"; return MAID_EINVAL; }
    if (d->reg != MAID_REG_QUADRATIC && !(d->eps_tv > 0 && finite(d->eps_tv))) { why = "eps_tv must be > 0"; return MAID_EINVAL; }
    if (!finite(d->beta) || d->beta < 0) { why = "beta must be finite and >= 0"; return MAID_EINVAL; }
    if (!finite(d->h1_w0) || d->h1_w0 < 0) { why = "h1_w0 must be finite and >= 0"; return MAID_EINVAL; }
    const double n = (double)d->H * d->W * d->C;
    if (n > 4.0e9) { why = "image too large"; return MAID_EINVAL; }
    return MAID_OK;
}

// copy a field range of the device state to / from the pinned mirror
int pull(maid_ctx* c, hipStream_t s, size_t off, size_t n) {
    HIP_TRY(hipMemcpyAsync((char*)c->host + off, (char*)c->dev + off, n, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return MAID_OK;
}
int push(maid_ctx* c, hipStream_t s, size_t off, size_t n) {
    HIP_TRY(hipMemcpyAsync((char*)c->dev + off, (char*)c->host + off, n, hipMemcpyHostToDevice, s));
    return MAID_OK;
}
constexpr size_t kOffApg = offsetof(DevCtx, apg);
constexpr size_t kOffCg = offsetof(DevCtx, cg);
constexpr size_t kOffRed = offsetof(DevCtx, red);

int status_code(int st) {
    switch (st) {
        case ST_OK: return MAID_OK;
        case ST_MAXITER: return MAID_MAXITER;
        case ST_NOT_SPD: return MAID_NOT_SPD;
        default: return MAID_NONFINITE;
    }
}

// ------------------------------------------------------------------ profiling
hipEvent_t prof_event(maid_ctx* c) {
    if (!c->prof_pool.empty()) {
        hipEvent_t e = c->prof_pool.back();
        c->prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Accumulate the durations of recorded launches (waits for the last one).
void prof_harvest(maid_ctx* c) {
    if (c->prof_pending.empty()) return;
    (void)hipEventSynchronize(c->prof_pending.back().b);
    for (auto& r : c->prof_pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            c->prof_launches[r.kind] += 1;
            c->prof_ms[r.kind] += ms;
        }
        c->prof_pool.push_back(r.a);
        c->prof_pool.push_back(r.b);
    }
    c->prof_pending.clear();
}

struct ProfScope {
    maid_ctx* c;
    int kind;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(maid_ctx* c_, int k, hipStream_t s_) : c(c_), kind(k), s(s_) {
        if (!c->prof_on) return;
        a = prof_event(c);
        b = prof_event(c);
        if (a) (void)hipEventRecord(a, s);
    }
    ~ProfScope() {
        if (!c->prof_on || !a || !b) return;
        (void)hipEventRecord(b, s);
        c->prof_pending.push_back({kind, a, b});
        if (c->prof_pending.size() >= 4096) prof_harvest(c);
    }
};

// Launch expression `expr` (returning hipError_t) timed as `kind`.
#define LAUNCH(kind, expr)                       \
    do {                                         \
        ProfScope ps_(c, (kind), s);             \
        HIP_TRY(expr);                           \
    } while (0)

// ------------------------------------------------------------------ graph-captured chunks
// A chunk of solver passes is captured once into a HIP graph (per kind, the
// caller pointers the launches embed, chunk length and tile rows) and
// replayed; the passes read everything that changes between replays from
// the device-resident state.  With profiling on, passes launch directly so
// that each one is bracketed by its own events.
enum { G_APG = 1, G_CG = 2 };

template <typename F>
int run_chunk(maid_ctx* c, int kind, const void* k1, const void* k2, int chunk, hipStream_t s, F enqueue) {
    if (c->prof_on || !c->use_graphs) return enqueue(s);
    const int R = c->R();
    for (auto& g : c->graphs)
        if (g.kind == kind && g.k1 == k1 && g.k2 == k2 && g.chunk == chunk && g.R == R) {
            HIP_TRY(hipGraphLaunch(g.exec, s));
            return MAID_OK;
        }
    HIP_TRY(hipStreamBeginCapture(c->cap, hipStreamCaptureModeRelaxed));
    int rc = enqueue(c->cap);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(c->cap, &graph);
    if (rc != MAID_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return fail(c, MAID_EHIP, std::string("graph capture failed: ") + hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(c, MAID_EHIP, std::string("graph instantiation failed: ") + hipGetErrorString(e));
    if (c->graphs.size() >= 48) {
        (void)hipGraphExecDestroy(c->graphs.front().exec);
        c->graphs.erase(c->graphs.begin());
    }
    c->graphs.push_back({kind, k1, k2, chunk, R, exec});
    HIP_TRY(hipGraphLaunch(exec, s));
    return MAID_OK;
}

// ------------------------------------------------------------------ lower level
template <typename T>
int lower_solve_t(maid_ctx* c, const double* theta, const T* y, T* x, double tol, int max_iter, double* L_inout,
                  maid_solve_info* info, int32_t* trace_bt, hipStream_t s) {
    const Shape& d = c->shape;
    const int R = c->R();
    ApgState& h = c->host->apg[0];
    std::memset(&h, 0, sizeof(h));
    h.L = *L_inout;
    h.t = 1.0;
    h.t_prev = 1.0;
    h.m = 0.0;
    h.tol = tol;
    h.max_iter = max_iter;
    h.status = ST_OK;
    h.phase = PH_START;
    h.cur = 0;
    h.prev = 1;
    h.nxt = 2;
    h.trace_cap = c->trace_cap;
    int rc = push(c, s, kOffApg, sizeof(ApgState));
    if (rc) return rc;
    T* th = (T*)c->th_c;
    T* thf = (T*)c->thf_c;
    LAUNCH(MAID_PROF_OTHER, Ops<T>::prep_kernel(&c->dev->apg[0].L, nullptr, theta, th, thf, d.K, s));
    const size_t bytes = (size_t)c->N * sizeof(T);
    HIP_TRY(hipMemcpyAsync(c->X[0], x, bytes, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(c->X[1], x, bytes, hipMemcpyDeviceToDevice, s));
    LAUNCH(MAID_PROF_CONV, Ops<T>::conv(d, R, thf, (const T*)c->X[0], nullptr, (T*)c->KX[0], nullptr, s));
    HIP_TRY(hipMemcpyAsync(c->KX[1], c->KX[0], bytes, hipMemcpyDeviceToDevice, s));
    ApgBufs<T> b;
    for (int i = 0; i < 3; ++i) {
        b.X[i] = (T*)c->X[i];
        b.KX[i] = (T*)c->KX[i];
    }
    b.G = (T*)c->G;
    b.y = y;
    b.th = th;
    b.thf = thf;
    b.pA = c->pA;
    b.pB = c->pB;
    b.nbA = b.nbB = stencil_blocks(d, R);
    b.trace = c->trace;
    // each slot is one gradient pass and one trial pass; a slot advances the
    // solve by one iteration or by one backtracking step
    const long slot_cap = (long)max_iter + 256 + 1;
    const Params pr = c->params();
    long slots = 0;
    int chunk = 1;
    for (;;) {
        rc = run_chunk(c, G_APG, y, nullptr, chunk, s, [&](hipStream_t s) {
            for (int k = 0; k < chunk; ++k) {
                LAUNCH(MAID_PROF_APG_GRAD, Ops<T>::apg_grad(d, R, pr, &c->dev->apg[0], &c->dev->apg[1], b, s));
                LAUNCH(MAID_PROF_APG_TRIAL, Ops<T>::apg_trial(d, R, pr, &c->dev->apg[1], &c->dev->apg[0], b, s));
            }
            return (int)MAID_OK;
        });
        if (rc) return rc;
        slots += chunk;
        rc = pull(c, s, kOffApg, sizeof(ApgState));
        if (rc) return rc;
        if (h.done) break;
        if (slots > slot_cap) return fail(c, MAID_NONFINITE, "lower_solve: backtracking did not terminate");
        chunk = std::min(chunk * 2, 16);
    }
    const int code = status_code(h.status);
    if (code >= 0) {
        LAUNCH(MAID_PROF_OTHER, Ops<T>::apg_final(&c->dev->apg[0], b, x, c->N, s));
        HIP_TRY(hipStreamSynchronize(s));
        *L_inout = h.L;
    }
    if (trace_bt && h.iters > 0) {
        const int n = std::min(h.iters, c->trace_cap);
        HIP_TRY(hipMemcpy(trace_bt, c->trace, n * sizeof(int), hipMemcpyDeviceToHost));
    }
    if (info) {
        info->iters = h.iters;
        info->backtracks = h.bt;
        info->status = code;
        info->res_norm = std::sqrt(h.gn2);
        info->obj = 0.0;
        info->L = h.L;
    }
    if (code < 0) return fail(c, code, "lower_solve: non-finite values met");
    return code;
}

template <typename T>
int upper_value_grad_t(maid_ctx* c, const double* a, const T* y, const T* x, T* grad_out, double* g_out, double* gn_out,
                       hipStream_t s) {
    const Shape& d = c->shape;
    const int R = c->R();
    const int nb = stencil_blocks(d, R);
    T* ac = (T*)c->a_c;
    T* af = (T*)c->af_c;
    LAUNCH(MAID_PROF_OTHER, Ops<T>::prep_kernel(nullptr, nullptr, a, ac, af, d.K, s));
    LAUNCH(MAID_PROF_CONV, Ops<T>::conv(d, R, af, x, y, (T*)c->tmp0, c->pC, s));
    LAUNCH(MAID_PROF_OTHER, launch_reduce(c->pC, nb, c->red(kRedG), s));
    T* gout = grad_out ? grad_out : (T*)c->gradg;
    LAUNCH(MAID_PROF_CONV, Ops<T>::conv(d, R, ac, (const T*)c->tmp0, nullptr, gout, c->pC, s));
    LAUNCH(MAID_PROF_OTHER, launch_reduce(c->pC, nb, c->red(kRedGrad), s));
    int rc = pull(c, s, kOffRed, sizeof(c->host->red));
    if (rc) return rc;
    if (g_out) *g_out = 0.5 * c->host->red[kRedG];
    if (gn_out) *gn_out = std::sqrt(c->host->red[kRedGrad]);
    return MAID_OK;
}

// ------------------------------------------------------------------ adjoint (CG)
template <typename T>
int adjoint_solve_t(maid_ctx* c, const double* theta, const T* xt, const T* rhs, T* q, double tol, int max_iter,
                    maid_solve_info* info, hipStream_t s) {
    const Shape& d = c->shape;
    const int R = c->R();
    CgState& h = c->host->cg[0];
    std::memset(&h, 0, sizeof(h));
    h.tol = tol;
    h.max = max_iter;
    h.status = ST_OK;
    h.first = 1;
    int rc = push(c, s, kOffCg, sizeof(CgState));
    if (rc) return rc;
    T* th = (T*)c->th_c;
    T* thf = (T*)c->thf_c;
    LAUNCH(MAID_PROF_OTHER, Ops<T>::prep_kernel(nullptr, nullptr, theta, th, thf, d.K, s));
    const size_t bytes = (size_t)c->N * sizeof(T);
    HIP_TRY(hipMemcpyAsync(c->cq, q, bytes, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(c->cr, q, bytes, hipMemcpyDeviceToDevice, s));
    CgBufs<T> b;
    b.q = (T*)c->cq;
    b.r = (T*)c->cr;
    b.P[0] = (T*)c->cP[0];
    b.P[1] = (T*)c->cP[1];
    b.Kp = (T*)c->cKp;
    b.Hp = (T*)c->cHp;
    b.xt = xt;
    b.b = rhs;
    b.th = th;
    b.thf = thf;
    b.pR = c->pR;
    b.pK = c->pK;
    b.nbK = stencil_blocks(d, R);
    b.nbR = c->ew_blocks;
    // r = rhs - H q0 (the direction pass in set-up mode copies q0 into p)
    const Params pr = c->params();
    CgState* S = c->dev->cg;
    LAUNCH(MAID_PROF_CG_DIR, Ops<T>::cg_dir(d, R, pr, &S[0], &S[1], b, 1, s));
    LAUNCH(MAID_PROF_CG_HVP, Ops<T>::cg_hvp(d, R, pr, &S[0], &S[2], b, 1, s));
    LAUNCH(MAID_PROF_OTHER, Ops<T>::cg_init(b, c->N, c->ew_blocks, s));
    int chunk = 1;
    long slots = 0;
    for (;;) {
        rc = run_chunk(c, G_CG, xt, rhs, chunk, s, [&](hipStream_t s) {
            for (int k = 0; k < chunk; ++k) {
                LAUNCH(MAID_PROF_CG_DIR, Ops<T>::cg_dir(d, R, pr, &S[0], &S[1], b, 0, s));
                LAUNCH(MAID_PROF_CG_HVP, Ops<T>::cg_hvp(d, R, pr, &S[1], &S[2], b, 0, s));
                LAUNCH(MAID_PROF_CG_UPDATE, Ops<T>::cg_update(&S[2], &S[0], b, c->N, c->ew_blocks, s));
            }
            return (int)MAID_OK;
        });
        if (rc) return rc;
        slots += chunk;
        rc = pull(c, s, kOffCg, sizeof(CgState));
        if (rc) return rc;
        if (h.done) break;
        if (slots > (long)max_iter + 2) return fail(c, MAID_EHIP, "adjoint_solve: iteration count lost");
        chunk = std::min(chunk * 2, 16);
    }
    const int code = status_code(h.status);
    if (code >= 0) {
        HIP_TRY(hipMemcpyAsync(q, c->cq, bytes, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    if (info) {
        info->iters = h.iters;
        info->backtracks = 0;
        info->status = code;
        info->res_norm = std::sqrt(h.gamma);
        info->obj = 0.0;
        info->L = 0.0;
    }
    if (code < 0) return fail(c, code, code == MAID_NOT_SPD ? "adjoint_solve: curvature <p,Hp> <= 0" : "adjoint_solve: non-finite values met");
    return code;
}

// ------------------------------------------------------------------ hypergradient
template <typename T>
int hypergrad_t(maid_ctx* c, const double* theta, const double* a, const T* y, const T* xt, const T* q, int with_r, double* z,
                double* znorm_out, hipStream_t s) {
    const Shape& d = c->shape;
    const int R = c->R();
    T* th = (T*)c->th_c;
    T* thf = (T*)c->thf_c;
    LAUNCH(MAID_PROF_OTHER, Ops<T>::prep_kernel(nullptr, nullptr, theta, th, thf, d.K, s));
    const int nblk = std::min(kHgMaxBlocks, hg_items(d));
    LAUNCH(MAID_PROF_CONV, Ops<T>::conv(d, R, thf, xt, y, (T*)c->tmp0, nullptr, s));
    LAUNCH(MAID_PROF_CONV, Ops<T>::conv(d, R, thf, q, nullptr, (T*)c->tmp1, nullptr, s));
    LAUNCH(MAID_PROF_HG_CORR, Ops<T>::hg_corr(d, (const T*)c->tmp0, q, (const T*)c->tmp1, xt, c->hg_part, nblk, s));
    LAUNCH(MAID_PROF_OTHER, launch_hg_final(d, c->d.beta, c->d.h1_w0, c->hg_part, nblk, theta, with_r ? a : nullptr, with_r, z,
                                            c->red(kRedZ), s));
    int rc = pull(c, s, kOffRed, sizeof(c->host->red));
    if (rc) return rc;
    if (znorm_out) *znorm_out = std::sqrt(c->host->red[kRedZ]);
    return MAID_OK;
}

template <typename T>
int apply_operator_t(maid_ctx* c, const double* theta, const T* in, T* out, int adjoint, hipStream_t s) {
    const Shape& d = c->shape;
    T* th = (T*)c->th_c;
    T* thf = (T*)c->thf_c;
    LAUNCH(MAID_PROF_OTHER, Ops<T>::prep_kernel(nullptr, nullptr, theta, th, thf, d.K, s));
    LAUNCH(MAID_PROF_CONV, Ops<T>::conv(d, c->R(), adjoint ? th : thf, in, nullptr, out, nullptr, s));
    HIP_TRY(hipStreamSynchronize(s));
    return MAID_OK;
}

int sobolev_value_impl(maid_ctx* c, const double* theta, const double* a, double* r, hipStream_t s) {
    if (c->d.beta == 0.0) {
        *r = 0.0;
        return MAID_OK;
    }
    LAUNCH(MAID_PROF_OTHER, launch_sobolev(c->d.beta, c->d.h1_w0, theta, a, c->d.K, c->red(kRedSob), s));
    int rc = pull(c, s, kOffRed, sizeof(c->host->red));
    if (rc) return rc;
    *r = c->host->red[kRedSob];
    return MAID_OK;
}

// ------------------------------------------------------------------ MAID (Algorithm 2)
template <typename T>
int maid_step_t(maid_ctx* c, const double* a, const T* y, maid_state* st, const maid_hparams* hp, maid_step_info* out,
                hipStream_t s) {
    const int KK = c->d.K * c->d.K;
    double* theta = (double*)st->theta;
    T* x = (T*)st->x;
    T* q = (T*)st->q;
    T* xs = (T*)c->xtrial;
    T* grad = (T*)c->gradg;
    double* z = c->zbuf;
    double* th2 = c->th_trial;
    const size_t bytes = (size_t)c->N * sizeof(T);
    maid_step_info I;
    std::memset(&I, 0, sizeof(I));
    double Lg = hp->L_g;
    if (!(Lg > 0)) {
        LAUNCH(MAID_PROF_OTHER, Ops<T>::prep_kernel(nullptr, c->red(kRedAbs), a, (T*)c->a_c, (T*)c->af_c, c->d.K, s));
        int rc = pull(c, s, kOffRed, sizeof(c->host->red));
        if (rc) return rc;
        Lg = c->host->red[kRedAbs] * c->host->red[kRedAbs];
    }
    int status = MAID_OK;
    int j = hp->max_bt;
    for (;;) {
        // InexactGradient(theta_k, eps_k, delta_k)
        maid_solve_info li, ci;
        int rc = lower_solve_t<T>(c, theta, y, x, st->eps * hp->mu, hp->max_lower_iter, &st->L, &li, nullptr, s);
        if (rc < 0) { status = rc; break; }
        I.lower_iters += li.iters;
        double g_k, n_k, r_k;
        rc = upper_value_grad_t<T>(c, a, y, x, grad, &g_k, &n_k, s);
        if (rc) { status = rc; break; }
        rc = sobolev_value_impl(c, theta, a, &r_k, s);
        if (rc) { status = rc; break; }
        const double ell_k = g_k + r_k;
        rc = adjoint_solve_t<T>(c, theta, x, grad, q, st->delta, hp->max_cg_iter, &ci, s);
        I.cg_iters += ci.iters;
        if (rc < 0) { status = rc; break; }
        double znorm;
        rc = hypergrad_t<T>(c, theta, a, y, x, q, 1, z, &znorm, s);
        if (rc) { status = rc; break; }
        I.ell_k = ell_k;
        I.znorm = znorm;
        bool accepted = false;
        for (int i = 0; i < j; ++i) {
            LAUNCH(MAID_PROF_OTHER, launch_theta_step(theta, z, st->step, th2, KK, s));
            HIP_TRY(hipMemcpyAsync(xs, x, bytes, hipMemcpyDeviceToDevice, s));
            rc = lower_solve_t<T>(c, th2, y, xs, st->eps * hp->mu, hp->max_lower_iter, &st->L, &li, nullptr, s);
            if (rc < 0) { status = rc; break; }
            I.lower_iters += li.iters;
            double g_n, n_n, r_n;
            rc = upper_value_grad_t<T>(c, a, y, xs, nullptr, &g_n, &n_n, s);
            if (rc) { status = rc; break; }
            rc = sobolev_value_impl(c, th2, a, &r_n, s);
            if (rc) { status = rc; break; }
            const double ell_n = g_n + r_n;
            const double e = st->eps;
            const double psi = ell_n + n_n * e + 0.5 * Lg * e * e - ell_k + n_k * e + hp->lambda * st->step * znorm * znorm;
            I.trials += 1;
            I.psi = psi;
            I.ell_next = ell_n;
            if (psi <= 0.0) {
                HIP_TRY(hipMemcpyAsync(theta, th2, KK * sizeof(double), hipMemcpyDeviceToDevice, s));
                HIP_TRY(hipMemcpyAsync(x, xs, bytes, hipMemcpyDeviceToDevice, s));
                HIP_TRY(hipStreamSynchronize(s));
                st->eps *= hp->nu_hi;
                st->delta *= hp->nu_hi;
                st->step *= hp->rho_hi;
                st->k += 1;
                accepted = true;
                break;
            }
            st->step *= hp->rho_lo;
        }
        if (status < 0) break;
        if (accepted) {
            I.accepted = 1;
            break;
        }
        st->eps *= hp->nu_lo;
        st->delta *= hp->nu_lo;
        j += 1;
        I.retries += 1;
        if (st->eps < hp->eps_min) {
            status = MAID_ACCURACY_FLOOR;
            break;
        }
    }
    I.status = status;
    if (out) *out = I;
    return status;
}

bool bad_tol(double t) { return !(t >= 0.0) || !std::isfinite(t); }

}  // namespace

// ====================================================================== C ABI
extern "C" {

int maid_create(const maid_desc* desc, maid_ctx** out) {
    if (!out) {
        g_create_error = "out is NULL";
        return MAID_EINVAL;
    }
    *out = nullptr;
    std::string why;
    int rc = validate_desc(desc, why);
    if (rc) {
        g_create_error = why;
        return rc;
    }
    maid_ctx* c = new maid_ctx();
    c->d = *desc;
    c->shape = Shape{desc->C, desc->H, desc->W, desc->K, desc->reg};
    c->N = (int64_t)desc->C * desc->H * desc->W;
    c->esz = desc->dtype == MAID_F64 ? 8 : 4;
    c->R_auto = auto_rows(c->shape);
    c->ew_blocks = (int)std::min<int64_t>((c->N + kNT - 1) / kNT, 2048);
    c->trace_cap = kTraceCap;
    const size_t img = ((size_t)c->N * c->esz + 255) / 256 * 256;
    const size_t kern = 1024 * 8;
    const size_t nblk = std::max<size_t>(stencil_blocks(c->shape, 1), (size_t)c->ew_blocks);
    const size_t part = ((nblk * sizeof(double)) + 255) / 256 * 256;
    const size_t hgp = (size_t)kHgMaxBlocks * 1024 * sizeof(double);
    c->ws_bytes = 18 * img + 6 * kern + 5 * part + hgp + kTraceCap * sizeof(int);
    hipError_t e = hipMalloc((void**)&c->ws, c->ws_bytes);
    if (e != hipSuccess) {
        g_create_error = std::string("hipMalloc of the workspace failed: ") + hipGetErrorString(e);
        delete c;
        return e == hipErrorOutOfMemory ? MAID_ENOMEM : MAID_EHIP;
    }
    char* p = c->ws;
    auto take = [&](size_t n) { char* r = p; p += n; return (void*)r; };
    for (int i = 0; i < 3; ++i) c->X[i] = take(img);
    for (int i = 0; i < 3; ++i) c->KX[i] = take(img);
    c->G = take(img);
    c->cq = take(img);
    c->cr = take(img);
    c->cP[0] = take(img);
    c->cP[1] = take(img);
    c->cKp = take(img);
    c->cHp = take(img);
    c->tmp0 = take(img);
    c->tmp1 = take(img);
    c->xtrial = take(img);
    c->gradg = take(img);
    take(img);  // spare
    c->th_c = take(kern);
    c->thf_c = take(kern);
    c->a_c = take(kern);
    c->af_c = take(kern);
    c->th_trial = (double*)take(kern);
    c->zbuf = (double*)take(kern);
    c->pA = (double*)take(part);
    c->pB = (double*)take(part);
    c->pR = (double*)take(part);
    c->pK = (double*)take(part);
    c->pC = (double*)take(part);
    c->hg_part = (double*)take(hgp);
    c->trace = (int*)take(kTraceCap * sizeof(int));
    e = hipMalloc((void**)&c->dev, sizeof(DevCtx));
    if (e == hipSuccess) e = hipHostMalloc((void**)&c->host, sizeof(DevCtx), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMemset(c->ws, 0, c->ws_bytes);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking);
    if (const char* g = std::getenv("MAID_GRAPHS")) c->use_graphs = std::strcmp(g, "0") != 0;
    if (e != hipSuccess) {
        g_create_error = std::string("allocation failed: ") + hipGetErrorString(e);
        maid_destroy(c);
        return MAID_EHIP;
    }
    std::memset(c->host, 0, sizeof(DevCtx));
    DevCtx* h = c->host;
    h->C = desc->C;
    h->H = desc->H;
    h->W = desc->W;
    h->K = desc->K;
    h->reg = desc->reg;
    h->alpha = desc->alpha;
    h->eps_tv = desc->eps_tv;
    h->beta = desc->beta;
    h->h1_w0 = desc->h1_w0;
    e = hipMemcpy(c->dev, c->host, sizeof(DevCtx), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        g_create_error = std::string("hipMemcpy failed: ") + hipGetErrorString(e);
        maid_destroy(c);
        return MAID_EHIP;
    }
    char buf[128];
    std::snprintf(buf, sizeof(buf), "rows_per_thread=%d tile=64x%d", c->R(), tile_h(c->R()));
    c->cfg = buf;
    *out = c;
    return MAID_OK;
}

void maid_destroy(maid_ctx* c) {
    if (!c) return;
    prof_harvest(c);
    for (hipEvent_t e : c->prof_pool) (void)hipEventDestroy(e);
    for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    if (c->ws) (void)hipFree(c->ws);
    if (c->dev) (void)hipFree(c->dev);
    if (c->host) (void)hipHostFree(c->host);
    delete c;
}

const char* maid_last_error(const maid_ctx* c) {
    if (!c) return g_create_error.c_str();
    return c->err.c_str();
}

const char* maid_config_string(const maid_ctx* c) {
    if (!c) return "";
    return c->cfg.c_str();
}

int maid_set_tile_rows(maid_ctx* c, int32_t rows) {
    if (!c) return MAID_EINVAL;
    if (rows != 0 && !valid_rows(rows)) return fail(c, MAID_EINVAL, "rows per thread must be 0, 1, 2 or 4");
    c->R_override = rows;
    char buf[128];
    std::snprintf(buf, sizeof(buf), "rows_per_thread=%d tile=64x%d", c->R(), tile_h(c->R()));
    c->cfg = buf;
    return MAID_OK;
}

int maid_profile(maid_ctx* c, int32_t enable) {
    if (!c) return MAID_EINVAL;
    prof_harvest(c);
    for (int k = 0; k < MAID_PROF_KINDS; ++k) {
        c->prof_launches[k] = 0;
        c->prof_ms[k] = 0.0;
    }
    c->prof_on = enable != 0;
    return MAID_OK;
}

int maid_profile_read(maid_ctx* c, int32_t kind, int64_t* launches, double* total_ms) {
    if (!c || kind < 0 || kind >= MAID_PROF_KINDS || !launches || !total_ms) return MAID_EINVAL;
    prof_harvest(c);
    *launches = c->prof_launches[kind];
    *total_ms = c->prof_ms[kind];
    return MAID_OK;
}

const char* maid_profile_name(int32_t kind) {
    static const char* names[MAID_PROF_KINDS] = {"conv", "apg_grad", "apg_trial", "cg_dir", "cg_hvp",
                                                  "cg_update", "hg_corr", "other"};
    if (kind < 0 || kind >= MAID_PROF_KINDS) return "";
    return names[kind];
}

int maid_lower_solve(maid_ctx* c, const void* theta, const void* y, void* x, double tol, int32_t max_iter, double* L_inout,
                     maid_solve_info* info, int32_t* trace_bt, hipStream_t s) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    if (!theta || !y || !x || !L_inout) return fail(c, MAID_EINVAL, "lower_solve: NULL argument");
    if (bad_tol(tol)) return fail(c, MAID_EINVAL, "lower_solve: tol must be finite and >= 0");
    if (max_iter < 0) return fail(c, MAID_EINVAL, "lower_solve: max_iter must be >= 0");
    if (trace_bt && max_iter > c->trace_cap) return fail(c, MAID_EINVAL, "lower_solve: max_iter exceeds the trace capacity");
    if (!std::isfinite(*L_inout)) return fail(c, MAID_EINVAL, "lower_solve: L must be finite");
    if (c->d.dtype == MAID_F64)
        return lower_solve_t<double>(c, (const double*)theta, (const double*)y, (double*)x, tol, max_iter, L_inout, info, trace_bt, s);
    return lower_solve_t<float>(c, (const double*)theta, (const float*)y, (float*)x, tol, max_iter, L_inout, info, trace_bt, s);
}

int maid_upper_value_grad(maid_ctx* c, const void* a, const void* y, const void* x, void* grad_out, double* g_out,
                          double* gradnorm_out, hipStream_t s) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    if (!a || !y || !x) return fail(c, MAID_EINVAL, "upper_value_grad: NULL argument");
    if (c->d.dtype == MAID_F64)
        return upper_value_grad_t<double>(c, (const double*)a, (const double*)y, (const double*)x, (double*)grad_out, g_out,
                                          gradnorm_out, s);
    return upper_value_grad_t<float>(c, (const double*)a, (const float*)y, (const float*)x, (float*)grad_out, g_out,
                                     gradnorm_out, s);
}

int maid_adjoint_solve(maid_ctx* c, const void* theta, const void* x_tilde, const void* rhs, void* q, double tol,
                       int32_t max_iter, maid_solve_info* info, hipStream_t s) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    if (!theta || !x_tilde || !rhs || !q) return fail(c, MAID_EINVAL, "adjoint_solve: NULL argument");
    if (bad_tol(tol)) return fail(c, MAID_EINVAL, "adjoint_solve: tol must be finite and >= 0");
    if (max_iter < 0) return fail(c, MAID_EINVAL, "adjoint_solve: max_iter must be >= 0");
    if (c->d.dtype == MAID_F64)
        return adjoint_solve_t<double>(c, (const double*)theta, (const double*)x_tilde, (const double*)rhs, (double*)q, tol,
                                       max_iter, info, s);
    return adjoint_solve_t<float>(c, (const double*)theta, (const float*)x_tilde, (const float*)rhs, (float*)q, tol, max_iter,
                                  info, s);
}

int maid_hypergrad(maid_ctx* c, const void* theta, const void* a, const void* y, const void* x_tilde, const void* q,
                   int32_t with_r, double* z, double* znorm_out, hipStream_t s) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    if (!theta || !y || !x_tilde || !q || !z) return fail(c, MAID_EINVAL, "hypergrad: NULL argument");
    if (with_r && c->d.beta != 0.0 && !a) return fail(c, MAID_EINVAL, "hypergrad: a is needed for the Sobolev term");
    if (c->d.dtype == MAID_F64)
        return hypergrad_t<double>(c, (const double*)theta, (const double*)a, (const double*)y, (const double*)x_tilde,
                                   (const double*)q, with_r && c->d.beta != 0.0, z, znorm_out, s);
    return hypergrad_t<float>(c, (const double*)theta, (const double*)a, (const float*)y, (const float*)x_tilde,
                              (const float*)q, with_r && c->d.beta != 0.0, z, znorm_out, s);
}

int maid_apply_operator(maid_ctx* c, const void* theta, const void* in, void* out, int32_t adjoint, hipStream_t s) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    if (!theta || !in || !out) return fail(c, MAID_EINVAL, "apply_operator: NULL argument");
    if (in == out) return fail(c, MAID_EINVAL, "apply_operator: in and out must not alias");
    if (c->d.dtype == MAID_F64)
        return apply_operator_t<double>(c, (const double*)theta, (const double*)in, (double*)out, adjoint, s);
    return apply_operator_t<float>(c, (const double*)theta, (const float*)in, (float*)out, adjoint, s);
}

int maid_sobolev_value(maid_ctx* c, const void* theta, const void* a, double* r_out, hipStream_t s) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    if (!theta || !a || !r_out) return fail(c, MAID_EINVAL, "sobolev_value: NULL argument");
    return sobolev_value_impl(c, (const double*)theta, (const double*)a, r_out, s);
}

int maid_step(maid_ctx* c, const void* a, const void* y, maid_state* st, const maid_hparams* hp, maid_step_info* info,
              hipStream_t s) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    if (!a || !y || !st || !hp || !st->theta || !st->x || !st->q) return fail(c, MAID_EINVAL, "maid_step: NULL argument");
    if (!(hp->rho_lo > 0 && hp->rho_lo < 1) || !(hp->nu_lo > 0 && hp->nu_lo < 1) || !(hp->rho_hi > 1) || !(hp->nu_hi > 1))
        return fail(c, MAID_EINVAL, "maid_step: need 0 < rho_lo, nu_lo < 1 < rho_hi, nu_hi");
    if (hp->max_bt < 1 || hp->max_lower_iter < 0 || hp->max_cg_iter < 0 || !(hp->lambda > 0) || !(hp->mu > 0))
        return fail(c, MAID_EINVAL, "maid_step: bad hyperparameters");
    if (!(st->eps > 0) || !(st->delta > 0) || !(st->step > 0)) return fail(c, MAID_EINVAL, "maid_step: eps, delta, step must be > 0");
    if (c->d.dtype == MAID_F64) return maid_step_t<double>(c, (const double*)a, (const double*)y, st, hp, info, s);
    return maid_step_t<float>(c, (const double*)a, (const float*)y, st, hp, info, s);
}

}  // extern "C"
