// api.cpp -- the C ABI of libmaid (include/maid.h): argument checking and
// marshalling onto the batched drivers of engine.cpp.  A plain context is a
// batch of one instance.
#include "maid.h"

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "engine.h"

using namespace maid;

namespace {

thread_local std::string g_create_error;

bool bad_tol(double t) { return !(t >= 0.0) || !std::isfinite(t); }

int need_single(maid_ctx* c, const char* what) {
    if (c->n != 1)
        return fail(c, MAID_EINVAL, std::string(what) + ": this context holds a batch; use the maid_batch_* entry points");
    return MAID_OK;
}

int check_hparams(maid_ctx* c, const maid_hparams* hp) {
    if (!(hp->rho_lo > 0 && hp->rho_lo < 1) || !(hp->nu_lo > 0 && hp->nu_lo < 1) || !(hp->rho_hi > 1) || !(hp->nu_hi > 1))
        return fail(c, MAID_EINVAL, "maid_step: need 0 < rho_lo, nu_lo < 1 < rho_hi, nu_hi");
    if (hp->max_bt < 1 || hp->max_lower_iter < 0 || hp->max_cg_iter < 0 || !(hp->lambda > 0) || !(hp->mu > 0))
        return fail(c, MAID_EINVAL, "maid_step: bad hyperparameters");
    return MAID_OK;
}

int check_state(maid_ctx* c, const maid_state* st) {
    if (!st->theta || !st->x || !st->q) return fail(c, MAID_EINVAL, "maid_step: NULL argument");
    if (!(st->eps > 0) || !(st->delta > 0) || !(st->step > 0))
        return fail(c, MAID_EINVAL, "maid_step: eps, delta, step must be > 0");
    return MAID_OK;
}

template <typename P> std::vector<P> one(P p) { return std::vector<P>(1, p); }

template <typename T, typename V> std::vector<T> cast_all(V const* p, int n) {
    std::vector<T> out(n);
    for (int i = 0; i < n; ++i) out[i] = (T)p[i];
    return out;
}

// the message that goes with a per-instance failure code
int report(maid_ctx* c, int code, const char* what) {
    if (code == MAID_NOT_SPD) return fail(c, code, std::string(what) + ": curvature <p,Hp> <= 0");
    if (code < 0) return fail(c, code, std::string(what) + ": non-finite values met");
    return code;
}

template <typename T>
int lower_one(maid_ctx* c, const double* theta, const T* y, T* x, double tol, int max_iter, double* L_inout,
              maid_solve_info* info, int32_t* trace_bt, hipStream_t s) {
    int code = MAID_OK;
    int rc = lower_batch<T>(c, one<char>(1), one<const double*>(theta), one<const T*>(y), one<T*>(x), one<double>(tol),
                            max_iter, L_inout, info, &code, trace_bt, s);
    if (rc) return rc;
    return report(c, code, "lower_solve");
}

template <typename T>
int adjoint_one(maid_ctx* c, const double* theta, const T* xt, const T* rhs, T* q, double tol, int max_iter,
                maid_solve_info* info, hipStream_t s) {
    int code = MAID_OK;
    int rc = adjoint_batch<T>(c, one<char>(1), one<const double*>(theta), one<const T*>(xt), one<const T*>(rhs),
                              one<T*>(q), one<double>(tol), max_iter, info, &code, s);
    if (rc) return rc;
    return report(c, code, "adjoint_solve");
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

int maid_create(const maid_desc* desc, maid_ctx** out) { return maid_create_batch(desc, 1, out); }

int maid_create_batch(const maid_desc* descs, int32_t n, maid_ctx** out) {
    if (!out) {
        g_create_error = "out is NULL";
        return MAID_EINVAL;
    }
    *out = nullptr;
    if (!descs || n < 1) {
        g_create_error = "need n >= 1 descriptions";
        return MAID_EINVAL;
    }
    std::string why;
    const int rc = create_ctx(descs, n, out, why);
    if (rc) g_create_error = why;
    return rc;
}

int32_t maid_batch_size(const maid_ctx* c) { return c ? c->n : 0; }

void maid_destroy(maid_ctx* c) { destroy_ctx(c); }

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
    if (rows != 0 && !valid_rows(rows)) return fail(c, MAID_EINVAL, "rows per thread must be 0, 1, 2, 4 or 8");
    c->R_override = rows;
    return relayout(c);
}

int maid_set_one_pass(maid_ctx* c, int32_t mode) {
    if (!c) return MAID_EINVAL;
    if (mode < -1 || mode > 1) return fail(c, MAID_EINVAL, "mode must be -1 or 0 (two-pass) or 1 (one-pass)");
    c->fuse_pin = mode;
    return relayout(c);
}

int maid_one_pass_forms(const maid_ctx* c, int32_t* out) {
    if (!c || !out) return MAID_EINVAL;
    for (int i = 0; i < c->n; ++i) out[i] = c->m[i].nbf > 0 ? 1 : 0;
    return MAID_OK;
}

int maid_set_one_pass_cg(maid_ctx* c, int32_t enable) {
    if (!c) return MAID_EINVAL;
    c->cg_fuse = enable != 0;
    return relayout(c);
}

int maid_set_mfma(maid_ctx* c, int32_t enable) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    c->mfma = enable != 0;
    return relayout(c);
}

int maid_set_team(maid_ctx* c, int32_t members) {
    if (!c) return MAID_EINVAL;
    if (members < -1 || members > kTeamMax)
        return fail(c, MAID_EINVAL, "members per team must be -1 (size rule), 0 (off) or 1..128");
    c->team_req = members;
    return relayout(c);
}

int maid_profile(maid_ctx* c, int32_t enable) {
    if (!c) return MAID_EINVAL;
    prof_harvest(c);
    for (int k = 0; k < MAID_PROF_KINDS; ++k) {
        c->prof_launches[k] = 0;
        c->prof_work[k] = 0;
        c->prof_ms[k] = 0.0;
    }
    c->prof_on = enable != 0;
    return MAID_OK;
}

int maid_profile_read(maid_ctx* c, int32_t kind, int64_t* launches, int64_t* work_launches, double* total_ms) {
    if (!c || kind < 0 || kind >= MAID_PROF_KINDS || !launches || !total_ms) return MAID_EINVAL;
    prof_harvest(c);
    *launches = c->prof_launches[kind];
    if (work_launches) *work_launches = c->prof_work[kind];
    *total_ms = c->prof_ms[kind];
    return MAID_OK;
}

const char* maid_profile_name(int32_t kind) {
    static const char* names[MAID_PROF_KINDS] = {"conv",    "apg_grad", "apg_trial", "cg_dir",   "cg_hvp",
                                                  "cg_update", "hg_corr", "other",    "apg_team", "cg_team",
                                                  "apg_step", "cg_step"};
    if (kind < 0 || kind >= MAID_PROF_KINDS) return "";
    return names[kind];
}

int maid_lower_solve(maid_ctx* c, const void* theta, const void* y, void* x, double tol, int32_t max_iter, double* L_inout,
                     maid_solve_info* info, int32_t* trace_bt, hipStream_t s) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    if (int rc = need_single(c, "lower_solve")) return rc;
    if (!theta || !y || !x || !L_inout) return fail(c, MAID_EINVAL, "lower_solve: NULL argument");
    if (bad_tol(tol)) return fail(c, MAID_EINVAL, "lower_solve: tol must be finite and >= 0");
    if (max_iter < 0) return fail(c, MAID_EINVAL, "lower_solve: max_iter must be >= 0");
    if (trace_bt && max_iter > kTraceCap) return fail(c, MAID_EINVAL, "lower_solve: max_iter exceeds the trace capacity");
    if (!std::isfinite(*L_inout)) return fail(c, MAID_EINVAL, "lower_solve: L must be finite");
    if (c->dtype == MAID_F64)
        return lower_one<double>(c, (const double*)theta, (const double*)y, (double*)x, tol, max_iter, L_inout, info,
                                 trace_bt, s);
    return lower_one<float>(c, (const double*)theta, (const float*)y, (float*)x, tol, max_iter, L_inout, info, trace_bt, s);
}

int maid_lower_solve_refined(maid_ctx* c, const void* theta, const void* y, void* x, double tol, int32_t max_iter,
                             double rel_tol, int32_t max_newton, int32_t max_cg, double* L_inout, maid_solve_info* info,
                             maid_refine_info* rinfo, hipStream_t s) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    if (int rc = need_single(c, "lower_solve_refined")) return rc;
    if (!theta || !y || !x || !L_inout) return fail(c, MAID_EINVAL, "lower_solve_refined: NULL argument");
    if (bad_tol(tol) || bad_tol(rel_tol)) return fail(c, MAID_EINVAL, "lower_solve_refined: tolerances must be finite and >= 0");
    if (max_iter < 0 || max_newton < 0 || max_cg < 0)
        return fail(c, MAID_EINVAL, "lower_solve_refined: iteration caps must be >= 0");
    if (!std::isfinite(*L_inout)) return fail(c, MAID_EINVAL, "lower_solve_refined: L must be finite");
    const double cg_rel = 1e-2;
    int rc;
    if (c->dtype == MAID_F64) {
        rc = lower_one<double>(c, (const double*)theta, (const double*)y, (double*)x, tol, max_iter, L_inout, info,
                               nullptr, s);
        if (rc < 0) return rc;
        const int r2 = refine_one<double>(c, (const double*)theta, (const double*)y, (double*)x, rel_tol, max_newton,
                                          max_cg, cg_rel, rinfo, s);
        return r2 ? r2 : (rinfo && rinfo->status ? rinfo->status : MAID_OK);
    }
    rc = lower_one<float>(c, (const double*)theta, (const float*)y, (float*)x, tol, max_iter, L_inout, info, nullptr, s);
    if (rc < 0) return rc;
    const int r2 = refine_one<float>(c, (const double*)theta, (const float*)y, (float*)x, rel_tol, max_newton, max_cg,
                                     cg_rel, rinfo, s);
    return r2 ? r2 : (rinfo && rinfo->status ? rinfo->status : MAID_OK);
}

int maid_upper_value_grad(maid_ctx* c, const void* a, const void* y, const void* x, void* grad_out, double* g_out,
                          double* gradnorm_out, hipStream_t s) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    if (int rc = need_single(c, "upper_value_grad")) return rc;
    if (!a || !y || !x) return fail(c, MAID_EINVAL, "upper_value_grad: NULL argument");
    double g = 0.0, gn = 0.0;
    int rc;
    if (c->dtype == MAID_F64)
        rc = upper_batch<double>(c, one<char>(1), one<const double*>((const double*)a), one<const double*>((const double*)y),
                                 one<const double*>((const double*)x), one<double*>((double*)grad_out), &g, &gn, s);
    else
        rc = upper_batch<float>(c, one<char>(1), one<const double*>((const double*)a), one<const float*>((const float*)y),
                                one<const float*>((const float*)x), one<float*>((float*)grad_out), &g, &gn, s);
    if (rc) return rc;
    if (g_out) *g_out = g;
    if (gradnorm_out) *gradnorm_out = gn;
    return MAID_OK;
}

int maid_adjoint_solve(maid_ctx* c, const void* theta, const void* x_tilde, const void* rhs, void* q, double tol,
                       int32_t max_iter, maid_solve_info* info, hipStream_t s) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    if (int rc = need_single(c, "adjoint_solve")) return rc;
    if (!theta || !x_tilde || !rhs || !q) return fail(c, MAID_EINVAL, "adjoint_solve: NULL argument");
    if (bad_tol(tol)) return fail(c, MAID_EINVAL, "adjoint_solve: tol must be finite and >= 0");
    if (max_iter < 0) return fail(c, MAID_EINVAL, "adjoint_solve: max_iter must be >= 0");
    if (c->dtype == MAID_F64)
        return adjoint_one<double>(c, (const double*)theta, (const double*)x_tilde, (const double*)rhs, (double*)q, tol,
                                   max_iter, info, s);
    return adjoint_one<float>(c, (const double*)theta, (const float*)x_tilde, (const float*)rhs, (float*)q, tol, max_iter,
                              info, s);
}

int maid_hypergrad(maid_ctx* c, const void* theta, const void* a, const void* y, const void* x_tilde, const void* q,
                   int32_t with_r, double* z, double* znorm_out, hipStream_t s) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    if (int rc = need_single(c, "hypergrad")) return rc;
    if (!theta || !y || !x_tilde || !q || !z) return fail(c, MAID_EINVAL, "hypergrad: NULL argument");
    const int wr = with_r && c->m[0].d.beta != 0.0;
    if (wr && !a) return fail(c, MAID_EINVAL, "hypergrad: a is needed for the Sobolev term");
    double zn = 0.0;
    int rc;
    if (c->dtype == MAID_F64)
        rc = hypergrad_batch<double>(c, one<char>(1), one<const double*>((const double*)theta),
                                     one<const double*>((const double*)a), one<const double*>((const double*)y),
                                     one<const double*>((const double*)x_tilde), one<const double*>((const double*)q), wr,
                                     one<double*>(z), &zn, s);
    else
        rc = hypergrad_batch<float>(c, one<char>(1), one<const double*>((const double*)theta),
                                    one<const double*>((const double*)a), one<const float*>((const float*)y),
                                    one<const float*>((const float*)x_tilde), one<const float*>((const float*)q), wr,
                                    one<double*>(z), &zn, s);
    if (rc) return rc;
    if (znorm_out) *znorm_out = zn;
    return MAID_OK;
}

int maid_apply_operator(maid_ctx* c, const void* theta, const void* in, void* out, int32_t adjoint, hipStream_t s) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    if (int rc = need_single(c, "apply_operator")) return rc;
    if (!theta || !in || !out) return fail(c, MAID_EINVAL, "apply_operator: NULL argument");
    if (in == out) return fail(c, MAID_EINVAL, "apply_operator: in and out must not alias");
    if (c->dtype == MAID_F64)
        return apply_operator_one<double>(c, (const double*)theta, (const double*)in, (double*)out, adjoint, s);
    return apply_operator_one<float>(c, (const double*)theta, (const float*)in, (float*)out, adjoint, s);
}

int maid_sobolev_value(maid_ctx* c, const void* theta, const void* a, double* r_out, hipStream_t s) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    if (int rc = need_single(c, "sobolev_value")) return rc;
    if (!theta || !a || !r_out) return fail(c, MAID_EINVAL, "sobolev_value: NULL argument");
    return sobolev_batch(c, one<char>(1), one<const double*>((const double*)theta), one<const double*>((const double*)a),
                         r_out, s);
}

int maid_step(maid_ctx* c, const void* a, const void* y, maid_state* st, const maid_hparams* hp, maid_step_info* info,
              hipStream_t s) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    if (int rc = need_single(c, "maid_step")) return rc;
    if (!a || !y || !st || !hp) return fail(c, MAID_EINVAL, "maid_step: NULL argument");
    if (int rc = check_hparams(c, hp)) return rc;
    if (int rc = check_state(c, st)) return rc;
    int code = MAID_OK;
    int rc;
    if (c->dtype == MAID_F64)
        rc = step_batch<double>(c, one<const double*>((const double*)a), one<const double*>((const double*)y), st, hp,
                                info, &code, s);
    else
        rc = step_batch<float>(c, one<const double*>((const double*)a), one<const float*>((const float*)y), st, hp, info,
                               &code, s);
    if (rc) return rc;
    return report(c, code, "maid_step");
}

int maid_set_step_trace(maid_ctx* c, int32_t inst, int32_t* words, int32_t cap_words, double* values,
                        int32_t cap_values) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    auto& t = c->strace;
    if (!words || !values) {
        t = maid_ctx::StepTrace{};
        return MAID_OK;
    }
    if (inst < 0 || inst >= c->n || cap_words < 1 || cap_values < 1)
        return fail(c, MAID_EINVAL, "set_step_trace: bad instance or capacity");
    t.inst = inst;
    t.w = words;
    t.v = values;
    t.cap_w = cap_words;
    t.cap_v = cap_values;
    t.n_w = t.n_v = 0;
    t.full = false;
    return MAID_OK;
}

int maid_step_trace_length(const maid_ctx* c, int32_t* n_words, int32_t* n_values) {
    if (!c || !n_words || !n_values) return MAID_EINVAL;
    *n_words = c->strace.n_w;
    *n_values = c->strace.n_v;
    return MAID_OK;
}

int maid_autotune(maid_ctx* c, const void* const* theta, const void* const* y, int32_t probe_iters, int32_t* rows_out,
                  hipStream_t s) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    if (!theta || !y) return fail(c, MAID_EINVAL, "autotune: NULL argument");
    if (probe_iters < 1 || probe_iters > 1000) return fail(c, MAID_EINVAL, "autotune: probe_iters must be in 1..1000");
    for (int i = 0; i < c->n; ++i)
        if (!theta[i] || !y[i]) return fail(c, MAID_EINVAL, "autotune: NULL argument");
    const int n = c->n;
    if (c->dtype == MAID_F64)
        return autotune_batch<double>(c, cast_all<const double*>(theta, n), cast_all<const double*>(y, n), probe_iters,
                                      rows_out, s);
    return autotune_batch<float>(c, cast_all<const double*>(theta, n), cast_all<const float*>(y, n), probe_iters, rows_out,
                                 s);
}

// ---------------------------------------------------------------------- batched form
int maid_batch_lower_solve(maid_ctx* c, const void* const* theta, const void* const* y, void* const* x, const double* tol,
                           int32_t max_iter, double* L_inout, maid_solve_info* info, hipStream_t s) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    if (!theta || !y || !x || !tol || !L_inout) return fail(c, MAID_EINVAL, "batch_lower_solve: NULL argument");
    if (max_iter < 0) return fail(c, MAID_EINVAL, "batch_lower_solve: max_iter must be >= 0");
    for (int i = 0; i < c->n; ++i) {
        if (!theta[i] || !y[i] || !x[i]) return fail(c, MAID_EINVAL, "batch_lower_solve: NULL argument");
        if (bad_tol(tol[i])) return fail(c, MAID_EINVAL, "batch_lower_solve: tol must be finite and >= 0");
        if (!std::isfinite(L_inout[i])) return fail(c, MAID_EINVAL, "batch_lower_solve: L must be finite");
    }
    const int n = c->n;
    std::vector<char> act(n, 1);
    std::vector<int> codes(n, MAID_OK);
    std::vector<double> t(tol, tol + n);
    int rc;
    if (c->dtype == MAID_F64)
        rc = lower_batch<double>(c, act, cast_all<const double*>(theta, n), cast_all<const double*>(y, n),
                                 cast_all<double*>(x, n), t, max_iter, L_inout, info, codes.data(), nullptr, s);
    else
        rc = lower_batch<float>(c, act, cast_all<const double*>(theta, n), cast_all<const float*>(y, n),
                                cast_all<float*>(x, n), t, max_iter, L_inout, info, codes.data(), nullptr, s);
    if (rc) return rc;
    return report(c, combine_codes(codes.data(), n), "batch_lower_solve");
}

int maid_batch_adjoint_solve(maid_ctx* c, const void* const* theta, const void* const* x_tilde, const void* const* rhs,
                             void* const* q, const double* tol, int32_t max_iter, maid_solve_info* info, hipStream_t s) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    if (!theta || !x_tilde || !rhs || !q || !tol) return fail(c, MAID_EINVAL, "batch_adjoint_solve: NULL argument");
    if (max_iter < 0) return fail(c, MAID_EINVAL, "batch_adjoint_solve: max_iter must be >= 0");
    for (int i = 0; i < c->n; ++i) {
        if (!theta[i] || !x_tilde[i] || !rhs[i] || !q[i]) return fail(c, MAID_EINVAL, "batch_adjoint_solve: NULL argument");
        if (bad_tol(tol[i])) return fail(c, MAID_EINVAL, "batch_adjoint_solve: tol must be finite and >= 0");
    }
    const int n = c->n;
    std::vector<char> act(n, 1);
    std::vector<int> codes(n, MAID_OK);
    std::vector<double> t(tol, tol + n);
    int rc;
    if (c->dtype == MAID_F64)
        rc = adjoint_batch<double>(c, act, cast_all<const double*>(theta, n), cast_all<const double*>(x_tilde, n),
                                   cast_all<const double*>(rhs, n), cast_all<double*>(q, n), t, max_iter, info,
                                   codes.data(), s);
    else
        rc = adjoint_batch<float>(c, act, cast_all<const double*>(theta, n), cast_all<const float*>(x_tilde, n),
                                  cast_all<const float*>(rhs, n), cast_all<float*>(q, n), t, max_iter, info, codes.data(),
                                  s);
    if (rc) return rc;
    return report(c, combine_codes(codes.data(), n), "batch_adjoint_solve");
}

int maid_batch_upper_value_grad(maid_ctx* c, const void* const* a, const void* const* y, const void* const* x,
                                void* const* grad_out, double* g_out, double* gradnorm_out, hipStream_t s) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    if (!a || !y || !x) return fail(c, MAID_EINVAL, "batch_upper_value_grad: NULL argument");
    const int n = c->n;
    for (int i = 0; i < n; ++i)
        if (!a[i] || !y[i] || !x[i]) return fail(c, MAID_EINVAL, "batch_upper_value_grad: NULL argument");
    std::vector<char> act(n, 1);
    std::vector<double> g(n, 0.0), gn(n, 0.0);
    std::vector<void*> go(n, nullptr);
    if (grad_out)
        for (int i = 0; i < n; ++i) go[i] = grad_out[i];
    int rc;
    if (c->dtype == MAID_F64)
        rc = upper_batch<double>(c, act, cast_all<const double*>(a, n), cast_all<const double*>(y, n),
                                 cast_all<const double*>(x, n), cast_all<double*>(go.data(), n), g.data(), gn.data(), s);
    else
        rc = upper_batch<float>(c, act, cast_all<const double*>(a, n), cast_all<const float*>(y, n),
                                cast_all<const float*>(x, n), cast_all<float*>(go.data(), n), g.data(), gn.data(), s);
    if (rc) return rc;
    for (int i = 0; i < n; ++i) {
        if (g_out) g_out[i] = g[i];
        if (gradnorm_out) gradnorm_out[i] = gn[i];
    }
    return MAID_OK;
}

int maid_batch_hypergrad(maid_ctx* c, const void* const* theta, const void* const* a, const void* const* y,
                         const void* const* x_tilde, const void* const* q, int32_t with_r, void* const* z,
                         double* znorm_out, hipStream_t s) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    if (!theta || !y || !x_tilde || !q || !z) return fail(c, MAID_EINVAL, "batch_hypergrad: NULL argument");
    const int n = c->n;
    std::vector<const void*> av(n, nullptr);
    for (int i = 0; i < n; ++i) {
        if (!theta[i] || !y[i] || !x_tilde[i] || !q[i] || !z[i]) return fail(c, MAID_EINVAL, "batch_hypergrad: NULL argument");
        if (a) av[i] = a[i];
        if (with_r && c->m[i].d.beta != 0.0 && !av[i])
            return fail(c, MAID_EINVAL, "batch_hypergrad: a is needed for the Sobolev term");
    }
    std::vector<char> act(n, 1);
    std::vector<double> zn(n, 0.0);
    int rc;
    if (c->dtype == MAID_F64)
        rc = hypergrad_batch<double>(c, act, cast_all<const double*>(theta, n), cast_all<const double*>(av.data(), n),
                                     cast_all<const double*>(y, n), cast_all<const double*>(x_tilde, n),
                                     cast_all<const double*>(q, n), with_r != 0, cast_all<double*>(z, n), zn.data(), s);
    else
        rc = hypergrad_batch<float>(c, act, cast_all<const double*>(theta, n), cast_all<const double*>(av.data(), n),
                                    cast_all<const float*>(y, n), cast_all<const float*>(x_tilde, n),
                                    cast_all<const float*>(q, n), with_r != 0, cast_all<double*>(z, n), zn.data(), s);
    if (rc) return rc;
    if (znorm_out)
        for (int i = 0; i < n; ++i) znorm_out[i] = zn[i];
    return MAID_OK;
}

int maid_batch_step(maid_ctx* c, const void* const* a, const void* const* y, maid_state* states, const maid_hparams* hp,
                    maid_step_info* info, hipStream_t s) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    if (!a || !y || !states || !hp) return fail(c, MAID_EINVAL, "batch_step: NULL argument");
    if (int rc = check_hparams(c, hp)) return rc;
    for (int i = 0; i < c->n; ++i) {
        if (!a[i] || !y[i]) return fail(c, MAID_EINVAL, "batch_step: NULL argument");
        if (int rc = check_state(c, &states[i])) return rc;
    }
    const int n = c->n;
    std::vector<int> codes(n, MAID_OK);
    int rc;
    if (c->dtype == MAID_F64)
        rc = step_batch<double>(c, cast_all<const double*>(a, n), cast_all<const double*>(y, n), states, hp, info,
                                codes.data(), s);
    else
        rc = step_batch<float>(c, cast_all<const double*>(a, n), cast_all<const float*>(y, n), states, hp, info,
                               codes.data(), s);
    if (rc) return rc;
    return report(c, combine_codes(codes.data(), n), "batch_step");
}

int maid_batch_steps(maid_ctx* c, const void* const* a, const void* const* y, maid_state* states, const maid_hparams* hp,
                     maid_step_info* info, int32_t n_steps, hipStream_t s) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    if (!a || !y || !states || !hp) return fail(c, MAID_EINVAL, "batch_steps: NULL argument");
    if (n_steps < 1) return fail(c, MAID_EINVAL, "batch_steps: n_steps must be >= 1");
    if (int rc = check_hparams(c, hp)) return rc;
    for (int i = 0; i < c->n; ++i) {
        if (!a[i] || !y[i]) return fail(c, MAID_EINVAL, "batch_steps: NULL argument");
        if (int rc = check_state(c, &states[i])) return rc;
    }
    const int n = c->n;
    std::vector<char> act(n, 1);
    std::vector<int> codes(n, MAID_OK), last(n, MAID_OK);
    std::vector<maid_step_info> one(n), sum(n);
    std::memset(sum.data(), 0, n * sizeof(maid_step_info));
    for (int k = 0; k < n_steps; ++k) {
        bool any_act = false;
        for (char v : act) any_act = any_act || v;
        if (!any_act) break;
        int rc;
        if (c->dtype == MAID_F64)
            rc = step_batch<double>(c, cast_all<const double*>(a, n), cast_all<const double*>(y, n), states, hp,
                                    one.data(), codes.data(), s, &act);
        else
            rc = step_batch<float>(c, cast_all<const double*>(a, n), cast_all<const float*>(y, n), states, hp,
                                   one.data(), codes.data(), s, &act);
        if (rc) return rc;
        for (int i = 0; i < n; ++i) {
            if (!act[i]) continue;
            maid_step_info& t = sum[i];
            const maid_step_info& o = one[i];
            t.accepted += o.accepted;
            t.trials += o.trials;
            t.retries += o.retries;
            t.lower_iters += o.lower_iters;
            t.cg_iters += o.cg_iters;
            t.psi = o.psi;
            t.ell_k = o.ell_k;
            t.ell_next = o.ell_next;
            t.znorm = o.znorm;
            t.status = o.status;
            if (o.lower_status) t.lower_status = o.lower_status;
            if (o.cg_status) t.cg_status = o.cg_status;
            // a capped solve is carried on with; the floor or an error ends the instance's run
            if (codes[i] == MAID_MAXITER) {
                if (last[i] == MAID_OK) last[i] = MAID_MAXITER;
            } else if (codes[i] != MAID_OK) {
                last[i] = codes[i];
            }
            if (codes[i] != MAID_OK && codes[i] != MAID_MAXITER) act[i] = 0;
        }
    }
    if (info)
        for (int i = 0; i < n; ++i) info[i] = sum[i];
    return report(c, combine_codes(last.data(), n), "batch_steps");
}

int maid_batch_create(const maid_desc* descs, int32_t n, maid_ctx** out) { return maid_create_batch(descs, n, out); }

// ---------------------------------------------------------------------- Section 4.1's baselines
int maid_gd_solve(maid_ctx* c, const void* theta, const void* y, void* x, double step, int32_t n_iter, double tol,
                  void* hist, maid_solve_info* info, hipStream_t s) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    if (int rc = need_single(c, "gd_solve")) return rc;
    if (!theta || !y || !x) return fail(c, MAID_EINVAL, "gd_solve: NULL argument");
    if (!(step > 0.0) || !std::isfinite(step)) return fail(c, MAID_EINVAL, "gd_solve: step must be finite and > 0");
    if (n_iter < 0) return fail(c, MAID_EINVAL, "gd_solve: n_iter must be >= 0");
    if (bad_tol(tol)) return fail(c, MAID_EINVAL, "gd_solve: tol must be finite and >= 0");
    if (c->dtype == MAID_F64)
        return gd_one<double>(c, (const double*)theta, (const double*)y, (double*)x, step, n_iter, tol, (double*)hist,
                              info, s);
    return gd_one<float>(c, (const double*)theta, (const float*)y, (float*)x, step, n_iter, tol, (float*)hist, info, s);
}

int maid_hessian_apply(maid_ctx* c, const void* theta, const void* x, const void* w, void* out, hipStream_t s) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    if (int rc = need_single(c, "hessian_apply")) return rc;
    if (!theta || !x || !w || !out) return fail(c, MAID_EINVAL, "hessian_apply: NULL argument");
    if (out == w || out == x) return fail(c, MAID_EINVAL, "hessian_apply: out must not alias x or w");
    if (c->dtype == MAID_F64)
        return hessian_one<double>(c, (const double*)theta, (const double*)x, (const double*)w, (double*)out, s);
    return hessian_one<float>(c, (const double*)theta, (const float*)x, (const float*)w, (float*)out, s);
}

int maid_ift_step(maid_ctx* c, const void* a, const void* y, maid_state* st, int32_t n_lower, double lambda_x,
                  double cg_tol, int32_t max_cg, maid_step_info* info, hipStream_t s) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    if (int rc = need_single(c, "ift_step")) return rc;
    if (!a || !y || !st || !st->theta || !st->x || !st->q) return fail(c, MAID_EINVAL, "ift_step: NULL argument");
    if (n_lower < 0 || max_cg < 0) return fail(c, MAID_EINVAL, "ift_step: iteration counts must be >= 0");
    if (!(lambda_x > 0.0) || !std::isfinite(lambda_x) || !(st->step > 0.0) || !std::isfinite(st->step))
        return fail(c, MAID_EINVAL, "ift_step: lambda_x and the step must be finite and > 0");
    if (bad_tol(cg_tol)) return fail(c, MAID_EINVAL, "ift_step: cg_tol must be finite and >= 0");
    if (c->dtype == MAID_F64)
        return ift_step_one<double>(c, (const double*)a, (const double*)y, st, n_lower, lambda_x, cg_tol, max_cg, info,
                                    s);
    return ift_step_one<float>(c, (const double*)a, (const float*)y, st, n_lower, lambda_x, cg_tol, max_cg, info, s);
}

int maid_lista_step(maid_ctx* c, const void* a, const void* y, maid_state* st, int32_t n_unroll, double lambda_x,
                    maid_step_info* info, hipStream_t s) {
    if (!c) return MAID_EINVAL;
    c->err.clear();
    if (int rc = need_single(c, "lista_step")) return rc;
    if (!a || !y || !st || !st->theta || !st->x) return fail(c, MAID_EINVAL, "lista_step: NULL argument");
    if (n_unroll < 1) return fail(c, MAID_EINVAL, "lista_step: n_unroll must be >= 1");
    if (!(lambda_x > 0.0) || !std::isfinite(lambda_x) || !(st->step > 0.0) || !std::isfinite(st->step))
        return fail(c, MAID_EINVAL, "lista_step: lambda_x and the step must be finite and > 0");
    if (c->dtype == MAID_F64)
        return lista_step_one<double>(c, (const double*)a, (const double*)y, st, n_unroll, lambda_x, info, s);
    return lista_step_one<float>(c, (const double*)a, (const float*)y, st, n_unroll, lambda_x, info, s);
}

}  // extern "C"
