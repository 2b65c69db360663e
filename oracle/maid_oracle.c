/*
 * maid_oracle.c -- FP64 CPU oracle for the MAID hot path.
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, by the package's smoke() check
 * and by bench.py's CPU-baseline leg.  The product path never loads it.
 *
 * Everything is written from the definitions in the paper (arXiv 2502.09758),
 * in plain loops, double precision, no reordering beyond what a definition
 * states.  Conventions are listed in maid_oracle.h.  Whole-image loops over
 * pixels may run on several OpenMP threads: each thread writes distinct
 * outputs, and every reduction (norm, dot product, objective) is a serial
 * loop in a fixed order, so results do not depend on the thread count.
 */
#include "maid_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------
 * indexing and boundary handling
 * ---------------------------------------------------------------------- */
static inline int64_t npix(const om_problem* p) { return (int64_t)p->C * p->H * p->W; }

static inline int wrap(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }

/* kernel channels and the taps that blur image channel c: theta holds kc
   planes of KxK taps, one shared plane (kc = 1) or one per channel (kc = C) */
static inline int nkc(const om_problem* p) { return p->kc > 1 ? p->kc : 1; }
static inline int bad_kc(const om_problem* p) { return p->kc > 1 && p->kc != p->C; }
static inline const double* taps(const om_problem* p, const double* th, int c) {
    return p->kc > 1 ? th + (int64_t)c * p->K * p->K : th;
}

/* x_c(i,j) with zero extension outside the image (or periodic wrap). */
static inline double at(const om_problem* p, const double* x, int c, int i, int j) {
    if (p->periodic) { i = wrap(i, p->H); j = wrap(j, p->W); }
    else if (i < 0 || i >= p->H || j < 0 || j >= p->W) return 0.0;
    return x[((int64_t)c * p->H + i) * p->W + j];
}

/* forward differences: (D_h x)(i,j) = x(i,j+1) - x(i,j), 0 in the last column
   (Neumann); (D_v x)(i,j) = x(i+1,j) - x(i,j), 0 in the last row.  Periodic
   mode wraps.  Section 4.2 names forward differences for the TV gradient. */
static inline double dh_at(const om_problem* p, const double* x, int c, int i, int j) {
    if (p->periodic) return at(p, x, c, i, j + 1) - at(p, x, c, i, j);
    return (j < p->W - 1) ? at(p, x, c, i, j + 1) - at(p, x, c, i, j) : 0.0;
}
static inline double dv_at(const om_problem* p, const double* x, int c, int i, int j) {
    if (p->periodic) return at(p, x, c, i + 1, j) - at(p, x, c, i, j);
    return (i < p->H - 1) ? at(p, x, c, i + 1, j) - at(p, x, c, i, j) : 0.0;
}

/* ------------------------------------------------------------------------
 * convolution T(theta, x) of Eq. (2.4) as a 2D same-size convolution
 * ---------------------------------------------------------------------- */
static double conv_px(const om_problem* p, const double* th, const double* x, int c, int i, int j) {
    const int K = p->K, c0 = (K - 1) / 2;
    th = taps(p, th, c);
    double s = 0.0;
    for (int u = 0; u < K; ++u)
        for (int v = 0; v < K; ++v)
            s += th[u * K + v] * at(p, x, c, i + c0 - u, j + c0 - v);
    return s;
}

static double conv_adj_px(const om_problem* p, const double* th, const double* r, int c, int i, int j) {
    const int K = p->K, c0 = (K - 1) / 2;
    th = taps(p, th, c);
    double s = 0.0;
    for (int u = 0; u < K; ++u)
        for (int v = 0; v < K; ++v)
            s += th[u * K + v] * at(p, r, c, i - c0 + u, j - c0 + v);
    return s;
}

void oracle_conv(const om_problem* p, const double* th, const double* x, double* out) {
    const int C = p->C, H = p->H, W = p->W;
#pragma omp parallel for collapse(2) schedule(static)
    for (int c = 0; c < C; ++c)
        for (int i = 0; i < H; ++i)
            for (int j = 0; j < W; ++j)
                out[((int64_t)c * H + i) * W + j] = conv_px(p, th, x, c, i, j);
}

void oracle_conv_adj(const om_problem* p, const double* th, const double* r, double* out) {
    const int C = p->C, H = p->H, W = p->W;
#pragma omp parallel for collapse(2) schedule(static)
    for (int c = 0; c < C; ++c)
        for (int i = 0; i < H; ++i)
            for (int j = 0; j < W; ++j)
                out[((int64_t)c * H + i) * W + j] = conv_adj_px(p, th, r, c, i, j);
}

void oracle_diff(const om_problem* p, const double* x, double* dh, double* dv) {
    const int C = p->C, H = p->H, W = p->W;
    for (int c = 0; c < C; ++c)
        for (int i = 0; i < H; ++i)
            for (int j = 0; j < W; ++j) {
                int64_t e = ((int64_t)c * H + i) * W + j;
                dh[e] = dh_at(p, x, c, i, j);
                dv[e] = dv_at(p, x, c, i, j);
            }
}

/* adjoint of the forward differences: (D_h^T q)(i,j) = q(i,j-1)[j>=1] - q(i,j)[j<=W-2]
   in Neumann mode, q(i,j-1 mod W) - q(i,j) in periodic mode; D_v^T likewise. */
static double dhT_px(const om_problem* p, const double* q, int c, int i, int j) {
    if (p->periodic) return at(p, q, c, i, j - 1) - at(p, q, c, i, j);
    double s = 0.0;
    if (j >= 1) s += at(p, q, c, i, j - 1);
    if (j <= p->W - 2) s -= at(p, q, c, i, j);
    return s;
}
static double dvT_px(const om_problem* p, const double* q, int c, int i, int j) {
    if (p->periodic) return at(p, q, c, i - 1, j) - at(p, q, c, i, j);
    double s = 0.0;
    if (i >= 1) s += at(p, q, c, i - 1, j);
    if (i <= p->H - 2) s -= at(p, q, c, i, j);
    return s;
}

void oracle_diff_adj(const om_problem* p, const double* ph, const double* pv, double* out) {
    const int C = p->C, H = p->H, W = p->W;
    for (int c = 0; c < C; ++c)
        for (int i = 0; i < H; ++i)
            for (int j = 0; j < W; ++j)
                out[((int64_t)c * H + i) * W + j] = dhT_px(p, ph, c, i, j) + dvT_px(p, pv, c, i, j);
}

/* ------------------------------------------------------------------------
 * smoothed total variation (Section 4.2): R(x) = sum phi(|grad x|),
 * phi(s) = sqrt(s^2 + eps^2) - eps, isotropic per pixel.
 * ---------------------------------------------------------------------- */
/* squared gradient magnitude at pixel (i,j): over all channels (reg 0, one
   magnitude per pixel couples the colour channels) or channel c only (reg 1) */
static double s2_px(const om_problem* p, const double* x, int c, int i, int j) {
    double s = 0.0;
    if (p->reg == 0) {
        for (int cc = 0; cc < p->C; ++cc) {
            double a = dh_at(p, x, cc, i, j), b = dv_at(p, x, cc, i, j);
            s += a * a + b * b;
        }
    } else {
        double a = dh_at(p, x, c, i, j), b = dv_at(p, x, c, i, j);
        s = a * a + b * b;
    }
    return s;
}

/* weight w = (s^2+eps^2)^(-1/2) = phi'(s)/s; constant 1 for the quadratic reg */
static double w_px(const om_problem* p, const double* x, int c, int i, int j) {
    if (p->reg == 2) return 1.0;
    double s2 = s2_px(p, x, c, i, j);
    return 1.0 / sqrt(s2 + p->eps_tv * p->eps_tv);
}

/* contribution of one "site" to R: a pixel for reg 0, a (channel, pixel)
   for reg 1 and reg 2 */
static double site_value(const om_problem* p, const double* x, int c, int i, int j) {
    if (p->reg == 2) {
        double a = dh_at(p, x, c, i, j), b = dv_at(p, x, c, i, j);
        return 0.5 * (a * a + b * b);
    }
    double s2 = s2_px(p, x, c, i, j);
    return sqrt(s2 + p->eps_tv * p->eps_tv) - p->eps_tv;
}

static int n_site_channels(const om_problem* p) { return p->reg == 0 ? 1 : p->C; }

double oracle_reg_value(const om_problem* p, const double* x) {
    double s = 0.0;
    for (int c = 0; c < n_site_channels(p); ++c)
        for (int i = 0; i < p->H; ++i)
            for (int j = 0; j < p->W; ++j) s += site_value(p, x, c, i, j);
    return s;
}

/* grad R(x)_c = D_h^T(w D_h x_c) + D_v^T(w D_v x_c): the flux w*Dx is formed
   at the three pixels the adjoint difference touches. */
static double flux_h(const om_problem* p, const double* x, int c, int i, int j) {
    if (!p->periodic && (i < 0 || i >= p->H || j < 0 || j >= p->W)) return 0.0;
    return w_px(p, x, c, i, j) * dh_at(p, x, c, i, j);
}
static double flux_v(const om_problem* p, const double* x, int c, int i, int j) {
    if (!p->periodic && (i < 0 || i >= p->H || j < 0 || j >= p->W)) return 0.0;
    return w_px(p, x, c, i, j) * dv_at(p, x, c, i, j);
}

static double reg_grad_px(const om_problem* p, const double* x, int c, int i, int j) {
    double s = 0.0;
    /* D_h^T part */
    if (p->periodic || j >= 1) s += flux_h(p, x, c, i, j - 1);
    if (p->periodic || j <= p->W - 2) s -= flux_h(p, x, c, i, j);
    /* D_v^T part */
    if (p->periodic || i >= 1) s += flux_v(p, x, c, i - 1, j);
    if (p->periodic || i <= p->H - 2) s -= flux_v(p, x, c, i, j);
    return s;
}

void oracle_reg_grad(const om_problem* p, const double* x, double* out) {
    const int C = p->C, H = p->H, W = p->W;
#pragma omp parallel for collapse(2) schedule(static)
    for (int c = 0; c < C; ++c)
        for (int i = 0; i < H; ++i)
            for (int j = 0; j < W; ++j)
                out[((int64_t)c * H + i) * W + j] = reg_grad_px(p, x, c, i, j);
}

/* Hessian-vector product: the derivative of w*Dx_c in direction d is
   w*Dd_c - w^3 * m * Dx_c, with m = sum over the coupled channels of
   <Dx, Dd> at the pixel (d/dt (s^2+eps^2)^(-1/2) = -w^3 * d(s^2)/dt / 2). */
static double hflux(const om_problem* p, const double* x, const double* d, int c, int i, int j, int horiz) {
    if (!p->periodic && (i < 0 || i >= p->H || j < 0 || j >= p->W)) return 0.0;
    double dd = horiz ? dh_at(p, d, c, i, j) : dv_at(p, d, c, i, j);
    if (p->reg == 2) return dd;
    double dx = horiz ? dh_at(p, x, c, i, j) : dv_at(p, x, c, i, j);
    double w = w_px(p, x, c, i, j);
    double m = 0.0;
    if (p->reg == 0) {
        for (int cc = 0; cc < p->C; ++cc)
            m += dh_at(p, x, cc, i, j) * dh_at(p, d, cc, i, j) + dv_at(p, x, cc, i, j) * dv_at(p, d, cc, i, j);
    } else {
        m = dh_at(p, x, c, i, j) * dh_at(p, d, c, i, j) + dv_at(p, x, c, i, j) * dv_at(p, d, c, i, j);
    }
    return w * dd - w * w * w * m * dx;
}

static double reg_hvp_px(const om_problem* p, const double* x, const double* d, int c, int i, int j) {
    double s = 0.0;
    if (p->periodic || j >= 1) s += hflux(p, x, d, c, i, j - 1, 1);
    if (p->periodic || j <= p->W - 2) s -= hflux(p, x, d, c, i, j, 1);
    if (p->periodic || i >= 1) s += hflux(p, x, d, c, i - 1, j, 0);
    if (p->periodic || i <= p->H - 2) s -= hflux(p, x, d, c, i, j, 0);
    return s;
}

void oracle_reg_hvp(const om_problem* p, const double* x, const double* d, double* out) {
    const int C = p->C, H = p->H, W = p->W;
#pragma omp parallel for collapse(2) schedule(static)
    for (int c = 0; c < C; ++c)
        for (int i = 0; i < H; ++i)
            for (int j = 0; j < W; ++j)
                out[((int64_t)c * H + i) * W + j] = reg_hvp_px(p, x, d, c, i, j);
}

/* ------------------------------------------------------------------------
 * lower level h(x; theta) = 1/2 ||theta*x - y||^2 + alpha R(x)
 * gradient and Hessian as in Proposition 1 (with the 1/2 on the data term)
 * ---------------------------------------------------------------------- */
static double* dalloc(int64_t n) { return (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double)); }

static double dot(const double* a, const double* b, int64_t n) {
    double s = 0.0;
    for (int64_t e = 0; e < n; ++e) s += a[e] * b[e];
    return s;
}

double oracle_h_value(const om_problem* p, const double* th, const double* y, const double* x) {
    int64_t N = npix(p);
    double* r = dalloc(N);
    oracle_conv(p, th, x, r);
    double s = 0.0;
    for (int64_t e = 0; e < N; ++e) { double d = r[e] - y[e]; s += 0.5 * d * d; }
    free(r);
    return s + p->alpha * oracle_reg_value(p, x);
}

void oracle_h_grad(const om_problem* p, const double* th, const double* y, const double* x, double* out) {
    int64_t N = npix(p);
    double* r = dalloc(N);
    double* gr = dalloc(N);
    oracle_conv(p, th, x, r);
    for (int64_t e = 0; e < N; ++e) r[e] -= y[e];
    oracle_conv_adj(p, th, r, out);
    oracle_reg_grad(p, x, gr);
    for (int64_t e = 0; e < N; ++e) out[e] += p->alpha * gr[e];
    free(r); free(gr);
}

void oracle_h_hvp(const om_problem* p, const double* th, const double* x, const double* d, double* out) {
    int64_t N = npix(p);
    double* kd = dalloc(N);
    double* hr = dalloc(N);
    oracle_conv(p, th, d, kd);
    oracle_conv_adj(p, th, kd, out);
    oracle_reg_hvp(p, x, d, hr);
    for (int64_t e = 0; e < N; ++e) out[e] += p->alpha * hr[e];
    free(kd); free(hr);
}

/* ------------------------------------------------------------------------
 * upper-level Sobolev term r(theta) = beta * ||theta - a||_{H^1}^2 (Eq. 2.5,
 * discretised with forward differences on the KxK grid as in Section 4.2)
 * ---------------------------------------------------------------------- */
static void ksz_problem(const om_problem* p, om_problem* q) {
    memset(q, 0, sizeof(*q));
    q->C = 1; q->H = p->K; q->W = p->K; q->K = 1; q->periodic = 0; q->reg = 2;
}

double oracle_sobolev_value(const om_problem* p, const double* th, const double* a) {
    if (p->beta == 0.0) return 0.0;
    const int KK = p->K * p->K;
    om_problem q; ksz_problem(p, &q);
    double* e = dalloc(KK); double* dh = dalloc(KK); double* dv = dalloc(KK);
    double s = 0.0;
    for (int k = 0; k < nkc(p); ++k) {   /* one KxK grid per kernel channel */
        for (int t = 0; t < KK; ++t) e[t] = th[k * KK + t] - a[k * KK + t];
        oracle_diff(&q, e, dh, dv);
        s += p->h1_w0 * dot(e, e, KK) + dot(dh, dh, KK) + dot(dv, dv, KK);
    }
    free(e); free(dh); free(dv);
    return p->beta * s;
}

void oracle_sobolev_grad(const om_problem* p, const double* th, const double* a, double* out) {
    const int KK = p->K * p->K;
    if (p->beta == 0.0) { for (int t = 0; t < nkc(p) * KK; ++t) out[t] = 0.0; return; }
    om_problem q; ksz_problem(p, &q);
    double* e = dalloc(KK); double* dh = dalloc(KK); double* dv = dalloc(KK); double* lap = dalloc(KK);
    for (int k = 0; k < nkc(p); ++k) {
        for (int t = 0; t < KK; ++t) e[t] = th[k * KK + t] - a[k * KK + t];
        oracle_diff(&q, e, dh, dv);
        oracle_diff_adj(&q, dh, dv, lap);
        for (int t = 0; t < KK; ++t) out[k * KK + t] = 2.0 * p->beta * (p->h1_w0 * e[t] + lap[t]);
    }
    free(e); free(dh); free(dv); free(lap);
}

/* ------------------------------------------------------------------------
 * Algorithm 1, lower-level solve: accelerated gradient (FISTA, Beck-Teboulle)
 * with backtracking on the Lipschitz estimate L (factor 2), for the smooth
 * problem min_x h(x; theta).  Stops at the extrapolated point v once
 * ||grad h(v)|| <= tol (tol = eps * mu in Algorithm 1), which is the point
 * returned.
 *
 * replay_bt (nullable): if given, the solve runs exactly max_iter iterations
 * and at iteration n rejects exactly replay_bt[n] trial steps before
 * accepting, instead of applying its own tests.  trace_bt (nullable, length
 * >= max_iter) receives the number of rejected trials per iteration.
 * ---------------------------------------------------------------------- */
static double sum_abs(const double* a, int n) { double s = 0; for (int t = 0; t < n; ++t) s += fabs(a[t]); return s; }

/* (max_c ||theta_c||_1)^2 bounds ||theta*.||^2: Young's inequality on each
   channel's convolution, and the channels do not mix */
static double l1_bound_sq(const om_problem* p, const double* th) {
    const int KK = p->K * p->K;
    double m = 0.0;
    for (int k = 0; k < nkc(p); ++k) { double s = sum_abs(th + k * KK, KK); if (s > m) m = s; }
    return m * m;
}

/* h(v + dl) - h(v) for the trial increment dl = -G/L, evaluated through the
   increment so that no two nearly equal objective values are subtracted:
     data part  1/2||r + d||^2 - 1/2||r||^2 = sum_e d_e (r_e + d_e/2), d = theta*dl,
     TV site    phi(s') - phi(s) = (s'^2 - s^2) / (sqrt(s'^2+eps^2) + sqrt(s^2+eps^2))
                with s'^2 - s^2 = sum a (a + 2 b), a = D dl, b = D v over the
                site's channels (quadratic R: sum a (b + a/2)). */
static double site_difference(const om_problem* p, const double* v, const double* dl, int c, int i, int j) {
    int c_lo = c, c_hi = c + 1;
    if (p->reg == 0) { c_lo = 0; c_hi = p->C; }
    double ds2 = 0.0, s2 = 0.0;
    for (int cc = c_lo; cc < c_hi; ++cc) {
        const double ah = dh_at(p, dl, cc, i, j), av = dv_at(p, dl, cc, i, j);
        const double bh = dh_at(p, v, cc, i, j), bv = dv_at(p, v, cc, i, j);
        if (p->reg == 2) { ds2 += ah * (bh + 0.5 * ah) + av * (bv + 0.5 * av); continue; }
        ds2 += ah * (ah + 2.0 * bh) + av * (av + 2.0 * bv);
        s2 += bh * bh + bv * bv;
    }
    if (p->reg == 2) return ds2;
    const double e2 = p->eps_tv * p->eps_tv;
    return ds2 / (sqrt(s2 + ds2 + e2) + sqrt(s2 + e2));
}

static double h_difference(const om_problem* p, const double* th, const double* rv,
                           const double* v, const double* dl, double* dtmp) {
    const int64_t N = npix(p);
    oracle_conv(p, th, dl, dtmp);
    double d = 0.0;
    for (int64_t e = 0; e < N; ++e) d += dtmp[e] * (rv[e] + 0.5 * dtmp[e]);
    double dr = 0.0;
    for (int c = 0; c < n_site_channels(p); ++c)
        for (int i = 0; i < p->H; ++i)
            for (int j = 0; j < p->W; ++j)
                dr += site_difference(p, v, dl, c, i, j);
    return d + p->alpha * dr;
}

int oracle_lower_solve(const om_problem* p, const double* th, const double* y, double* x,
                       double tol, int32_t max_iter, double* L_inout, om_solve_info* info,
                       const int32_t* replay_bt, int32_t* trace_bt) {
    if (!p || !th || !y || !x || !L_inout || max_iter < 0 || tol < 0 || bad_kc(p)) return OM_EINVAL;
    const int64_t N = npix(p);
    double *xp = dalloc(N), *xc = dalloc(N), *v = dalloc(N), *G = dalloc(N);
    double *xn = dalloc(N), *rv = dalloc(N), *dl = dalloc(N), *dtmp = dalloc(N);
    memcpy(xp, x, N * sizeof(double));
    memcpy(xc, x, N * sizeof(double));
    double L = *L_inout;
    if (!(L > 0)) L = l1_bound_sq(p, th);
    double t_prev = 1.0, t = 1.0, gn2 = 0.0;
    int n = 0, bt_total = 0, status = OM_OK;
    for (n = 0;; ++n) {
        const double m = (t_prev - 1.0) / t;
        for (int64_t e = 0; e < N; ++e) v[e] = xc[e] + m * (xc[e] - xp[e]);
        oracle_h_grad(p, th, y, v, G);
        gn2 = dot(G, G, N);
        if (!replay_bt && sqrt(gn2) <= tol) { status = OM_OK; break; }
        if (n == max_iter) { status = replay_bt ? OM_OK : OM_MAXITER; break; }
        oracle_conv(p, th, v, rv);
        for (int64_t e = 0; e < N; ++e) rv[e] -= y[e];
        int nb = 0;
        for (;;) {
            for (int64_t e = 0; e < N; ++e) { dl[e] = -G[e] / L; xn[e] = v[e] + dl[e]; }
            int accept;
            if (replay_bt) {
                accept = (nb >= replay_bt[n]);
            } else {
                double delta = h_difference(p, th, rv, v, dl, dtmp);
                accept = (delta <= -gn2 / (2.0 * L));
            }
            if (accept) break;
            L *= 2.0;
            ++nb;
        }
        bt_total += nb;
        if (trace_bt) trace_bt[n] = nb;
        memcpy(xp, xc, N * sizeof(double));
        memcpy(xc, xn, N * sizeof(double));
        const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
        t_prev = t;
        t = tn;
    }
    memcpy(x, v, N * sizeof(double));
    *L_inout = L;
    if (info) {
        info->iters = n;
        info->backtracks = bt_total;
        info->status = status;
        info->res_norm = sqrt(gn2);
        info->obj = oracle_h_value(p, th, y, v);
        info->L = L;
    }
    free(xp); free(xc); free(v); free(G); free(xn); free(rv); free(dl); free(dtmp);
    return status;
}

/* g(x) = 1/2 ||a*x - y||^2 and grad g(x) = a.(a*x - y) */
void oracle_upper_value_grad(const om_problem* p, const double* a, const double* y, const double* x,
                             double* grad_out, double* g_out, double* gradnorm_out) {
    const int64_t N = npix(p);
    double* rho = dalloc(N);
    double* gr = dalloc(N);
    oracle_conv(p, a, x, rho);
    double g = 0.0;
    for (int64_t e = 0; e < N; ++e) { rho[e] -= y[e]; g += 0.5 * rho[e] * rho[e]; }
    oracle_conv_adj(p, a, rho, gr);
    if (grad_out) memcpy(grad_out, gr, N * sizeof(double));
    if (g_out) *g_out = g;
    if (gradnorm_out) *gradnorm_out = sqrt(dot(gr, gr, N));
    free(rho); free(gr);
}

/* ------------------------------------------------------------------------
 * Algorithm 1, Hessian system: conjugate gradients on
 * (theta.theta* + alpha grad^2 R(xt)) q = rhs, stopping when the recursive
 * residual norm sqrt(gamma) <= tol.
 * ---------------------------------------------------------------------- */
int oracle_adjoint_solve(const om_problem* p, const double* th, const double* xt, const double* rhs,
                         double* q_io, double tol, int32_t max_iter, om_solve_info* info,
                         double* true_res_out) {
    if (!p || !th || !xt || !rhs || !q_io || max_iter < 0 || tol < 0 || bad_kc(p)) return OM_EINVAL;
    const int64_t N = npix(p);
    double *q = dalloc(N), *r = dalloc(N), *pd = dalloc(N), *w = dalloc(N);
    memcpy(q, q_io, N * sizeof(double));
    oracle_h_hvp(p, th, xt, q, w);
    for (int64_t e = 0; e < N; ++e) { r[e] = rhs[e] - w[e]; pd[e] = r[e]; }
    double gamma = dot(r, r, N);
    int n, status = OM_OK;
    for (n = 0;; ++n) {
        if (sqrt(gamma) <= tol) { status = OM_OK; break; }
        if (n == max_iter) { status = OM_MAXITER; break; }
        oracle_h_hvp(p, th, xt, pd, w);
        const double kappa = dot(pd, w, N);
        if (!(kappa > 0.0)) { status = OM_NOT_SPD; break; }
        const double a = gamma / kappa;
        for (int64_t e = 0; e < N; ++e) { q[e] += a * pd[e]; r[e] -= a * w[e]; }
        const double gnew = dot(r, r, N);
        const double b = gnew / gamma;
        for (int64_t e = 0; e < N; ++e) pd[e] = r[e] + b * pd[e];
        gamma = gnew;
    }
    if (status != OM_NOT_SPD) memcpy(q_io, q, N * sizeof(double));
    if (true_res_out) {
        oracle_h_hvp(p, th, xt, q, w);
        double s = 0.0;
        for (int64_t e = 0; e < N; ++e) { double d = rhs[e] - w[e]; s += d * d; }
        *true_res_out = sqrt(s);
    }
    if (info) {
        info->iters = n;
        info->backtracks = 0;
        info->status = status;
        info->res_norm = sqrt(gamma);
        info->obj = 0.0;
        info->L = 0.0;
    }
    free(q); free(r); free(pd); free(w);
    return status;
}

/* ------------------------------------------------------------------------
 * Algorithm 1, last line / Eq. (3.2): z = -(d/dtheta <theta*x - y, theta*q>) + grad r.
 * d(theta*x)(i,j)/d theta(u,v) = x(i+c0-u, j+c0-v), so
 * Z(u,v) = sum_{c,i,j} rho(i,j) q(i+c0-u, j+c0-v) + w(i,j) x(i+c0-u, j+c0-v)
 * with rho = theta*x - y and w = theta*q.
 * ---------------------------------------------------------------------- */
void oracle_hypergrad(const om_problem* p, const double* th, const double* a, const double* y,
                      const double* xt, const double* q, int32_t with_r, double* z, double* znorm_out) {
    const int64_t N = npix(p);
    const int K = p->K, c0 = (K - 1) / 2, C = p->C, H = p->H, W = p->W, KC = nkc(p);
    double* rho = dalloc(N);
    double* w = dalloc(N);
    oracle_conv(p, th, xt, rho);
    for (int64_t e = 0; e < N; ++e) rho[e] -= y[e];
    oracle_conv(p, th, q, w);
    /* a shared kernel collects every channel's products; kernel channel k of
       a per-channel kernel only those of image channel k */
#pragma omp parallel for collapse(3) schedule(static)
    for (int k = 0; k < KC; ++k)
    for (int u = 0; u < K; ++u)
        for (int v = 0; v < K; ++v) {
            double s = 0.0;
            for (int c = (KC > 1 ? k : 0); c < (KC > 1 ? k + 1 : C); ++c)
                for (int i = 0; i < H; ++i)
                    for (int j = 0; j < W; ++j) {
                        int64_t e = ((int64_t)c * H + i) * W + j;
                        s += rho[e] * at(p, q, c, i + c0 - u, j + c0 - v)
                           + w[e] * at(p, xt, c, i + c0 - u, j + c0 - v);
                    }
            z[(k * K + u) * K + v] = -s;
        }
    if (with_r && p->beta != 0.0 && a) {
        double* gr = dalloc(KC * K * K);
        oracle_sobolev_grad(p, th, a, gr);
        for (int t = 0; t < KC * K * K; ++t) z[t] += gr[t];
        free(gr);
    }
    if (znorm_out) *znorm_out = sqrt(dot(z, z, KC * K * K));
    free(rho); free(w);
}

/* ------------------------------------------------------------------------
 * Algorithm 2 (MAID), one outer iteration k, with the sufficient-decrease
 * function psi of Eq. (3.4):
 *   psi = l(u') + ||grad_x l(u')|| e + L_g/2 e^2 - l(u_k) + ||grad_x l(u_k)|| e + lambda s ||z||^2
 * where l = g + r, grad_x l = grad g, and the trial lower-level solution u'
 * is solved at the current accuracy e = eps_k.
 *
 * Decision trace (om_trace, see the header): free-running, the step records
 * what it decided; with a replay trace it takes every decision from there
 * (iterations and rejected trials of each lower-level solve, iterations of
 * each CG solve, acceptance of each psi test) and records its own values
 * beside the same words.
 * ---------------------------------------------------------------------- */
typedef struct {
    om_trace* t;
    int32_t rp;        /* read position in t->replay */
    int bad;           /* replay trace malformed or a buffer too small */
} tracer;

static void tr_word(tracer* T, int32_t w) {
    if (!T->t || !T->t->words) return;
    if (T->t->n_words >= T->t->cap_words) { T->bad = 1; return; }
    T->t->words[T->t->n_words++] = w;
}
static void tr_value(tracer* T, double v) {
    if (!T->t || !T->t->values) return;
    if (T->t->n_values >= T->t->cap_values) { T->bad = 1; return; }
    T->t->values[T->t->n_values++] = v;
}
static int replaying(const tracer* T) { return T->t && T->t->replay; }
static int32_t rd(tracer* T) {
    if (T->rp >= T->t->n_replay) { T->bad = 1; return 0; }
    return T->t->replay[T->rp++];
}

/* one lower-level solve (role 0: InexactGradient at theta_k, 1: psi trial) */
static int traced_lower(const om_problem* p, const double* th, const double* y, double* x, double tol,
                        int32_t max_iter, double* L, om_solve_info* li, tracer* T, int role) {
    int st;
    if (replaying(T)) {
        int32_t kind = rd(T), rl = rd(T), iters = rd(T), status = rd(T);
        if (kind != 1 || rl != role || iters < 0 || T->rp + iters > T->t->n_replay) { T->bad = 1; return OM_EINVAL; }
        const int32_t* bt = T->t->replay + T->rp;
        T->rp += iters;
        oracle_lower_solve(p, th, y, x, 0.0, iters, L, li, iters > 0 ? bt : NULL, NULL);
        li->status = status;
        st = status;
        tr_word(T, 1); tr_word(T, role); tr_word(T, iters); tr_word(T, status);
        for (int32_t n = 0; n < iters; ++n) tr_word(T, bt[n]);
    } else {
        int32_t* bt = (T->t && T->t->words) ? (int32_t*)calloc((size_t)max_iter + 1, sizeof(int32_t)) : NULL;
        st = oracle_lower_solve(p, th, y, x, tol, max_iter, L, li, NULL, bt);
        tr_word(T, 1); tr_word(T, role); tr_word(T, li->iters); tr_word(T, li->status);
        if (bt) for (int32_t n = 0; n < li->iters; ++n) tr_word(T, bt[n]);
        free(bt);
    }
    tr_value(T, li->res_norm);
    tr_value(T, *L);
    return st;
}

static int traced_cg(const om_problem* p, const double* th, const double* xt, const double* rhs, double* q,
                     double tol, int32_t max_iter, om_solve_info* ci, tracer* T) {
    int st;
    if (replaying(T)) {
        int32_t kind = rd(T), iters = rd(T), status = rd(T);
        if (kind != 3 || iters < 0) { T->bad = 1; return OM_EINVAL; }
        st = oracle_adjoint_solve(p, th, xt, rhs, q, 0.0, iters, ci, NULL);
        if (st != OM_NOT_SPD) { st = status; ci->status = status; }
    } else {
        st = oracle_adjoint_solve(p, th, xt, rhs, q, tol, max_iter, ci, NULL);
    }
    tr_word(T, 3); tr_word(T, ci->iters); tr_word(T, ci->status);
    tr_value(T, ci->res_norm);
    return st;
}

static void traced_upper(tracer* T, int role, double g, double gn, double r) {
    if (replaying(T)) {
        int32_t kind = rd(T), rl = rd(T);
        if (kind != 2 || rl != role) T->bad = 1;
    }
    tr_word(T, 2); tr_word(T, role);
    tr_value(T, g); tr_value(T, gn); tr_value(T, r);
}

int oracle_maid_step_traced(const om_problem* p, const double* a, const double* y, om_state* st,
                            const om_hparams* hp, om_step_info* info, om_trace* trace) {
    if (!p || !a || !y || !st || !hp || !st->theta || !st->x || !st->q || bad_kc(p)) return OM_EINVAL;
    tracer T = {trace, 0, 0};
    if (trace) { trace->n_words = 0; trace->n_values = 0; }
    const int64_t N = npix(p);
    const int KK = nkc(p) * p->K * p->K;    /* every tap of theta */
    double *xt = dalloc(N), *xs = dalloc(N), *G = dalloc(N), *q = dalloc(N);
    double *z = dalloc(KK), *th2 = dalloc(KK);
    double Lg = hp->L_g;
    if (!(Lg > 0)) Lg = l1_bound_sq(p, a);
    om_step_info I; memset(&I, 0, sizeof(I));
    int status = OM_OK;
    int j = hp->max_bt;
    memcpy(xt, st->x, N * sizeof(double));
    memcpy(q, st->q, N * sizeof(double));
    for (;;) {
        /* InexactGradient(theta_k, eps_k, delta_k) */
        om_solve_info li, ci;
        int ls = traced_lower(p, st->theta, y, xt, st->eps * hp->mu, hp->max_lower_iter, &st->L, &li, &T, 0);
        if (T.bad) { status = OM_EINVAL; break; }
        I.lower_iters += li.iters;
        if (ls == OM_MAXITER) I.lower_status = OM_MAXITER;
        double g_k, n_k;
        oracle_upper_value_grad(p, a, y, xt, G, &g_k, &n_k);
        const double r_k = oracle_sobolev_value(p, st->theta, a);
        const double ell_k = g_k + r_k;
        traced_upper(&T, 0, g_k, n_k, r_k);
        int cs = traced_cg(p, st->theta, xt, G, q, st->delta, hp->max_cg_iter, &ci, &T);
        if (T.bad) { status = OM_EINVAL; break; }
        I.cg_iters += ci.iters;
        if (cs == OM_NOT_SPD) { status = OM_NOT_SPD; break; }
        if (cs == OM_MAXITER) I.cg_status = OM_MAXITER;
        double znorm;
        oracle_hypergrad(p, st->theta, a, y, xt, q, 1, z, &znorm);
        if (replaying(&T) && rd(&T) != 4) { status = OM_EINVAL; break; }
        tr_word(&T, 4);
        tr_value(&T, znorm);
        I.ell_k = ell_k;
        I.znorm = znorm;
        /* backtracking on the step size */
        int accepted = 0;
        for (int i = 0; i < j; ++i) {
            for (int t = 0; t < KK; ++t) th2[t] = st->theta[t] - st->step * z[t];
            memcpy(xs, xt, N * sizeof(double));
            ls = traced_lower(p, th2, y, xs, st->eps * hp->mu, hp->max_lower_iter, &st->L, &li, &T, 1);
            if (T.bad) break;
            I.lower_iters += li.iters;
            if (ls == OM_MAXITER) I.lower_status = OM_MAXITER;
            double g_n, n_n;
            oracle_upper_value_grad(p, a, y, xs, NULL, &g_n, &n_n);
            const double r_n = oracle_sobolev_value(p, th2, a);
            const double ell_n = g_n + r_n;
            traced_upper(&T, 1, g_n, n_n, r_n);
            const double e = st->eps;
            const double psi = ell_n + n_n * e + 0.5 * Lg * e * e - ell_k + n_k * e
                             + hp->lambda * st->step * znorm * znorm;
            I.trials += 1;
            I.psi = psi;
            I.ell_next = ell_n;
            int acc = psi <= 0.0;
            if (replaying(&T)) {
                if (rd(&T) != 5) { T.bad = 1; break; }
                acc = rd(&T) != 0;
            }
            tr_word(&T, 5); tr_word(&T, acc);
            tr_value(&T, psi);
            if (acc) {
                memcpy(st->theta, th2, KK * sizeof(double));
                memcpy(xt, xs, N * sizeof(double));
                st->eps *= hp->nu_hi;
                st->delta *= hp->nu_hi;
                st->step *= hp->rho_hi;
                st->k += 1;
                accepted = 1;
                break;
            }
            st->step *= hp->rho_lo;
        }
        if (T.bad) { status = OM_EINVAL; break; }
        if (accepted) { I.accepted = 1; break; }
        st->eps *= hp->nu_lo;
        st->delta *= hp->nu_lo;
        j += 1;
        I.retries += 1;
        if (st->eps < hp->eps_min) { status = OM_ACCURACY_FLOOR; break; }
    }
    memcpy(st->x, xt, N * sizeof(double));
    memcpy(st->q, q, N * sizeof(double));
    if (status == OM_OK && (I.lower_status == OM_MAXITER || I.cg_status == OM_MAXITER)) status = OM_MAXITER;
    I.status = status;
    if (info) *info = I;
    free(xt); free(xs); free(G); free(q); free(z); free(th2);
    return status;
}

int oracle_maid_step(const om_problem* p, const double* a, const double* y, om_state* st,
                     const om_hparams* hp, om_step_info* info) {
    return oracle_maid_step_traced(p, a, y, st, hp, info, NULL);
}

/* ------------------------------------------------------------------------
 * per-pixel evaluations (flat index e = (c*H + i)*W + j)
 * ---------------------------------------------------------------------- */
void oracle_conv_at(const om_problem* p, const double* th, const double* x,
                    const int64_t* idx, int64_t n, double* out) {
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < n; ++t) {
        int64_t e = idx[t];
        int j = (int)(e % p->W), i = (int)((e / p->W) % p->H), c = (int)(e / ((int64_t)p->W * p->H));
        out[t] = conv_px(p, th, x, c, i, j);
    }
}

void oracle_h_grad_at(const om_problem* p, const double* th, const double* y, const double* x,
                      const int64_t* idx, int64_t n, double* out) {
    const int K = p->K, c0 = (K - 1) / 2;
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < n; ++t) {
        int64_t e = idx[t];
        int j = (int)(e % p->W), i = (int)((e / p->W) % p->H), c = (int)(e / ((int64_t)p->W * p->H));
        double s = 0.0;
        for (int u = 0; u < K; ++u)
            for (int v = 0; v < K; ++v) {
                int ii = i - c0 + u, jj = j - c0 + v;
                if (!p->periodic && (ii < 0 || ii >= p->H || jj < 0 || jj >= p->W)) continue;
                if (p->periodic) { ii = wrap(ii, p->H); jj = wrap(jj, p->W); }
                double r = conv_px(p, th, x, c, ii, jj) - y[((int64_t)c * p->H + ii) * p->W + jj];
                s += taps(p, th, c)[u * K + v] * r;
            }
        out[t] = s + p->alpha * reg_grad_px(p, x, c, i, j);
    }
}

void oracle_h_hvp_at(const om_problem* p, const double* th, const double* x, const double* d,
                     const int64_t* idx, int64_t n, double* out) {
    const int K = p->K, c0 = (K - 1) / 2;
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < n; ++t) {
        int64_t e = idx[t];
        int j = (int)(e % p->W), i = (int)((e / p->W) % p->H), c = (int)(e / ((int64_t)p->W * p->H));
        double s = 0.0;
        for (int u = 0; u < K; ++u)
            for (int v = 0; v < K; ++v) {
                int ii = i - c0 + u, jj = j - c0 + v;
                if (!p->periodic && (ii < 0 || ii >= p->H || jj < 0 || jj >= p->W)) continue;
                if (p->periodic) { ii = wrap(ii, p->H); jj = wrap(jj, p->W); }
                s += taps(p, th, c)[u * K + v] * conv_px(p, th, d, c, ii, jj);
            }
        out[t] = s + p->alpha * reg_hvp_px(p, x, d, c, i, j);
    }
}
