/*
 * maid_oracle.h -- FP64 CPU oracle for the MAID hot path (TEST INFRASTRUCTURE).
 *
 * This library exists only to check the HIP path.  It is a plain, slow,
 * double-precision transcription of the mathematics of
 *   Salehi, Bubba, Korolev, "Fast Inexact Bilevel Optimization for Analytical
 *   Deep Image Priors" (arXiv 2502.09758):
 *     - the ADP-beta bilevel problem, Eq. (2.5), with T(b,x) a 2D convolution
 *       (Section 4.2) and the smoothed TV regulariser of Section 4.2;
 *     - the IFT hypergradient, Eq. (3.2);
 *     - Algorithm 1 (InexactGradient) and Algorithm 2 (MAID) with the
 *       sufficient-decrease function psi of Eq. (3.4);
 *     - the lower-level gradient and Hessian of Proposition 1.
 * Only tests/, the package's smoke() entry and bench.py's CPU-baseline leg may
 * load it.  It shares no code, header or constant with the HIP library.
 *
 * Conventions (every array is double, contiguous, host memory):
 *   images x, y, q: planar [C][H][W], row-major, index (c,i,j), i = row;
 *   kernels theta, a: [kc][K][K] row-major, K odd, c0 = (K-1)/2, with kc = 1
 *   (one kernel shared by every channel) or kc = C (channel c blurred by its
 *   own kernel theta_c: the colour variant that Section 4.2's figures imply
 *   when they plot one channel of the kernel); theta_c means theta_0 when kc = 1;
 *   (theta*x)_c(i,j)   = sum_{u,v} theta_c(u,v) x_c(i+c0-u, j+c0-v)
 *   (theta.r)_c(i,j)   = sum_{u,v} theta_c(u,v) r_c(i-c0+u, j-c0+v)   (adjoint)
 *   with x = 0 outside the image (periodic mode wraps; test only).
 *   D_h x(i,j) = x(i,j+1)-x(i,j) for j<W-1 else 0, D_v likewise on rows
 *   (periodic mode wraps instead).
 *   Smoothed TV: R(x) = sum_p phi(s_p), phi(s) = sqrt(s^2+eps^2) - eps,
 *   s_p^2 = sum_c (D_h x_c)_p^2 + (D_v x_c)_p^2  (vectorial, reg=0), or per
 *   channel (reg=1); reg=2 is the quadratic R = 1/2 ||Dx||^2 used by the
 *   closed-form tests.
 *   h(x;theta) = 1/2 ||theta*x - y||^2 + alpha R(x)          (lower level)
 *   g(x)       = 1/2 ||a*x - y||^2                            (upper level)
 *   r(theta)   = beta ( w0 ||theta-a||^2 + ||D_h(theta-a)||^2 + ||D_v(theta-a)||^2 )
 *   with Neumann forward differences on each KxK grid (no difference across
 *   kernel channels).
 */
#ifndef MAID_ORACLE_H
#define MAID_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t C, H, W, K;
    int32_t periodic;   /* 0 zero boundary, 1 periodic (tests only) */
    int32_t reg;        /* 0 vectorial TV, 1 channelwise TV, 2 quadratic */
    int32_t kc;         /* kernel channels: 0 or 1 shared kernel, C per channel */
    double alpha, eps_tv, beta, h1_w0;
} om_problem;

typedef struct {
    int32_t iters, backtracks, status;
    double res_norm, obj, L;
} om_solve_info;

typedef struct {
    double rho_lo, rho_hi, nu_lo, nu_hi, lambda, mu, L_g, eps_min;
    int32_t max_bt, max_lower_iter, max_cg_iter;
} om_hparams;

typedef struct {
    double *theta, *x, *q;              /* kc*K*K, N, N (warm starts in/out) */
    double eps, delta, step, L;
    int32_t k;
} om_state;

typedef struct {
    int32_t accepted, trials, retries, lower_iters, cg_iters, status;
    double psi, ell_k, ell_next, znorm;
    /* worst status (OM_OK or OM_MAXITER) of the step's lower-level solves and
       of its CG solves: a solve that stops at its iteration cap is carried on
       with (Section 4.1 reports the lower-level cap as never reached) and
       flagged here, and the step then returns OM_MAXITER unless it ends in
       another non-OK state */
    int32_t lower_status, cg_status;
} om_step_info;

enum { OM_OK = 0, OM_MAXITER = 1, OM_ACCURACY_FLOOR = 2, OM_EINVAL = -1, OM_NOT_SPD = -4 };

/* OpenMP threads of the whole-image loops (results do not depend on it) */
int  oracle_num_threads(void);
void oracle_set_num_threads(int n);

/* operators */
void   oracle_conv(const om_problem*, const double* th, const double* x, double* out);
void   oracle_conv_adj(const om_problem*, const double* th, const double* r, double* out);
void   oracle_diff(const om_problem*, const double* x, double* dh, double* dv);
void   oracle_diff_adj(const om_problem*, const double* ph, const double* pv, double* out);
double oracle_reg_value(const om_problem*, const double* x);
void   oracle_reg_grad(const om_problem*, const double* x, double* out);
void   oracle_reg_hvp(const om_problem*, const double* x, const double* d, double* out);
double oracle_h_value(const om_problem*, const double* th, const double* y, const double* x);
void   oracle_h_grad(const om_problem*, const double* th, const double* y, const double* x, double* out);
void   oracle_h_hvp(const om_problem*, const double* th, const double* x, const double* d, double* out);
double oracle_sobolev_value(const om_problem*, const double* th, const double* a);
void   oracle_sobolev_grad(const om_problem*, const double* th, const double* a, double* out);

/* Alg. 1, line "solve the lower-level problem": FISTA with backtracking. */
int oracle_lower_solve(const om_problem*, const double* th, const double* y, double* x,
                       double tol, int32_t max_iter, double* L_inout, om_solve_info* info,
                       const int32_t* replay_bt, int32_t* trace_bt);
/* value and gradient of g at x (r is not included). */
void oracle_upper_value_grad(const om_problem*, const double* a, const double* y, const double* x,
                             double* grad_out, double* g_out, double* gradnorm_out);
/* Alg. 1, line "solve the Hessian system with residual delta": CG. */
int oracle_adjoint_solve(const om_problem*, const double* th, const double* xt, const double* rhs,
                         double* q, double tol, int32_t max_iter, om_solve_info* info,
                         double* true_res_out);
/* Alg. 1, last line: z = -(d^2 h / dx dtheta)^T q + grad r. a may be NULL if beta == 0;
   with_r = 0 drops grad r (the autograd backward). */
void oracle_hypergrad(const om_problem*, const double* th, const double* a, const double* y,
                      const double* xt, const double* q, int32_t with_r, double* z, double* znorm_out);
/* Alg. 2: one outer step (the for-j retry loop and the accepted update). */
int oracle_maid_step(const om_problem*, const double* a, const double* y, om_state* st,
                     const om_hparams* hp, om_step_info* info);

/* Decision trace of one Algorithm 2 step, in the order the work happens.
   Records (int32 words; FP64 values beside them):
     lower-level solve  words 1, role, iters, status, rejected trials of each
                        of the iters iterations;  values ||grad h||, L after
                        (role 0: the InexactGradient solve at theta_k,
                         role 1: a psi trial solve at theta')
     upper level        words 2, role;            values g, ||grad g||, r(theta)
     CG solve           words 3, iters, status;   values recursive residual norm
     hypergradient      words 4;                  values ||z||
     psi test           words 5, accepted;        values psi
   Free-running (replay == NULL) the step records its own decisions.  With a
   replay trace it takes every decision from there instead (each lower solve
   runs exactly `iters` iterations rejecting the recorded trials, each CG
   solve exactly `iters` iterations, each psi test takes the recorded
   acceptance) and records the same words with its own values, so the two
   traces can be compared value by value.  A malformed replay trace or a
   full buffer makes the step return OM_EINVAL. */
typedef struct {
    const int32_t* replay;    /* nullable */
    int32_t n_replay;
    int32_t* words;           /* nullable: no recording */
    double* values;
    int32_t cap_words, cap_values;
    int32_t n_words, n_values;   /* out */
} om_trace;
int oracle_maid_step_traced(const om_problem*, const double* a, const double* y, om_state* st,
                            const om_hparams* hp, om_step_info* info, om_trace* trace);

/* per-pixel evaluations, for sampled checks at sizes where whole-image
   oracle passes are too slow: out[n] = value at flat index idx[n] */
void oracle_h_grad_at(const om_problem*, const double* th, const double* y, const double* x,
                      const int64_t* idx, int64_t n, double* out);
void oracle_h_hvp_at(const om_problem*, const double* th, const double* x, const double* d,
                     const int64_t* idx, int64_t n, double* out);
void oracle_conv_at(const om_problem*, const double* th, const double* x,
                    const int64_t* idx, int64_t n, double* out);

#ifdef __cplusplus
}
#endif
#endif
