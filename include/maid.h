/*
 * maid.h -- C ABI of libmaid, the MI355X (gfx950) implementation of the hot
 * path of MAID (method of adaptive inexact descent) applied to the
 * Sobolev-regularised analytic deep prior (ADP-beta) for semi-blind
 * deblurring, after Salehi, Bubba, Korolev, "Fast Inexact Bilevel
 * Optimization for Analytical Deep Image Priors" (arXiv 2502.09758).
 *
 * The problem (Eq. 2.5 with T(b,x) a 2D convolution, Section 4.2):
 *   upper:  min_theta  g(xhat(theta)) + r(theta),
 *           g(x) = 1/2 ||a*x - y||^2,
 *           r(theta) = beta (w0 ||theta-a||^2 + ||D_h(theta-a)||^2 + ||D_v(theta-a)||^2)
 *   lower:  xhat(theta) = argmin_x h(x;theta) = 1/2 ||theta*x - y||^2 + alpha R(x)
 * with R the smoothed total variation R(x) = sum_p sqrt(s_p^2 + eps^2) - eps,
 * s_p the forward-difference gradient magnitude at pixel p (joint over the
 * colour channels), a the known kernel of the upper-level operator.
 *
 * Conventions for every entry point:
 *   - Images (x, y, q, gradients) are DEVICE arrays, planar [C][H][W],
 *     row-major, contiguous, element type float (MAID_F32) or double
 *     (MAID_F64) as fixed at maid_create.  Kernels theta, a are DEVICE arrays
 *     of kc planes of K*K doubles ([kc][K][K], row-major), K odd, centre
 *     (c0,c0), c0 = (K-1)/2, kc = 1 (one kernel blurs every channel) or
 *     kc = C (channel c blurred by its own plane theta_c; see maid_desc).
 *     Every "K*K doubles" below is kc*K*K doubles.
 *   - (theta*x)_c(i,j) = sum_{u,v} theta_c(u,v) x_c(i+c0-u, j+c0-v), theta_c
 *     the plane of channel c (plane 0 when kc = 1): true convolution, zero
 *     outside the image, same output size.
 *   - Arrays are caller-owned and must not alias each other unless stated.
 *     The library never frees caller memory; a context owns only its
 *     workspace.
 *   - Every call enqueues work on `stream` and returns after that work has
 *     completed (the solvers poll a device-side completion flag once per
 *     chunk of iterations; scalar results are returned in host memory).
 *   - Return codes: MAID_OK, or MAID_MAXITER (a warning: results written,
 *     info holds the last residual), MAID_ACCURACY_FLOOR (maid_step only), or
 *     a negative error, in which case the output arrays are not written and
 *     maid_last_error describes the failure.  No exception crosses the ABI.
 *   - One context serves one stream at a time; calls on one context must not
 *     overlap.  For a given context and tile configuration, results are
 *     bitwise reproducible (all reductions run in a fixed order).
 */
#ifndef MAID_H
#define MAID_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { MAID_F32 = 0, MAID_F64 = 1 };
enum { MAID_BOUNDARY_ZERO = 0, MAID_BOUNDARY_PERIODIC = 1 };
enum { MAID_REG_TV = 0, MAID_REG_TV_CHANNELWISE = 1, MAID_REG_QUADRATIC = 2 };

enum {
    MAID_OK = 0,
    MAID_MAXITER = 1,
    MAID_ACCURACY_FLOOR = 2,
    MAID_EINVAL = -1,
    MAID_ENOMEM = -2,
    MAID_EHIP = -3,
    MAID_NOT_SPD = -4,
    MAID_NONFINITE = -5
};

/* Problem description.  C in 1..3, K odd with 1 <= K <= 31 and K <= min(H,W),
   H*W < 2^31.
   boundary: MAID_BOUNDARY_ZERO (the blur reads zero outside the image; the
   setting of Section 4.2's experiments, and the only one the kernels
   implement: MAID_BOUNDARY_PERIODIC is rejected with MAID_EINVAL).
   reg: MAID_REG_TV (smoothed TV, one gradient magnitude per pixel over all
   channels), MAID_REG_TV_CHANNELWISE (one per channel and pixel) or
   MAID_REG_QUADRATIC (R = 1/2 ||Dx||^2, the Tikhonov case).  alpha >= 0,
   eps_tv > 0 (TV only), beta >= 0, h1_w0 = weight of the L2 part of the H1
   norm (1 full norm, 0 seminorm).
   kc: kernel planes, 0 or 1 for one kernel shared by the channels, C for one
   kernel per colour channel (the colour variant behind Section 4.2's plots of
   a single kernel channel); any other value is rejected with MAID_EINVAL.
   With kc = C the hypergradient has one K*K plane per channel (a channel's
   plane collects only that channel's products), r(theta) sums the planes'
   Sobolev terms (no difference across planes), and the Lipschitz bounds
   ||theta||_1^2 and ||a||_1^2 take the largest plane's l1 norm. */
typedef struct {
    int32_t H, W, C, K, dtype, boundary, reg, kc;
    double alpha, eps_tv, beta, h1_w0;
} maid_desc;

typedef struct {
    int32_t iters;       /* gradient evaluations (lower) / CG iterations */
    int32_t backtracks;  /* rejected trial steps (lower solve only) */
    int32_t status;      /* return code of the solve */
    double res_norm;     /* lower: ||grad h(x)||; CG: recursive residual norm */
    double obj;          /* reserved (0) */
    double L;            /* lower: final Lipschitz estimate */
} maid_solve_info;

/* Algorithm 2 hyperparameters (rho_lo/rho_hi: step-size factors, nu_lo/nu_hi:
   accuracy factors, lambda: sufficient-decrease constant of Eq. 3.4, mu:
   lower-level tolerance scale in Algorithm 1 (tol = eps*mu), L_g: Lipschitz
   constant of grad g in Eq. 3.4 (<= 0: use ||a||_1^2), eps_min: stop with
   MAID_ACCURACY_FLOOR once eps falls below it). */
typedef struct {
    double rho_lo, rho_hi, nu_lo, nu_hi, lambda, mu, L_g, eps_min;
    int32_t max_bt, max_lower_iter, max_cg_iter;
} maid_hparams;

/* MAID state: theta (DEVICE, K*K doubles, updated in place), x and q
   (DEVICE images, warm starts for the lower-level and CG solves, updated in
   place), accuracies eps (lower level) and delta (CG), step size, lower-level
   Lipschitz estimate L (<= 0: start from ||theta||_1^2), outer counter k. */
typedef struct {
    void* theta;
    void* x;
    void* q;
    double eps, delta, step, L;
    int32_t k;
} maid_state;

/* One outer iteration's record: accepted (1 if theta moved), psi trials,
   retries (accuracy reductions), lower-level and CG iterations, the step's
   return code, the last psi of Eq. (3.4), ell(u_k), ell(u') of the last
   trial, ||z||; lower_status / cg_status: MAID_MAXITER if any lower-level /
   CG solve of the step stopped at its iteration cap (the step carries on
   with that solve's result and then returns MAID_MAXITER, a warning, where
   it would otherwise return MAID_OK), else MAID_OK. */
typedef struct {
    int32_t accepted, trials, retries, lower_iters, cg_iters, status;
    double psi, ell_k, ell_next, znorm;
    int32_t lower_status, cg_status;
} maid_step_info;

typedef struct maid_ctx maid_ctx;

/* Allocate a context and its device workspace for problems of this shape on
   the current HIP device.  Errors: MAID_EINVAL (bad description; nothing
   allocated), MAID_ENOMEM, MAID_EHIP.  *out is NULL on error. */
int maid_create(const maid_desc* desc, maid_ctx** out);
void maid_destroy(maid_ctx* ctx);
/* Text of the last error on this context ("" if none); valid until the next
   call on the context.  maid_last_error(NULL) reports the last maid_create
   failure of the calling thread. */
const char* maid_last_error(const maid_ctx* ctx);
/* Name of the tile configuration (rows per thread) chosen for each group of
   instances. */
const char* maid_config_string(const maid_ctx* ctx);
/* Override the rows-per-thread tile parameter of the stencil kernels for
   every instance (1, 2, 4 or 8; 8 applies to K >= 5, K <= 3 uses 4 at most;
   0 = back to the autotuner's choice, else the size rule). */
int maid_set_tile_rows(maid_ctx* ctx, int32_t rows);
/* Persistent loops for small instances.  The lower-level and CG loops of a
   group of instances with at most 16384 pixels each (and tile rows 1, 2 or 4)
   run inside one kernel per solve on teams of blocks, one team per XCD,
   which meet at barriers through the XCD's L2 instead of at kernel
   boundaries; a batch runs up to eight instances at once.  Results are
   bitwise those of the multi-kernel passes (same passes, same sums).
   members: -1 = size rule (one member per tile of the group's largest
   instance, capped by occupancy and by the tiles of the smallest instance),
   0 = never, 1..128 = that many (capped the same way; larger instances
   then take the team path too).  If a team cannot assemble (its blocks not
   resident together), the solve is repeated on the multi-kernel passes
   and the context stays on them.  The choice shows in
   maid_config_string ("team=P"). */
int maid_set_team(maid_ctx* ctx, int32_t members);
/* One-pass CG (enable != 0; off by default) for the instances on the
   one-pass lower-level form: the Chronopoulos-Gear recurrences need one
   reduction and so one pass per iteration (measured at 256x256, K = 9: 11.9
   against 14.7 us per iteration); 0 (the default) = the three-pass
   Hestenes-Stiefel kernels (the oracle's form) for every instance.  The
   one-pass forms are opt-in because GPUs were lost while their tests ran
   and no cause has been found.  Both forms' iterates drift from the
   oracle's by loss of orthogonality, the one-pass form's differently
   (measured at equal iteration counts: FP64, 30-50 iterations, <= 1.6e-6
   relative against <= 1e-6; FP32, 83 iterations, 2.2e-5 against 4.7e-5). */
int maid_set_one_pass_cg(maid_ctx* ctx, int32_t enable);
/* Matrix cores for the large-kernel correlations (enable != 0, the
   default): with FP32 storage, K >= 13 and tiles of 4 or 8 rows per thread,
   the K x K correlations of the solver passes (Proposition 1's gradient and
   Hessian products) and of the hypergradient's convolutions run as banded
   products on v_mfma_f32_16x16x32_f16, each FP32 operand split into two
   FP16 parts (three products; tile and kernel scaled by powers of two),
   accumulated in FP32; 0 = the FP32 vector ALUs.  Both are deterministic;
   they round differently (measured on random tiles: within 4e-7 of the
   FP64 correlation, relative to the largest output).  FP64 storage and the
   upper-level convolutions (FP64 taps and sums) are unaffected.  Takes
   effect at the next call. */
int maid_set_mfma(maid_ctx* ctx, int32_t enable);
/* Lower-level form of the instances that can take the one-pass form (one
   channel, 3 <= K <= 11, tile rows <= 4): mode -1 (the default) or 0 = two
   passes per iteration; 1 = one pass (opt-in, see maid_set_one_pass_cg).  With the same tile rows and form, an instance
   computes bitwise the same in any context (alone or in any batch).
   MAID_EINVAL for another mode. */
int maid_set_one_pass(maid_ctx* ctx, int32_t mode);
/* out[i] (HOST, maid_batch_size entries) = 1 if instance i runs the
   one-pass lower-level form under the context's current layout, else 0. */
int maid_one_pass_forms(const maid_ctx* ctx, int32_t* out);
/* Autotuner: for each group of instances with the same K, time a short
   lower-level solve and a short CG solve (probe_iters iterations each,
   1..1000, tolerance 0) with every rows-per-thread candidate on
   the caller's data (theta[i], y[i]: HOST arrays of n DEVICE pointers, as
   for the batched calls; only workspace is written) and keep the fastest
   (candidates 1, 2, 4, and 8 for K >= 5; each with the lower-level form
   the layout takes: the one-pass form where the context is pinned to it,
   maid_set_one_pass(ctx, 1), and it applies, else the two-pass form; each
   candidate runs twice and the second run, with the launch predictors
   set, is timed).
   rows_out (HOST, n, nullable): the choice per instance.  A later
   maid_set_tile_rows(ctx, r != 0) overrides the choice. */
int maid_autotune(maid_ctx* ctx, const void* const* theta, const void* const* y, int32_t probe_iters,
                  int32_t* rows_out, hipStream_t stream);

/* Algorithm 1, lower-level solve: accelerated gradient (FISTA) with
   backtracking (factor 2) on min_x h(x;theta).  Each iteration evaluates
   G = grad h(v) at the extrapolated point v and stops there once
   ||G||_2 <= tol (Algorithm 1 uses tol = eps * mu(b)), returning v; otherwise
   it steps x+ = v - G/L and doubles L until h(x+) - h(v) <= -||G||^2/(2L).
   x: in = starting point, out = the returned point.  L_inout: Lipschitz
   estimate in/out (<= 0 on input: ||theta||_1^2).  trace_bt (HOST, nullable,
   length >= max_iter): rejected trials per iteration.  info: nullable.
   Two forms of one iteration: two passes (gradient, then trial step), or
   -- for one channel and 3 <= K <= 11 -- one pass in which every tile also
   computes G on its convolution halo and takes the trial step at once (the
   stop and decrease tests move to the start of the next pass; the same
   decisions, iterates equal to rounding of the partial sums).  The
   autotuner chooses per K; untuned, the one-pass form is used for instances
   of at most 320 of its tiles of 64 - (K - 1) columns by 8 rows (about
   380 x 380 for K = 9 at one row per thread). */
int maid_lower_solve(maid_ctx* ctx, const void* theta, const void* y, void* x,
                     double tol, int32_t max_iter, double* L_inout,
                     maid_solve_info* info, int32_t* trace_bt, hipStream_t stream);

/* Outcome of maid_lower_solve_refined's Newton steps. */
typedef struct {
    int32_t newton_steps;   /* steps taken (an undone step not counted) */
    int32_t cg_iters;       /* CG iterations over all steps */
    int32_t status;         /* MAID_OK: rel_step <= rel_tol; MAID_MAXITER otherwise */
    double rel_step;        /* ||d|| / ||x|| of the last step taken */
    double grad_norm;       /* ||grad_x h|| at the returned x (residual with FP64 sums) */
} maid_refine_info;

/* The precision form of Algorithm 1's lower-level solve (Section 4's
   accuracy at any storage type): maid_lower_solve to tol (FISTA), then
   Newton refinement -- steps x <- x - d with
   (theta.theta* + alpha grad^2 R(x)) d = grad_x h(x) (Proposition 1's
   Hessian and gradient), d solved by CG (the adjoint kernels) in the
   storage type to 1e-2 relative residual.  With FP32 storage this is
   mixed-precision iterative refinement: the iterate is accumulated in FP64,
   its gradient is evaluated by the FP64 passes of a companion FP64 context
   of the same shape (allocated at the first call on the context, about
   twice the context's own workspace, kept until maid_destroy), and x is that
   iterate rounded to FP32.  Steps stop when ||d|| <= rel_tol ||x||, when a
   step is larger than the one before (it is undone; MAXITER), or after
   max_newton steps.  Arrays as in maid_lower_solve; info describes the
   FISTA phase, rinfo (nullable) the refinement (grad_norm: the FP64
   gradient norm at the FP64 iterate).  Returns the FISTA phase's error if
   it failed, else MAID_OK / MAID_MAXITER of the refinement, or an error. */
int maid_lower_solve_refined(maid_ctx* ctx, const void* theta, const void* y, void* x, double tol,
                             int32_t max_iter, double rel_tol, int32_t max_newton, int32_t max_cg,
                             double* L_inout, maid_solve_info* info, maid_refine_info* rinfo,
                             hipStream_t stream);

/* Upper-level value and gradient at x (Eq. 2.5 with T(a, .) the blur by the
   known kernel a; its gradient is the right-hand side of Algorithm 1's
   Hessian system): rho = a*x - y, g = 1/2||rho||^2, grad_out = a.rho
   (adjoint convolution; nullable), gradnorm = ||grad||_2. */
int maid_upper_value_grad(maid_ctx* ctx, const void* a, const void* y, const void* x,
                          void* grad_out, double* g_out, double* gradnorm_out,
                          hipStream_t stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
   serving loops, harnesses that forbid allocation): maid_upper_value_grad
   of one instance described by `desc`, with no context.  The same kernels
   and the same arithmetic as maid_upper_value_grad on a new context of
   that description (tile rows from the size rule), so the results are
   bitwise equal.  Its workspace (instance table, the kernel a in the
   storage type, per-block partial sums, reduction slots, the residual
   a*x - y, and the gradient when grad_out is NULL) is one fixed device
   array of 64 MiB in the library, held by every device the library runs on
   until the process ends: instances needing more (C*H*W*element size above
   about 64 MiB, half that with grad_out NULL) are rejected with
   MAID_EINVAL before any GPU work.  No hipMalloc, hipFree or other
   allocation is made.  All calls on one device share that array and
   overwrite it: calls that overlap on one device (other streams, other
   host threads) race and must not be made.  Arrays as in
   maid_upper_value_grad (device pointers, desc->dtype storage, a FP64);
   the call synchronises `stream` and writes g and ||grad g|| to the host
   pointers (nullable).  why (nullable): on an error, a message valid until
   the next call on this host thread. */
int maid_upper_value_grad_noalloc(const maid_desc* desc, const void* a, const void* y, const void* x,
                                  void* grad_out, double* g_out, double* gradnorm_out, const char** why,
                                  hipStream_t stream);

/* Algorithm 1, Hessian system: conjugate gradients on
   (theta.theta* + alpha grad^2 R(x_tilde)) q = rhs, stopping when the
   recursive residual satisfies ||r||_2 <= tol (the accuracy delta).
   q: in = starting point, out = solution.  MAID_NOT_SPD if a curvature
   <p,Hp> <= 0 is met (q not written).  Instances on the one-pass form (see
   maid_lower_solve) run the Chronopoulos-Gear form of CG, which needs one
   reduction per iteration (<r,r> and <r,Hr> together) and so one pass:
   the same iterates in exact arithmetic, the same stop and curvature
   tests; see maid_set_one_pass_cg. */
int maid_adjoint_solve(maid_ctx* ctx, const void* theta, const void* x_tilde,
                       const void* rhs, void* q, double tol, int32_t max_iter,
                       maid_solve_info* info, hipStream_t stream);

/* Algorithm 1, last line, and Eq. (3.2): the hypergradient
   z(u,v) = -sum_{c,i,j} [rho_c(i,j) q_c(i+c0-u,j+c0-v) + (theta*q)_c(i,j) x_c(i+c0-u,j+c0-v)]
            + with_r * grad r(theta)(u,v),
   rho = theta*x_tilde - y; with kc = C, plane c of z sums over channel c
   only.  z: DEVICE, K*K doubles.  a may be NULL when
   with_r == 0 or beta == 0.  znorm_out (HOST, nullable) = ||z||_2. */
int maid_hypergrad(maid_ctx* ctx, const void* theta, const void* a, const void* y,
                   const void* x_tilde, const void* q, int32_t with_r, double* z,
                   double* znorm_out, hipStream_t stream);

/* The blur operator T(theta, .) of Eq. (2.4) as a 2D convolution:
   out = theta * in (adjoint = 0) or out = theta . in, the adjoint correlation
   (adjoint = 1), zero boundary, same size.  in and out must not alias. */
int maid_apply_operator(maid_ctx* ctx, const void* theta, const void* in, void* out, int32_t adjoint,
                        hipStream_t stream);

/* The objective values used by Eq. (3.4): r(theta) (HOST out). */
int maid_sobolev_value(maid_ctx* ctx, const void* theta, const void* a, double* r_out,
                       hipStream_t stream);

/* Algorithm 2, one outer iteration k: the retry loop over accuracies
   (j = max_bt, max_bt+1, ...), each computing InexactGradient and testing up
   to j step sizes with psi(step) <= 0 (Eq. 3.4, all terms in FP64; the trial
   lower-level solve runs at the current accuracy eps); on success
   theta <- theta - step*z and eps, delta, step grow by nu_hi, nu_hi, rho_hi;
   on failure of all j trials eps, delta shrink by nu_lo.  Returns
   MAID_ACCURACY_FLOOR (theta unchanged) once eps < eps_min. */
int maid_step(maid_ctx* ctx, const void* a, const void* y, maid_state* state,
              const maid_hparams* hp, maid_step_info* info, hipStream_t stream);

/* Decision trace of Algorithm 2, for a checker that replays the step's
   decisions (the same solves with the same iteration counts, rejected trials
   and acceptances, so that the two sides can be compared value by value
   where a free-running comparison would diverge on rounding).  While
   set, every maid_step / maid_batch_step call writes, for instance `inst`,
   from the start of the caller's HOST buffers, in the order the work runs:
     lower-level solve  words 1, role, iters, status, then the rejected trial
                        steps of each of its iters iterations;
                        values ||grad h|| at the returned point, L after
                        (role 0: the InexactGradient solve at theta_k,
                         role 1: the solve of a psi trial at theta')
     upper level        words 2, role;           values g, ||grad g||, r(theta)
     CG solve           words 3, iters, status;  values recursive residual
     hypergradient      words 4;                 values ||z||
     psi test           words 5, accepted;       values psi
   Tracing reads the backtracking record of every traced solve back at once
   (host round trips; the results are unchanged).  words == NULL turns it
   off.  A step whose trace outgrows the buffers returns MAID_EINVAL after
   completing.  maid_step_trace_length reports the words and values written
   by the last step. */
int maid_set_step_trace(maid_ctx* ctx, int32_t inst, int32_t* words, int32_t cap_words, double* values,
                        int32_t cap_values);
int maid_step_trace_length(const maid_ctx* ctx, int32_t* n_words, int32_t* n_values);

/* ---------------------------------------------------------------- Section 4.1's baselines
   The two methods MAID is compared with in Section 4.1 (ADP-IFT and
   ADP-LISTA), rebuilt on this library's kernels for the 2D problem.  Both
   run the proximal-gradient iteration of the lower level with a fixed step
   lambda_x; the smooth TV regulariser's proximal map is the identity, so an
   iteration is x <- x - lambda_x grad_x h(x; theta).  Single-instance
   contexts only. */

/* n_iter fixed-step iterations x_{k+1} = x_k - step grad_x h(x_k; theta)
   (fewer if ||grad_x h(x_k)|| <= tol first; tol = 0: exactly n_iter), on the
   FISTA passes with the momentum off and every step accepted.  x: in x_0,
   out the last iterate.  hist (DEVICE, nullable, n_iter*C*H*W elements of
   the storage type): x_1 .. x_n in order, x_k at hist + (k-1)*C*H*W; it
   needs the two-pass lower-level form (maid_set_one_pass(ctx, 0) for
   instances that would take the one-pass form; MAID_EINVAL otherwise).
   info as for maid_lower_solve (iters = steps taken, backtracks 0, L =
   1/step).  Returns MAID_OK if the tolerance was met, MAID_MAXITER after
   n_iter steps, or an error. */
int maid_gd_solve(maid_ctx* ctx, const void* theta, const void* y, void* x, double step, int32_t n_iter,
                  double tol, void* hist, maid_solve_info* info, hipStream_t stream);

/* Proposition 1's Hessian of the lower level at x applied to w:
   out = (theta.theta* + alpha grad^2 R(x)) w, computed by the adjoint
   solve's set-up passes (the same kernels and arithmetic as its products).
   out must not alias x or w. */
int maid_hessian_apply(maid_ctx* ctx, const void* theta, const void* x, const void* w, void* out,
                       hipStream_t stream);

/* One upper-level iteration of ADP-IFT: n_lower fixed-step iterations of
   the lower level from state->x (warm start), the upper-level gradient
   there, CG on H(x) q = grad g (Algorithm 1's Hessian system) from state->q
   to ||r|| <= cg_tol ||grad g|| or max_cg iterations, the hypergradient z of
   Eq. (3.2) (with the Sobolev term), and theta <- theta - state->step z.
   state->theta, x and q are updated in place, state->k incremented (eps,
   delta, L unused).  info (HOST, nullable): lower_iters, cg_iters, ell_k =
   g(x) + r(theta) before the step, znorm = ||z||, cg_status; accepted =
   trials = 1.  Returns MAID_MAXITER if CG stopped at max_cg. */
int maid_ift_step(maid_ctx* ctx, const void* a, const void* y, maid_state* state, int32_t n_lower,
                  double lambda_x, double cg_tol, int32_t max_cg, maid_step_info* info, hipStream_t stream);

/* One upper-level iteration of ADP-LISTA: n_unroll fixed-step iterations
   from state->x, keeping every iterate (library workspace, allocated at the
   first call and grown on demand: (n_unroll + 1)*C*H*W elements), the loss
   g(x_n) + r(theta), its exact gradient in theta through the unrolled
   iterations by the reverse recursion
     w_n = grad g(x_n),  dtheta = grad r(theta) + lambda_x sum_k z(x_k, w_{k+1}),
     w_k = w_{k+1} - lambda_x H(x_k) w_{k+1},
   with z(x, w) = -(d grad_x h / d theta)^T w (the correlation of Eq. 3.2)
   and H Proposition 1's Hessian, and theta <- theta - state->step dtheta.
   state->x becomes x_n, state->k is incremented (q, eps, delta, L unused).
   Needs the two-pass lower-level form (maid_set_one_pass(ctx, 0);
   MAID_EINVAL otherwise).  info (HOST, nullable): lower_iters = n_unroll,
   cg_iters = Hessian products taken, ell_k = the loss before the step,
   znorm = ||dtheta||; accepted = trials = 1. */
int maid_lista_step(maid_ctx* ctx, const void* a, const void* y, maid_state* state, int32_t n_unroll,
                    double lambda_x, maid_step_info* info, hipStream_t stream);

/* ---------------------------------------------------------------- batched form
   One context over n independent problem instances of different sizes (a
   ragged batch; each instance has its own maid_desc, all with the same
   dtype).  Every solver pass is one kernel launch per group of instances
   that share K and the tile configuration, covering all tiles of all
   instances of the group; elementwise passes are one launch for the whole
   batch.  Each instance keeps its own solver state, tolerance, step sizes
   and decisions, so its results are bitwise those of a context created for
   it alone (same tile configuration).  maid_create(desc, out) is
   maid_create_batch(desc, 1, out); the single-instance entry points above
   require a context of one instance (MAID_EINVAL otherwise), the
   maid_batch_* entry points accept any.

   Per-instance arguments are HOST arrays of length n: of DEVICE pointers
   (images and kernels, as for the single-instance calls), of tolerances, of
   Lipschitz estimates (in/out), of maid_state (updated in place), of info
   records (nullable; info[i].status holds instance i's code).  The return
   value is a negative error of the call as a whole (bad argument, HIP
   failure; nothing written), else MAID_OK if every instance returned
   MAID_OK, else the code of the first instance that did not (instances with
   a negative code leave their outputs unwritten; the others are written). */
int maid_create_batch(const maid_desc* descs, int32_t n, maid_ctx** out);
/* The same call under the name maid_batch_create. */
int maid_batch_create(const maid_desc* descs, int32_t n, maid_ctx** out);
/* Number of instances of a context (0 for NULL). */
int32_t maid_batch_size(const maid_ctx* ctx);
/* maid_lower_solve for every instance i: theta[i], y[i], x[i] (in/out),
   tol[i], L_inout[i]; one max_iter for all. */
int maid_batch_lower_solve(maid_ctx* ctx, const void* const* theta, const void* const* y,
                           void* const* x, const double* tol, int32_t max_iter,
                           double* L_inout, maid_solve_info* info, hipStream_t stream);
/* maid_adjoint_solve for every instance i. */
int maid_batch_adjoint_solve(maid_ctx* ctx, const void* const* theta, const void* const* x_tilde,
                             const void* const* rhs, void* const* q, const double* tol,
                             int32_t max_iter, maid_solve_info* info, hipStream_t stream);
/* maid_upper_value_grad for every instance i: a[i], y[i], x[i], grad_out[i]
   (grad_out nullable, or any of its entries NULL), g_out[i] and
   gradnorm_out[i] (HOST arrays of n, nullable). */
int maid_batch_upper_value_grad(maid_ctx* ctx, const void* const* a, const void* const* y,
                                const void* const* x, void* const* grad_out, double* g_out,
                                double* gradnorm_out, hipStream_t stream);
/* maid_hypergrad for every instance i: z[i] (DEVICE, K_i*K_i doubles),
   znorm_out[i] (HOST array of n, nullable); a may be NULL when with_r == 0. */
int maid_batch_hypergrad(maid_ctx* ctx, const void* const* theta, const void* const* a,
                         const void* const* y, const void* const* x_tilde, const void* const* q,
                         int32_t with_r, void* const* z, double* znorm_out, hipStream_t stream);
/* maid_step for every instance i (one outer iteration of Algorithm 2 each,
   run in lockstep: the lower-level, CG and trial solves of all instances
   that need one at the same point of the algorithm share launches); one set
   of hyperparameters for all. */
int maid_batch_step(maid_ctx* ctx, const void* const* a, const void* const* y,
                    maid_state* states, const maid_hparams* hp, maid_step_info* info,
                    hipStream_t stream);
/* n_steps (>= 1) outer iterations of Algorithm 2 for every instance, in
   lockstep as maid_batch_step (the same as n_steps calls of it, except that
   an instance whose step returns MAID_ACCURACY_FLOOR or an error takes no
   further step).  info[i] (HOST, nullable): accepted, trials, retries,
   lower_iters and cg_iters summed over the instance's steps; psi, ell_k,
   ell_next, znorm and status of its last step; lower_status / cg_status
   MAID_MAXITER if any of its solves stopped at the cap.  Returns the first
   instance's final code that is not MAID_OK (a cap reached in any step
   counts as MAID_MAXITER unless a later step ended the instance's run). */
int maid_batch_steps(maid_ctx* ctx, const void* const* a, const void* const* y,
                     maid_state* states, const maid_hparams* hp, maid_step_info* info,
                     int32_t n_steps, hipStream_t stream);

/* Kernel timing (for measurement and profiling tools).  maid_profile(ctx, 1)
   resets the counters and, until maid_profile(ctx, 0), launches every kernel
   of the context directly (no graph replay) with a pair of HIP events that
   the dispatch stamps with the kernel's own start and end times;
   maid_profile_read returns, for one kernel kind, the number of timed
   launches, how many of them did a pass of work (solver passes launched in
   a chunk exit early once the solve has finished or when a backtracking
   step needs no gradient; work_launches is nullable), and their summed GPU
   duration in milliseconds. */
enum {
    MAID_PROF_CONV = 0,       /* convolution / adjoint passes (setup, upper level, hypergradient) */
    MAID_PROF_APG_GRAD = 1,   /* lower level: gradient at the extrapolated point */
    MAID_PROF_APG_TRIAL = 2,  /* lower level: trial step and decrease test */
    MAID_PROF_CG_DIR = 3,     /* CG: new direction and theta*p */
    MAID_PROF_CG_HVP = 4,     /* CG: Hessian-vector product and curvature */
    MAID_PROF_CG_UPDATE = 5,  /* CG: q, r update and residual norm */
    MAID_PROF_HG_CORR = 6,    /* hypergradient correlation (FP64 MFMA) */
    MAID_PROF_OTHER = 7,      /* small kernels */
    MAID_PROF_APG_TEAM = 8,   /* lower-level loop of small instances on one team per XCD (work: slots) */
    MAID_PROF_CG_TEAM = 9,    /* CG loop of small instances on one team per XCD (work: iterations) */
    MAID_PROF_APG_STEP = 10,  /* lower level, one-pass form: gradient and trial step in one pass */
    MAID_PROF_CG_STEP = 11,   /* CG, one-pass form: update and Hessian product in one pass */
    MAID_PROF_KINDS = 12
};
int maid_profile(maid_ctx* ctx, int32_t enable);
int maid_profile_read(maid_ctx* ctx, int32_t kind, int64_t* launches, int64_t* work_launches, double* total_ms);
const char* maid_profile_name(int32_t kind);

#ifdef __cplusplus
}
#endif
#endif
