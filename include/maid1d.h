/*
 * maid1d.h -- C ABI of the 1D problem of Section 4.1 in libmaid: ADP-beta
 * (Eq. 2.5) with beta = 0 for a signal of n samples whose operators are full
 * n x n matrices, and MAID (Algorithm 2) on the lower level's matrix B:
 *   upper:  min_B  g(xhat(B)) = 1/2 ||A xhat(B) - y||^2
 *   lower:  xhat(B) = argmin_x  h(x; B) = 1/2 ||B x - y||^2 + alpha1 ||x||_1 + alpha2 ||x||_2^2
 * (the elastic-net regulariser of Section 4.1), A the known blur matrix.
 * The lower level is solved by proximal gradient with a fixed step (Section
 * 4.1); the implicit-function adjoint is taken on the support of the
 * lower-level solution, where h is twice differentiable.
 *
 * A context holds `batch` independent instances of the same size n (a
 * batch of signals, each with its own y, B and state; one A for all).
 * Conventions as in maid.h: DEVICE arrays, caller-owned, FP64, row-major
 * matrices ([batch][n][n] for B, [n][n] for A, [batch][n] for vectors);
 * every call returns after its work has completed; return codes MAID_OK,
 * MAID_MAXITER (a warning), MAID_ACCURACY_FLOOR, or a negative error with
 * maid_last_error describing it.  Per-instance arrays of tolerances and
 * results are HOST arrays of length batch.
 */
#ifndef MAID1D_H
#define MAID1D_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#include "maid.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t n;        /* signal length, 1 <= n <= 4096 */
    int32_t batch;    /* instances, >= 1 */
    double alpha1;    /* weight of ||x||_1, >= 0 */
    double alpha2;    /* weight of ||x||_2^2, > 0 (the lower level is then strongly convex) */
} maid1d_desc;

typedef struct maid1d_ctx maid1d_ctx;

/* Allocate a context and its workspace (about 5 n^2 + 16 n doubles per
   instance).  MAID_EINVAL for a bad description, MAID_ENOMEM, MAID_EHIP. */
int maid1d_create(const maid1d_desc* desc, maid1d_ctx** out);
void maid1d_destroy(maid1d_ctx* ctx);
/* The last error on this context ("" if none); maid1d_last_error(NULL): the
   last maid1d_create failure of the calling thread. */
const char* maid1d_last_error(const maid1d_ctx* ctx);

/* Section 4.1's lower-level solver for every instance: proximal gradient with
   the fixed step `step`,
     x <- S_{step alpha1}(x - step (B^T (B x - y) + 2 alpha2 x)),
   S_t the soft threshold (the proximal map of t ||.||_1), stopped at the
   first iterate x with ||x - x+|| / step <= tol[i] (the proximal-gradient
   mapping, the nonsmooth counterpart of Algorithm 1's gradient test; that
   iterate is returned) or after max_iter steps (MAXITER).  x: in x_0, out
   the returned iterate.  info (HOST, batch, nullable): iters, res_norm (the
   mapping's norm at the returned point), status. */
int maid1d_lower_solve(maid1d_ctx* ctx, const double* B, const double* y, double* x, double step,
                       const double* tol, int32_t max_iter, maid_solve_info* info, hipStream_t stream);

/* g = 1/2 ||A x - y||^2 and grad_out = A^T (A x - y) (nullable) for every
   instance; g_out, gradnorm_out HOST (batch, nullable). */
int maid1d_upper_value_grad(maid1d_ctx* ctx, const double* A, const double* y, const double* x, double* grad_out,
                            double* g_out, double* gradnorm_out, hipStream_t stream);

/* Algorithm 1's Hessian system on the support S = {i : x_i != 0} of x:
   conjugate gradients on (B^T B + 2 alpha2 I)_SS q_S = rhs_S, q = 0 off S,
   stopped at ||r|| <= tol[i] (recursive residual).  q: in the start (its
   entries off S are ignored), out the solution. */
int maid1d_adjoint_solve(maid1d_ctx* ctx, const double* B, const double* x, const double* rhs, double* q,
                         const double* tol, int32_t max_iter, maid_solve_info* info, hipStream_t stream);

/* Eq. (3.2) for the matrix B: z = -(d grad_x h / dB)^T q
   = -((B x - y) q^T + (B q) x^T) (n x n per instance), q supported on the
   support of x.  znorm_out HOST (batch, nullable) = ||z||_F. */
int maid1d_hypergrad(maid1d_ctx* ctx, const double* B, const double* y, const double* x, const double* q, double* z,
                     double* znorm_out, hipStream_t stream);

/* MAID's per-instance schedule for maid1d_step: accuracies eps (lower
   level) and delta (CG), step size, outer counter (updated in place). */
typedef struct {
    double eps, delta, step;
    int32_t k;
} maid1d_sched;

/* One outer iteration of Algorithm 2 for every instance (lockstep: the
   instances that need a solve at the same point of the algorithm share its
   launches; each takes its own decisions), on B: the retry loop over
   accuracies; InexactGradient (the lower level to eps * mu by
   maid1d_lower_solve with the step lam_x, the adjoint to delta, z); up to j
   trial steps B' = B - step z, each tested with Eq. (3.4)'s psi
   (L_g = hp->L_g if > 0, else ||A||_1 ||A||_inf, an upper bound of
   ||A||_2^2; l = g as beta = 0); the schedule of Algorithm 2.  B
   ([batch][n][n]), x and q ([batch][n], the warm starts) are updated in
   place, as is sched (HOST, batch).  hp as for maid_step.  infos (HOST,
   batch, nullable) as for maid_step.  Returns MAID_OK, MAID_MAXITER (a
   solve stopped at its cap), MAID_ACCURACY_FLOOR (eps fell below
   hp->eps_min without an accepted step: that instance's B unchanged), or
   an error (the first instance's code that is not MAID_OK). */
int maid1d_step(maid1d_ctx* ctx, const double* A, const double* y, double* B, double* x, double* q,
                maid1d_sched* sched, const maid_hparams* hp, double lam_x, maid_step_info* infos,
                hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif
