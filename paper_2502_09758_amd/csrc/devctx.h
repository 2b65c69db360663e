// devctx.h -- device-resident state shared by the host control code and the
// kernels of libmaid.  One DevCtx lives in device memory per context; the
// host writes it before a solve and reads it back when polling.  Kernels
// read it through scalar loads; only the last block of a reduction pass
// writes it (with ordinary vector stores), and the next kernel launch orders
// those writes before any further read.
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>

namespace maid {

constexpr int kMaxC = 3;       // colour channels supported by the LDS tiles
constexpr int kMaxK = 31;      // largest odd kernel size
constexpr int kTW = 64;        // tile width: one wave64 spans a tile row
constexpr int kNT = 256;       // threads per block (4 waves)

enum Status : int32_t { ST_OK = 0, ST_MAXITER = 1, ST_NOT_SPD = -4, ST_NONFINITE = -5 };

// Lower-level (FISTA) solver state.  Two copies live in DevCtx: the
// gradient pass reads apg[0] and its block 0 writes apg[1]; the trial pass
// reads apg[1] and writes apg[0].  No kernel writes the copy it reads, so
// every block of a launch sees the same state.
enum ApgPhase : int32_t { PH_START = 0, PH_GRAD_READY = 1, PH_RETRY = 2, PH_TRIALED = 3 };

struct ApgState {
    double L, t, t_prev, m;      // Lipschitz estimate, momentum sequence, m = (t_prev-1)/t
    double gn2;                  // ||G||^2 at the current extrapolated point
    double tol;                  // stop when ||G|| <= tol
    double delta_last;           // last h(x+) - h(v)
    int32_t max_iter, iters, bt, nb_iter;
    int32_t status, done, phase;
    int32_t cur, prev, nxt;      // rotation of the three x / Kx buffers
    int32_t trace_cap, pad;
};

// CG state: three copies; the direction pass reads cg[0] and writes cg[1],
// the Hessian pass cg[1] -> cg[2], the update pass cg[2] -> cg[0].
struct CgState {
    double gamma, kappa, a, tol;
    int32_t max, iters, status, done, pc, first;
};

// Problem parameters the kernels need, passed by value (kernel arguments
// live in the constant kernarg segment and are read with scalar loads).
struct Params {
    int32_t C, H, W, reg;
    double alpha, eps_tv;
};

struct DevCtx {
    // ---------------- problem (fixed per context)
    int32_t C, H, W, K, reg;
    int32_t pad0;
    double alpha, eps_tv, beta, h1_w0;
    ApgState apg[2];
    CgState cg[3];
    // ---------------- generic reduction results
    double red[8];
};

__host__ __device__ constexpr int tile_h(int R) { return 4 * R; }

// ------------------------------------------------------------------ LDS sizes
// TV halo tile: rows ti0-1 .. ti0+TH, columns tj0-1 .. tj0+64
__host__ __device__ constexpr int tv_pitch() { return kTW + 2; }
__host__ __device__ constexpr int tv_rows(int R) { return tile_h(R) + 2; }
// flux positions: rows ti0-1 .. ti0+TH-1, columns tj0-1 .. tj0+63
__host__ __device__ constexpr int fx_pitch() { return kTW + 1; }
__host__ __device__ constexpr int fx_rows(int R) { return tile_h(R) + 1; }
// convolution tile with a c0 halo on every side
__host__ __device__ constexpr int cv_pitch(int K) { return kTW + K - 1; }
__host__ __device__ constexpr int cv_rows(int K, int R) { return tile_h(R) + K - 1; }
__host__ __device__ constexpr int cmax(int a, int b) { return a > b ? a : b; }

__host__ __device__ constexpr int lds_conv(int K, int R) { return cv_rows(K, R) * cv_pitch(K); }
__host__ __device__ constexpr int lds_apg_grad(int K, int R, int C, int nw) {
    return cmax(C * tv_rows(R) * tv_pitch() + nw * fx_rows(R) * fx_pitch(), lds_conv(K, R));
}
__host__ __device__ constexpr int lds_apg_trial(int K, int R, int C) {
    return 2 * C * tv_rows(R) * tv_pitch() + lds_conv(K, R);
}
__host__ __device__ constexpr int lds_cg_hvp(int K, int R, int C, int nw) {
    return cmax(2 * C * tv_rows(R) * tv_pitch() + 2 * nw * fx_rows(R) * fx_pitch(), lds_conv(K, R));
}

// ------------------------------------------------------------------ buffers
template <typename T> struct ApgBufs {
    T* X[3];           // iterates x_k (rotating: cur, prev, next)
    T* KX[3];          // theta * x_k, kept by linearity
    T* G;              // gradient at the extrapolated point
    const T* y;
    const T* th;       // theta, correlation (adjoint) form, column-major
    const T* thf;      // theta flipped (convolution form), column-major
    double* pA;        // per-block partials of ||G||^2 (gradient pass)
    double* pB;        // per-block partials of h(x+) - h(v) (trial pass)
    int nbA, nbB;      // grid sizes of the two passes
    int* trace;        // rejected trials per iteration
};

template <typename T> struct CgBufs {
    T* q;
    T* r;
    T* P[2];           // search direction (ping-pong)
    T* Kp;             // theta * p
    T* Hp;
    const T* xt;       // lower-level point the Hessian is taken at
    const T* b;        // right-hand side
    const T* th;
    const T* thf;
    double* pR;        // per-block partials of ||r||^2 (update / init pass)
    double* pK;        // per-block partials of <p, Hp> (Hessian pass)
    int nbR, nbK;
};

}  // namespace maid
