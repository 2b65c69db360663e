// d1.h -- the 1D problem's kernels (d1.hip) as seen from its host code:
// per-instance solver states and the launchers.
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>

namespace maid {
namespace d1 {

constexpr int kMaxN = 4096;   // the row and column products stage one vector of n doubles in LDS

// proximal-gradient solve, one per instance
struct ProxState {
    double tol, lam, res;
    int32_t iters, max, done, status, cur;
};
// conjugate gradients on the support, one per instance
struct CgState1 {
    double gamma, beta, alpha, tol, res;
    int32_t iters, max, done, status, first;
};

// the column product's epilogue
enum { kGrad = 0, kProx = 1, kHvp = 2 };
struct Epi {
    int mode;
    double alpha1, alpha2, lam;
    double* xa;            // kProx: the two iterate buffers (cur picks the current one)
    double* xb;
    const int* cur;
    const double* p;       // kHvp: the vector the Hessian is applied to
    const double* xsup;    // kHvp: the point whose support masks it
};

int row_blocks(int n);
int col_blocks(int n);
int ew_blocks(int n);

hipError_t gemv(const double* M, int64_t mstride, const double* v0, const double* v1, const int* vsel, int n, int nb,
                const double* sub, double* out, double* part, const int* done, hipStream_t s);
hipError_t gemvt(const double* M, int64_t mstride, const double* u, int n, int nb, const Epi& e, double* out,
                 double* part, const int* done, hipStream_t s);
hipError_t prox_decide(ProxState* st, const double* part, int nblk, int nb, int* done, int* cur, hipStream_t s);
hipError_t cg_gamma(CgState1* st, const double* part, int nblk, int nb, int* done, hipStream_t s);
hipError_t cg_alpha(CgState1* st, const double* part, int nblk, int nb, int* done, hipStream_t s);
hipError_t cg_setup(const double* x, const double* rhs, const double* hq, double* q, double* r, double* p, int n, int nb,
                    double* part, const int* done, hipStream_t s);
hipError_t cg_dir(const CgState1* st, const double* r, double* p, int n, int nb, hipStream_t s);
hipError_t cg_update(const CgState1* st, const double* p, const double* hp, double* q, double* r, int n, int nb,
                     double* part, hipStream_t s);
hipError_t outer(const double* r, const double* q, const double* u, const double* x, int n, int nb, double* z,
                 double* part, const int* skip, hipStream_t s);
hipError_t mat_step(const double* M, const double* z, const double* step, int n, int nb, double* out, const int* skip,
                    hipStream_t s);
hipError_t pick(const double* x0, const double* x1, const int* cur, int n, int nb, double* out, const int* skip,
                hipStream_t s);

}  // namespace d1
}  // namespace maid
