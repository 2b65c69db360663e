// d1.hip -- kernels of the 1D problem of Section 4.1 (dense n x n operators,
// a batch of instances of one size): matrix-vector products by rows and by
// columns with the solvers' elementwise work fused into their epilogues, the
// per-instance solver decisions, and the hypergradient's outer products.
// All FP64.  Every reduction runs in a fixed order (partials per block,
// summed in block order by one block per instance), so results are bitwise
// reproducible and an instance computes the same alone or in a batch.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "d1.h"

namespace maid {
namespace d1 {

constexpr int kT = 256;            // threads per block (4 waves)
constexpr int kRowsPerBlock = 16;  // rows of a row-product block (4 per wave)
constexpr int kColsPerBlock = 64;  // columns of a column-product block (one per lane)

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// sum of one value per thread of a 256-thread block, in a fixed order
__device__ __forceinline__ double block_sum256(double v, double* s4) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) s4[w] = v;
    __syncthreads();
    return ((s4[0] + s4[1]) + s4[2]) + s4[3];
}

__device__ __forceinline__ double soft(double v, double t) {
    const double a = fabs(v) - t;
    return a > 0.0 ? copysign(a, v) : 0.0;
}

// ------------------------------------------------------------------ row products
// out[b][i] = sum_j M[b][i][j] v[b][j] - sub[b][i] (sub nullable); with part,
// per-block partials of sum out^2.  v: the instance's vector, or X[state.cur]
// when vsel (the prox-gradient iterate); instances whose state is done skip.
__global__ __launch_bounds__(kT) void k_gemv(const double* __restrict__ M, int64_t mstride, const double* __restrict__ v0,
                                             const double* __restrict__ v1, const int* __restrict__ vsel, int n,
                                             const double* __restrict__ sub, double* __restrict__ out,
                                             double* __restrict__ part, const int* __restrict__ done) {
    extern __shared__ double s_v[];
    __shared__ double s4[4];
    const int b = blockIdx.y;
    if (done && done[b]) return;
    const double* v = ((vsel && vsel[b]) ? v1 : v0) + (int64_t)b * n;
    for (int j = threadIdx.x; j < n; j += kT) s_v[j] = v[j];
    __syncthreads();
    const double* Mb = M + (int64_t)b * mstride;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    double sq = 0.0;
#pragma unroll
    for (int k = 0; k < kRowsPerBlock / 4; ++k) {
        const int i = blockIdx.x * kRowsPerBlock + w * (kRowsPerBlock / 4) + k;
        if (i >= n) break;
        const double* row = Mb + (int64_t)i * n;
        double acc = 0.0;
        for (int j = l; j < n; j += 64) acc = fma(row[j], s_v[j], acc);
        acc = wave_sum(acc);
        const double o = sub ? acc - sub[(int64_t)b * n + i] : acc;
        if (l == 0) out[(int64_t)b * n + i] = o;
        sq = fma(o, o, sq);
    }
    if (part) {
        // one value per wave (lane 0 holds the wave's rows' sum)
        const double t = block_sum256(l == 0 ? sq : 0.0, s4);
        if (threadIdx.x == 0) part[(int64_t)b * gridDim.x + blockIdx.x] = t;
    }
}

// ------------------------------------------------------------------ column products
// acc_j = sum_i M[b][i][j] u[b][i], then the epilogue of `mode`:
//   kGrad:  out = acc;                             partial of out^2
//   kProx:  G = acc + 2 alpha2 x, x+ = S_{lam alpha1}(x - lam G) into the
//           other iterate buffer;                  partial of (x - x+)^2
//   kHvp:   out = acc + 2 alpha2 p on the support of x, 0 off it;
//                                                  partial of p * out

__global__ __launch_bounds__(kT) void k_gemvt(const double* __restrict__ M, int64_t mstride, const double* __restrict__ u,
                                              int n, Epi e, double* __restrict__ out, double* __restrict__ part,
                                              const int* __restrict__ done) {
    extern __shared__ double s_u[];
    __shared__ double s_acc[4][kColsPerBlock];
    __shared__ double s4[4];
    const int b = blockIdx.y;
    if (done && done[b]) return;
    const double* ub = u + (int64_t)b * n;
    for (int i = threadIdx.x; i < n; i += kT) s_u[i] = ub[i];
    __syncthreads();
    const double* Mb = M + (int64_t)b * mstride;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int j = blockIdx.x * kColsPerBlock + l;
    double acc = 0.0;
    if (j < n)
        for (int i = w; i < n; i += 4) acc = fma(Mb[(int64_t)i * n + j], s_u[i], acc);
    s_acc[w][l] = acc;
    __syncthreads();
    double pv = 0.0;
    if (w == 0 && j < n) {
        const double a = ((s_acc[0][l] + s_acc[1][l]) + s_acc[2][l]) + s_acc[3][l];
        const int64_t o = (int64_t)b * n + j;
        if (e.mode == kGrad) {
            out[o] = a;
            pv = a * a;
        } else if (e.mode == kProx) {
            const bool c1 = e.cur[b] != 0;
            const double xj = (c1 ? e.xb : e.xa)[o];
            const double g = fma(2.0 * e.alpha2, xj, a);
            const double xp = soft(fma(-e.lam, g, xj), e.lam * e.alpha1);
            (c1 ? e.xa : e.xb)[o] = xp;
            const double d = xj - xp;
            pv = d * d;
        } else {
            const double pj = e.p[o];
            const double hv = e.xsup[o] != 0.0 ? fma(2.0 * e.alpha2, pj, a) : 0.0;
            out[o] = hv;
            pv = pj * hv;
        }
    }
    const double t = block_sum256(pv, s4);
    if (part && threadIdx.x == 0) part[(int64_t)b * gridDim.x + blockIdx.x] = t;
}

// ------------------------------------------------------------------ per-instance decisions
// Proximal gradient: the mapping's norm from the partials, then stop (the
// iterate stays), or move to x+ (cur flips) and count the step.
__global__ void k_prox_decide(ProxState* __restrict__ st, const double* __restrict__ part, int nblk, int* __restrict__ done,
                              int* __restrict__ cur) {
    const int b = blockIdx.x;
    if (threadIdx.x != 0) return;
    ProxState s = st[b];
    if (s.done) return;
    double sum = 0.0;
    for (int k = 0; k < nblk; ++k) sum += part[(int64_t)b * nblk + k];
    const double res = sqrt(sum) / s.lam;
    s.res = res;
    if (!(res == res) || res > 1e300) {
        s.done = 1;
        s.status = -5;
    } else if (res <= s.tol) {
        s.done = 1;
        s.status = 0;
    } else if (s.iters >= s.max) {
        s.done = 1;
        s.status = 1;
    } else {
        s.cur ^= 1;
        s.iters += 1;
    }
    st[b] = s;
    done[b] = s.done;
    cur[b] = s.cur;
}

// CG: gamma from the partials of ||r||^2, the stop tests, beta.
__global__ void k_cg_gamma(CgState1* __restrict__ st, const double* __restrict__ part, int nblk, int* __restrict__ done) {
    const int b = blockIdx.x;
    if (threadIdx.x != 0) return;
    CgState1 s = st[b];
    if (s.done) return;
    double g = 0.0;
    for (int k = 0; k < nblk; ++k) g += part[(int64_t)b * nblk + k];
    s.beta = s.first ? 0.0 : g / s.gamma;
    s.gamma = g;
    s.res = sqrt(g);
    if (!(g == g) || g > 1e300) {
        s.done = 1;
        s.status = -5;
    } else if (sqrt(g) <= s.tol) {
        s.done = 1;
        s.status = 0;
    } else if (s.iters >= s.max) {
        s.done = 1;
        s.status = 1;
    }
    st[b] = s;
    done[b] = s.done;
}

// CG: the step a = gamma / <p, Hp> (curvature tested), one iteration counted.
__global__ void k_cg_alpha(CgState1* __restrict__ st, const double* __restrict__ part, int nblk, int* __restrict__ done) {
    const int b = blockIdx.x;
    if (threadIdx.x != 0) return;
    CgState1 s = st[b];
    if (s.done) return;
    double d = 0.0;
    for (int k = 0; k < nblk; ++k) d += part[(int64_t)b * nblk + k];
    if (!(d > 0.0) || d > 1e300) {
        s.done = 1;
        s.status = (d == d && d <= 1e300) ? -4 : -5;
    } else {
        s.alpha = s.gamma / d;
        s.iters += 1;
        s.first = 0;
    }
    st[b] = s;
    done[b] = s.done;
}

// ------------------------------------------------------------------ elementwise CG passes
// set-up: q = q0 on the support (0 off it), r = rhs - Hq0 on the support, p = r,
// partials of ||r||^2.  Hq (the set-up product) arrives in hq.
__global__ __launch_bounds__(kT) void k_cg_setup(const double* __restrict__ x, const double* __restrict__ rhs,
                                                 const double* __restrict__ hq, double* __restrict__ q,
                                                 double* __restrict__ r, double* __restrict__ p, int n,
                                                 double* __restrict__ part, const int* __restrict__ done) {
    __shared__ double s4[4];
    const int b = blockIdx.y;
    if (done && done[b]) return;
    double pv = 0.0;
    const int j = blockIdx.x * kT + threadIdx.x;
    if (j < n) {
        const int64_t o = (int64_t)b * n + j;
        const bool in = x[o] != 0.0;
        const double rv = in ? rhs[o] - hq[o] : 0.0;
        q[o] = in ? q[o] : 0.0;
        r[o] = rv;
        p[o] = rv;
        pv = rv * rv;
    }
    const double t = block_sum256(pv, s4);
    if (threadIdx.x == 0) part[(int64_t)b * gridDim.x + blockIdx.x] = t;
}

// p = r + beta p (beta = 0 on the first iteration: p = r already)
__global__ __launch_bounds__(kT) void k_cg_dir(const CgState1* __restrict__ st, const double* __restrict__ r,
                                               double* __restrict__ p, int n) {
    const int b = blockIdx.y;
    const CgState1 s = st[b];
    if (s.done || s.first) return;
    const int j = blockIdx.x * kT + threadIdx.x;
    if (j < n) {
        const int64_t o = (int64_t)b * n + j;
        p[o] = fma(s.beta, p[o], r[o]);
    }
}

// q += a p, r -= a Hp, partials of ||r||^2
__global__ __launch_bounds__(kT) void k_cg_update(const CgState1* __restrict__ st, const double* __restrict__ p,
                                                  const double* __restrict__ hp, double* __restrict__ q,
                                                  double* __restrict__ r, int n, double* __restrict__ part) {
    __shared__ double s4[4];
    const int b = blockIdx.y;
    const CgState1 s = st[b];
    if (s.done) return;
    double pv = 0.0;
    const int j = blockIdx.x * kT + threadIdx.x;
    if (j < n) {
        const int64_t o = (int64_t)b * n + j;
        q[o] = fma(s.alpha, p[o], q[o]);
        const double rv = fma(-s.alpha, hp[o], r[o]);
        r[o] = rv;
        pv = rv * rv;
    }
    const double t = block_sum256(pv, s4);
    if (threadIdx.x == 0) part[(int64_t)b * gridDim.x + blockIdx.x] = t;
}

// ------------------------------------------------------------------ hypergradient and steps
// z[b][i][j] = -(r_i q_j + u_i x_j); per-block partials of ||z||^2.
// Blocks of 256 threads over one row chunk of 256 columns each.
__global__ __launch_bounds__(kT) void k_outer(const double* __restrict__ r, const double* __restrict__ q,
                                              const double* __restrict__ u, const double* __restrict__ x, int n,
                                              double* __restrict__ z, double* __restrict__ part,
                                              const int* __restrict__ skip) {
    __shared__ double s4[4];
    const int b = blockIdx.z;
    if (skip && skip[b]) return;
    const int i = blockIdx.y;
    const int j = blockIdx.x * kT + threadIdx.x;
    double pv = 0.0;
    if (j < n) {
        const int64_t v = (int64_t)b * n;
        const double zv = -fma(r[v + i], q[v + j], u[v + i] * x[v + j]);
        z[((int64_t)b * n + i) * n + j] = zv;
        pv = zv * zv;
    }
    const double t = block_sum256(pv, s4);
    if (threadIdx.x == 0) part[((int64_t)b * gridDim.y + i) * gridDim.x + blockIdx.x] = t;
}

// out = M - s_b z (s per instance, n x n each); instances with skip set are left out
__global__ __launch_bounds__(kT) void k_mat_step(const double* __restrict__ M, const double* __restrict__ z,
                                                 const double* __restrict__ s, int64_t nn, double* __restrict__ out,
                                                 const int* __restrict__ skip) {
    const int b = blockIdx.y;
    if (skip && skip[b]) return;
    const double sb = s[b];
    const int64_t base = (int64_t)b * nn;
    for (int64_t k = (int64_t)blockIdx.x * kT + threadIdx.x; k < nn; k += (int64_t)gridDim.x * kT)
        out[base + k] = fma(-sb, z[base + k], M[base + k]);
}

// out[b] = X[cur[b]][b]
__global__ __launch_bounds__(kT) void k_pick(const double* __restrict__ x0, const double* __restrict__ x1,
                                             const int* __restrict__ cur, int n, double* __restrict__ out,
                                             const int* __restrict__ skip) {
    const int b = blockIdx.y;
    if (skip && skip[b]) return;
    const int j = blockIdx.x * kT + threadIdx.x;
    if (j < n) {
        const int64_t o = (int64_t)b * n + j;
        out[o] = (cur[b] ? x1 : x0)[o];
    }
}

// ------------------------------------------------------------------ launchers
namespace {
template <typename F, typename... A>
hipError_t go(F k, dim3 g, dim3 t, size_t lds, hipStream_t s, A... a) {
    hipLaunchKernelGGL(k, g, t, lds, s, a...);
    return hipGetLastError();
}
}  // namespace

int row_blocks(int n) { return (n + kRowsPerBlock - 1) / kRowsPerBlock; }
int col_blocks(int n) { return (n + kColsPerBlock - 1) / kColsPerBlock; }
int ew_blocks(int n) { return (n + kT - 1) / kT; }

hipError_t gemv(const double* M, int64_t mstride, const double* v0, const double* v1, const int* vsel, int n, int nb,
                const double* sub, double* out, double* part, const int* done, hipStream_t s) {
    return go(k_gemv, dim3(row_blocks(n), nb), dim3(kT), (size_t)n * sizeof(double), s, M, mstride, v0, v1, vsel, n,
              sub, out, part, done);
}

hipError_t gemvt(const double* M, int64_t mstride, const double* u, int n, int nb, const Epi& e, double* out,
                 double* part, const int* done, hipStream_t s) {
    return go(k_gemvt, dim3(col_blocks(n), nb), dim3(kT), (size_t)n * sizeof(double), s, M, mstride, u, n, e, out,
              part, done);
}

hipError_t prox_decide(ProxState* st, const double* part, int nblk, int nb, int* done, int* cur, hipStream_t s) {
    return go(k_prox_decide, dim3(nb), dim3(64), 0, s, st, part, nblk, done, cur);
}

hipError_t cg_gamma(CgState1* st, const double* part, int nblk, int nb, int* done, hipStream_t s) {
    return go(k_cg_gamma, dim3(nb), dim3(64), 0, s, st, part, nblk, done);
}

hipError_t cg_alpha(CgState1* st, const double* part, int nblk, int nb, int* done, hipStream_t s) {
    return go(k_cg_alpha, dim3(nb), dim3(64), 0, s, st, part, nblk, done);
}

hipError_t cg_setup(const double* x, const double* rhs, const double* hq, double* q, double* r, double* p, int n, int nb,
                    double* part, const int* done, hipStream_t s) {
    return go(k_cg_setup, dim3(ew_blocks(n), nb), dim3(kT), 0, s, x, rhs, hq, q, r, p, n, part, done);
}

hipError_t cg_dir(const CgState1* st, const double* r, double* p, int n, int nb, hipStream_t s) {
    return go(k_cg_dir, dim3(ew_blocks(n), nb), dim3(kT), 0, s, st, r, p, n);
}

hipError_t cg_update(const CgState1* st, const double* p, const double* hp, double* q, double* r, int n, int nb,
                     double* part, hipStream_t s) {
    return go(k_cg_update, dim3(ew_blocks(n), nb), dim3(kT), 0, s, st, p, hp, q, r, n, part);
}

hipError_t outer(const double* r, const double* q, const double* u, const double* x, int n, int nb, double* z,
                 double* part, const int* skip, hipStream_t s) {
    return go(k_outer, dim3(ew_blocks(n), n, nb), dim3(kT), 0, s, r, q, u, x, n, z, part, skip);
}

hipError_t mat_step(const double* M, const double* z, const double* step, int n, int nb, double* out, const int* skip,
                    hipStream_t s) {
    const int64_t nn = (int64_t)n * n;
    const int blocks = (int)std::min<int64_t>((nn + kT - 1) / kT, 1024);
    return go(k_mat_step, dim3(blocks, nb), dim3(kT), 0, s, M, z, step, nn, out, skip);
}

hipError_t pick(const double* x0, const double* x1, const int* cur, int n, int nb, double* out, const int* skip,
                hipStream_t s) {
    return go(k_pick, dim3(ew_blocks(n), nb), dim3(kT), 0, s, x0, x1, cur, n, out, skip);
}

}  // namespace d1
}  // namespace maid
