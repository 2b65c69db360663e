// kernels.cuh -- gfx950 kernels of libmaid (templated on storage type T,
// kernel size K and rows per thread R).
//
// Layout: images are planar [C][H][W]; a block of 256 threads (four wave64s)
// owns a 64-wide, 4R-tall tile of output pixels for all channels.  Lane tx of
// wave wy computes the R pixels in rows wy*R .. wy*R+R-1 of column tx.
// Inputs with the halo a stencil needs are staged through LDS with zero fill
// outside the image; convolution taps are read through uniform (scalar)
// loads, so every FMA takes its tap from an SGPR and its pixel from a VGPR
// column that is reused across the R outputs.  Blocks map to tiles in
// XCD-major order so that horizontally adjacent tiles (shared halos) run on
// the same XCD and share its L2.
//
// Reductions are accumulated in double: per thread, then wave64 butterfly,
// then the four waves in a fixed order, giving one partial per block.  The
// kernel that needs the total sums the partials itself, every block in the
// same order, so all blocks hold the bitwise-same value and take the same
// solver decision (stop tests, backtracking, CG coefficients) without a
// host round trip and without atomics or fences: the kernel boundary orders
// the partials before they are read.
//
// Every pass serves a batch: block b belongs to instance blk[b] of the
// instance table (a plain solve is a batch of one); the instance's blocks
// start at a multiple of 8 so that the XCD-major tile order holds within
// each instance.  Solver states are arrays over instances, read through one
// copy and written by the instance's block 0 into the next.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "devctx.h"

namespace maid {

// ------------------------------------------------------------------ helpers
template <typename T> __device__ __forceinline__ T dfma(T a, T b, T c);
template <> __device__ __forceinline__ float dfma<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <> __device__ __forceinline__ double dfma<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T> __device__ __forceinline__ T dsqrt(T v);
template <> __device__ __forceinline__ float dsqrt<float>(float v) { return sqrtf(v); }
template <> __device__ __forceinline__ double dsqrt<double>(double v) { return sqrt(v); }

// blockIdx -> tile id, XCD-major: the hardware hands block b to XCD b % 8;
// this bijection gives every XCD a contiguous run of tile ids.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int q = nb >> 3, r = nb & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum of one double per thread over the block, returned to every thread
// (wave butterflies, then the four waves in a fixed order).
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double s_w[4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) s_w[wid] = v;
    __syncthreads();
    return ((s_w[0] + s_w[1]) + s_w[2]) + s_w[3];
}

// Producer side of a grid-wide sum: one partial per block (index lb within
// its instance), plain store.
__device__ __forceinline__ void block_partial(double v, double* part, int lb) {
    const double s = block_sum(v);
    if (threadIdx.x == 0) part[lb] = s;
}

// Consumer side, at the start of the next kernel: every block sums the nb
// partials in the same fixed order and so obtains the bitwise-same total and
// takes the same decision; kernel boundaries order the producer's stores
// before these loads.  No atomics or fences are involved.
__device__ __forceinline__ double reduce_partials(const double* __restrict__ part, int nb) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += kNT) s += part[b];
    return block_sum(s);
}

__device__ __forceinline__ bool finite_d(double v) { return v == v && v <= 1.0e300 && v >= -1.0e300; }

// Field-by-field state stores (no whole-struct copy, so the local state stays
// in scalar registers) and select-based buffer picks (no runtime indexing
// into by-value argument arrays, which would go through scratch memory).
__device__ __forceinline__ void put_state(ApgState* __restrict__ o, const ApgState& s) {
    o->L = s.L; o->t = s.t; o->t_prev = s.t_prev; o->m = s.m; o->gn2 = s.gn2; o->tol = s.tol;
    o->delta_last = s.delta_last; o->max_iter = s.max_iter; o->iters = s.iters; o->bt = s.bt;
    o->nb_iter = s.nb_iter; o->status = s.status; o->done = s.done; o->phase = s.phase; o->cur = s.cur;
    o->prev = s.prev; o->nxt = s.nxt; o->trace_cap = s.trace_cap; o->pad = 0;
}
__device__ __forceinline__ void put_state(CgState* __restrict__ o, const CgState& s) {
    o->gamma = s.gamma; o->kappa = s.kappa; o->a = s.a; o->tol = s.tol; o->max = s.max; o->iters = s.iters;
    o->status = s.status; o->done = s.done; o->pc = s.pc; o->first = s.first;
}
template <typename P>
__device__ __forceinline__ P pick(P a0, P a1, P a2, int i) { return i == 0 ? a0 : (i == 1 ? a1 : a2); }
template <typename P>
__device__ __forceinline__ P pick(P a0, P a1, int i) { return i == 0 ? a0 : a1; }

// Stage f(global flat index) into an LDS tile s[ROWS][PITCH] covering rows
// gi0.., columns gj0..; zero outside [0,H) x [0,W).
template <int ROWS, int COLS, int PITCH, typename T, typename F>
__device__ __forceinline__ void load_tile(T* s, int gi0, int gj0, int H, int W, F f) {
    for (int idx = threadIdx.x; idx < ROWS * COLS; idx += kNT) {
        const int r = idx / COLS, cc = idx - r * COLS;
        const int gi = gi0 + r, gj = gj0 + cc;
        T val = T(0);
        if (gi >= 0 && gi < H && gj >= 0 && gj < W) val = f((int64_t)gi * W + gj);
        s[r * PITCH + cc] = val;
    }
}

// acc[o] += sum_{u,v} ker(u,v) * s[li0+o+u][tx+v]  (a KxK correlation of
// the staged tile; with the flipped kernel it is the true convolution).
// Taps are stored column-major, kT[v*K + u] = ker(u,v), so the K taps of one
// column arrive in a few wide scalar loads.  The column loop stays rolled
// for large K to bound register pressure (R+K-1 staged values, R
// accumulators, K taps in SGPRs per iteration).
template <typename T, int K, int R>
__device__ __forceinline__ void correlate_col(const T* s, int pitch, const T* __restrict__ kT, int li0, int tx, int v, T (&acc)[R]) {
    T col[R + K - 1];
#pragma unroll
    for (int t = 0; t < R + K - 1; ++t) col[t] = s[(li0 + t) * pitch + tx + v];
#pragma unroll
    for (int u = 0; u < K; ++u) {
        const T w = kT[v * K + u];
#pragma unroll
        for (int o = 0; o < R; ++o) acc[o] = dfma(w, col[o + u], acc[o]);
    }
}

template <typename T, int K, int R>
__device__ __forceinline__ void correlate(const T* s, int pitch, const T* __restrict__ kT, int li0, int tx, T (&acc)[R]) {
    if constexpr (K <= 5) {
#pragma unroll
        for (int v = 0; v < K; ++v) correlate_col<T, K, R>(s, pitch, kT, li0, tx, v, acc);
    } else {
#pragma unroll 1
        for (int v = 0; v < K; ++v) correlate_col<T, K, R>(s, pitch, kT, li0, tx, v, acc);
    }
}

// select one of three register arrays by a (uniform) runtime channel index
template <typename T, int R>
__device__ __forceinline__ T pick3(const T (&a)[R], const T (&b)[R], const T (&c)[R], int ch, int o) {
    return ch == 0 ? a[o] : (ch == 1 ? b[o] : c[o]);
}

// ------------------------------------------------------------------ TV pieces
// Weight w = (s^2+eps^2)^(-1/2) at extended positions of the flux grid,
// from a staged halo tile of v (C planes).  reg 0: one s over all channels;
// reg 1: one per channel (nw = C planes); reg 2 (quadratic): w = 1.  Zero
// at positions outside the image, so every flux there vanishes.
template <typename T, int R>
__device__ __forceinline__ void tv_weights(const T* s_v, T* s_w, int C, int reg, T eps2, int ti0, int tj0, int H, int W) {
    constexpr int VP = tv_pitch(), VR = tv_rows(R), WP = fx_pitch(), WR = fx_rows(R);
    for (int idx = threadIdx.x; idx < WR * WP; idx += kNT) {
        const int r = idx / WP, cc = idx - r * WP;
        const int gi = ti0 - 1 + r, gj = tj0 - 1 + cc;
        const bool in = (gi >= 0 && gi < H && gj >= 0 && gj < W);
        const bool hx = gj < W - 1, vx = gi < H - 1;
        T s2 = T(0);
        for (int ch = 0; ch < C; ++ch) {
            const T* V = s_v + ch * VR * VP;
            const T v0 = V[r * VP + cc];
            const T dh = hx ? V[r * VP + cc + 1] - v0 : T(0);
            const T dv = vx ? V[(r + 1) * VP + cc] - v0 : T(0);
            if (reg == 1) {
                s_w[ch * WR * WP + idx] = in ? T(1) / dsqrt(dh * dh + dv * dv + eps2) : T(0);
            } else {
                s2 += dh * dh + dv * dv;
            }
        }
        if (reg != 1) s_w[idx] = in ? (reg == 2 ? T(1) : T(1) / dsqrt(s2 + eps2)) : T(0);
    }
}

// grad R at the thread's pixel (li, tx) of channel ch:
// fh(i,j-1) - fh(i,j) + fv(i-1,j) - fv(i,j), flux f = w * (forward difference)
template <typename T, int R>
__device__ __forceinline__ T tv_grad_px(const T* s_v, const T* s_w, int ch, int reg, int li, int tx, int gi, int gj, int H, int W) {
    constexpr int VP = tv_pitch(), VR = tv_rows(R), WP = fx_pitch(), WR = fx_rows(R);
    const T* V = s_v + ch * VR * VP;
    const T* Wt = s_w + (reg == 1 ? ch * WR * WP : 0);
    const int r = li + 1, cc = tx + 1;
    const T v0 = V[r * VP + cc];
    const T dh_here = (gj < W - 1) ? V[r * VP + cc + 1] - v0 : T(0);
    const T dv_here = (gi < H - 1) ? V[(r + 1) * VP + cc] - v0 : T(0);
    const T dh_left = v0 - V[r * VP + cc - 1];
    const T dv_up = v0 - V[(r - 1) * VP + cc];
    const T w0 = Wt[r * WP + cc];
    return Wt[r * WP + cc - 1] * dh_left - w0 * dh_here + Wt[(r - 1) * WP + cc] * dv_up - w0 * dv_here;
}

// ------------------------------------------------------------------ instance lookup
// Block -> (instance, local block).  Padding blocks (lb >= nb) return at once.
#define MAID_STENCIL_PROLOGUE                                         \
    const int ii = blk[blockIdx.x];                                   \
    const Inst<T>& I = insts[ii];                                     \
    const int lb = (int)blockIdx.x - I.base;                          \
    if (lb >= I.nb) return;

#define MAID_EW_PROLOGUE                                              \
    const int ii = blk[blockIdx.x];                                   \
    const Inst<T>& I = insts[ii];                                     \
    const int lb = (int)blockIdx.x - I.base_e;                        \
    if (lb >= I.nbe) return;

// ------------------------------------------------------------------ generic convolution pass
// cv_out = cv_ker (x) cv_in  [- cv_sub]   (correlation with cv_ker; the
// flipped kernel gives the true convolution); with cv_part, per-block
// partials of sum cv_out^2.  Instances without cv_out take no part.
template <typename T, int K, int R>
__global__ __launch_bounds__(kNT) void k_conv(const Inst<T>* __restrict__ insts, const int* __restrict__ blk) {
    MAID_STENCIL_PROLOGUE
    if (!I.cv_out) return;
    constexpr int TH = tile_h(R), c0 = (K - 1) / 2, CP = cv_pitch(K), CR = cv_rows(K, R);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* s = reinterpret_cast<T*>(smem_raw);
    const int C = I.pr.C, H = I.pr.H, W = I.pr.W;
    const int64_t HW = (int64_t)H * W;
    const int ntx = (W + kTW - 1) / kTW;
    const int tile = xcd_tile(lb, I.nb);
    const int ti0 = (tile / ntx) * TH, tj0 = (tile % ntx) * kTW;
    const int tx = threadIdx.x & 63, li0 = (threadIdx.x >> 6) * R;
    const T* __restrict__ in = I.cv_in;
    const T* __restrict__ sub = I.cv_sub;
    T* __restrict__ out = I.cv_out;
    double sq = 0.0;
    for (int ch = 0; ch < C; ++ch) {
        const T* src = in + ch * HW;
        __syncthreads();
        load_tile<CR, CP, CP>(s, ti0 - c0, tj0 - c0, H, W, [&](int64_t g) { return src[g]; });
        __syncthreads();
        T acc[R];
#pragma unroll
        for (int o = 0; o < R; ++o) acc[o] = T(0);
        correlate<T, K, R>(s, CP, I.cv_ker, li0, tx, acc);
        const int gj = tj0 + tx;
#pragma unroll
        for (int o = 0; o < R; ++o) {
            const int gi = ti0 + li0 + o;
            if (gi < H && gj < W) {
                const int64_t e = ch * HW + (int64_t)gi * W + gj;
                T val = acc[o];
                if (sub) val -= sub[e];
                out[e] = val;
                sq += (double)val * (double)val;
            }
        }
    }
    if (I.cv_part) block_partial(sq, I.cv_part, lb);
}

// ------------------------------------------------------------------ lower level: FISTA
// Gradient pass.  Per instance: reads sin, block 0 writes sout.  If the
// previous trial pass ran, first finish its decrease h(x+) - h(v) from the
// partials and take the backtracking decision: accept (rotate buffers,
// advance the momentum sequence, then evaluate the new gradient) or reject
// (double L, no gradient work).  The gradient at v = x + m (x - x_prev),
// with theta*v = Kx + m (Kx - Kx_prev) by linearity, is
//   G = theta . (theta*v - y) + alpha grad R(v),
// and its per-block partials of ||G||^2 go to pA.
template <typename T, int K, int R>
__global__ __launch_bounds__(kNT) void k_apg_grad(const Inst<T>* __restrict__ insts, const int* __restrict__ blk,
                                                  const ApgState* __restrict__ sin, ApgState* __restrict__ sout) {
    MAID_STENCIL_PROLOGUE
    ApgState st = sin[ii];
    const bool writer = lb == 0 && threadIdx.x == 0;
    if (st.done) {
        if (writer) put_state(&sout[ii], st);
        return;
    }
    bool compute = true;
    if (st.phase == PH_TRIALED) {
        const double delta = reduce_partials(I.pB, I.nb);
        st.delta_last = delta;
        if (!finite_d(delta)) {
            st.done = 1;
            st.status = ST_NONFINITE;
            compute = false;
        } else if (delta <= -st.gn2 / (2.0 * st.L)) {
            if (writer && I.trace && st.iters < st.trace_cap) I.trace[st.iters] = st.nb_iter;
            st.iters += 1;
            const int p = st.prev;
            st.prev = st.cur;
            st.cur = st.nxt;
            st.nxt = p;
            const double t = st.t;
            const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
            st.t_prev = t;
            st.t = tn;
            st.m = (t - 1.0) / tn;
            st.phase = PH_GRAD_READY;
        } else {
            st.L = 2.0 * st.L;
            st.bt += 1;
            st.nb_iter += 1;
            st.phase = PH_RETRY;
            compute = false;
            if (st.nb_iter > 200) {
                st.done = 1;
                st.status = ST_NONFINITE;
            }
        }
    } else {
        st.phase = PH_GRAD_READY;
    }
    if (writer) put_state(&sout[ii], st);
    if (!compute) return;

    constexpr int TH = tile_h(R), c0 = (K - 1) / 2, CP = cv_pitch(K), CR = cv_rows(K, R);
    constexpr int VP = tv_pitch(), VR = tv_rows(R);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* sm = reinterpret_cast<T*>(smem_raw);
    const int C = I.pr.C, H = I.pr.H, W = I.pr.W, reg = I.pr.reg;
    const int64_t HW = (int64_t)H * W;
    const int ntx = (W + kTW - 1) / kTW;
    const int tile = xcd_tile(lb, I.nb);
    const int ti0 = (tile / ntx) * TH, tj0 = (tile % ntx) * kTW;
    const int tx = threadIdx.x & 63, li0 = (threadIdx.x >> 6) * R;
    const int gj = tj0 + tx;
    const T m = (T)st.m;
    const T alpha = (T)I.pr.alpha;
    const T* __restrict__ X = pick(I.X[0], I.X[1], I.X[2], st.cur);
    const T* __restrict__ XP = pick(I.X[0], I.X[1], I.X[2], st.prev);
    const T* __restrict__ KX = pick(I.KX[0], I.KX[1], I.KX[2], st.cur);
    const T* __restrict__ KXP = pick(I.KX[0], I.KX[1], I.KX[2], st.prev);
    const T* __restrict__ Y = I.y;

    // ---- TV gradient at v (all channels staged: the magnitude couples them)
    T* s_v = sm;
    T* s_w = sm + C * VR * VP;
    __syncthreads();
    for (int ch = 0; ch < C; ++ch) {
        const T* Xc = X + ch * HW;
        const T* XPc = XP + ch * HW;
        load_tile<VR, VP, VP>(s_v + ch * VR * VP, ti0 - 1, tj0 - 1, H, W,
                              [&](int64_t g) { const T xv = Xc[g]; return dfma(m, xv - XPc[g], xv); });
    }
    __syncthreads();
    tv_weights<T, R>(s_v, s_w, C, reg, (T)(I.pr.eps_tv * I.pr.eps_tv), ti0, tj0, H, W);
    __syncthreads();
    T tg0[R], tg1[R], tg2[R];
#pragma unroll
    for (int o = 0; o < R; ++o) {
        const int li = li0 + o, gi = ti0 + li;
        tg0[o] = tv_grad_px<T, R>(s_v, s_w, 0, reg, li, tx, gi, gj, H, W);
        tg1[o] = C > 1 ? tv_grad_px<T, R>(s_v, s_w, 1, reg, li, tx, gi, gj, H, W) : T(0);
        tg2[o] = C > 2 ? tv_grad_px<T, R>(s_v, s_w, 2, reg, li, tx, gi, gj, H, W) : T(0);
    }

    // ---- data term: theta . r_v, channel by channel
    double gsq = 0.0;
    for (int ch = 0; ch < C; ++ch) {
        const T* KXc = KX + ch * HW;
        const T* KXPc = KXP + ch * HW;
        const T* Yc = Y + ch * HW;
        __syncthreads();
        load_tile<CR, CP, CP>(sm, ti0 - c0, tj0 - c0, H, W, [&](int64_t g) {
            const T kx = KXc[g];
            return dfma(m, kx - KXPc[g], kx) - Yc[g];
        });
        __syncthreads();
        T acc[R];
#pragma unroll
        for (int o = 0; o < R; ++o) acc[o] = T(0);
        correlate<T, K, R>(sm, CP, I.th, li0, tx, acc);
#pragma unroll
        for (int o = 0; o < R; ++o) {
            const int gi = ti0 + li0 + o;
            if (gi < H && gj < W) {
                const T gv = dfma(alpha, pick3<T, R>(tg0, tg1, tg2, ch, o), acc[o]);
                I.G[ch * HW + (int64_t)gi * W + gj] = gv;
                gsq += (double)gv * (double)gv;
            }
        }
    }
    block_partial(gsq, I.pA, lb);
}

// Trial pass.  Per instance: reads sin, block 0 writes sout.  After a fresh
// gradient it finishes ||G||^2 and applies the stop tests (||G|| <= tol:
// done, the point is v; iteration cap: done with MAXITER); otherwise (or on
// a retry) it takes the trial x+ = v + dl, dl = -G/L, writes x+ and
// theta*x+ = theta*v + theta*dl into the spare buffers, and forms per-block
// partials of the decrease h(x+) - h(v) through the increment (no
// cancellation of objective values):
//   data: sum d (r_v + d/2), d = theta*dl;
//   TV:   sum_sites (s'^2 - s^2) / (sqrt(s'^2+eps^2) + sqrt(s^2+eps^2)),
//         s'^2 - s^2 = sum a (a + 2 b), a = D dl, b = D v,
// with every per-element product in double.
template <typename T, int K, int R>
__global__ __launch_bounds__(kNT) void k_apg_trial(const Inst<T>* __restrict__ insts, const int* __restrict__ blk,
                                                   const ApgState* __restrict__ sin, ApgState* __restrict__ sout) {
    MAID_STENCIL_PROLOGUE
    ApgState st = sin[ii];
    const bool writer = lb == 0 && threadIdx.x == 0;
    if (st.done) {
        if (writer) put_state(&sout[ii], st);
        return;
    }
    bool trial = true;
    if (st.phase == PH_GRAD_READY) {
        const double gn2 = reduce_partials(I.pA, I.nb);
        st.gn2 = gn2;
        st.nb_iter = 0;
        if (!finite_d(gn2)) {
            st.done = 1;
            st.status = ST_NONFINITE;
            trial = false;
        } else if (sqrt(gn2) <= st.tol) {
            st.done = 1;
            st.status = ST_OK;
            trial = false;
        } else if (st.iters >= st.max_iter) {
            st.done = 1;
            st.status = ST_MAXITER;
            trial = false;
        }
    }
    if (trial) st.phase = PH_TRIALED;
    if (writer) put_state(&sout[ii], st);
    if (!trial) return;

    constexpr int TH = tile_h(R), c0 = (K - 1) / 2, CP = cv_pitch(K), CR = cv_rows(K, R);
    constexpr int VP = tv_pitch(), VR = tv_rows(R);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* sm = reinterpret_cast<T*>(smem_raw);
    const int C = I.pr.C, H = I.pr.H, W = I.pr.W, reg = I.pr.reg;
    const int64_t HW = (int64_t)H * W;
    const int ntx = (W + kTW - 1) / kTW;
    const int tile = xcd_tile(lb, I.nb);
    const int ti0 = (tile / ntx) * TH, tj0 = (tile % ntx) * kTW;
    const int tx = threadIdx.x & 63, li0 = (threadIdx.x >> 6) * R;
    const int gj = tj0 + tx;
    const T m = (T)st.m;
    const T ninvL = (T)(-1.0 / st.L);
    const T* __restrict__ X = pick(I.X[0], I.X[1], I.X[2], st.cur);
    const T* __restrict__ XP = pick(I.X[0], I.X[1], I.X[2], st.prev);
    const T* __restrict__ KX = pick(I.KX[0], I.KX[1], I.KX[2], st.cur);
    const T* __restrict__ KXP = pick(I.KX[0], I.KX[1], I.KX[2], st.prev);
    T* __restrict__ XN = pick(I.X[0], I.X[1], I.X[2], st.nxt);
    T* __restrict__ KXN = pick(I.KX[0], I.KX[1], I.KX[2], st.nxt);
    const T* __restrict__ G = I.G;
    const T* __restrict__ Y = I.y;

    T* s_v = sm;
    T* s_d = sm + C * VR * VP;
    T* s_c = sm + 2 * C * VR * VP;
    __syncthreads();
    for (int ch = 0; ch < C; ++ch) {
        const T* Xc = X + ch * HW;
        const T* XPc = XP + ch * HW;
        const T* Gc = G + ch * HW;
        load_tile<VR, VP, VP>(s_v + ch * VR * VP, ti0 - 1, tj0 - 1, H, W,
                              [&](int64_t g) { const T xv = Xc[g]; return dfma(m, xv - XPc[g], xv); });
        load_tile<VR, VP, VP>(s_d + ch * VR * VP, ti0 - 1, tj0 - 1, H, W, [&](int64_t g) { return Gc[g] * ninvL; });
    }
    __syncthreads();

    // ---- TV part of the decrease, per site
    const double e2 = I.pr.eps_tv * I.pr.eps_tv;
    double dtv = 0.0;
#pragma unroll
    for (int o = 0; o < R; ++o) {
        const int li = li0 + o, gi = ti0 + li;
        if (gi < H && gj < W) {
            const int idx = (li + 1) * VP + tx + 1;
            const bool hx = gj < W - 1, vx = gi < H - 1;
            double ds2 = 0.0, s2 = 0.0;
            for (int ch = 0; ch < C; ++ch) {
                const T* V = s_v + ch * VR * VP;
                const T* D = s_d + ch * VR * VP;
                const double bh = hx ? (double)(V[idx + 1] - V[idx]) : 0.0;
                const double bv = vx ? (double)(V[idx + VP] - V[idx]) : 0.0;
                const double ah = hx ? (double)(D[idx + 1] - D[idx]) : 0.0;
                const double av = vx ? (double)(D[idx + VP] - D[idx]) : 0.0;
                if (reg == 2) {
                    ds2 += ah * (bh + 0.5 * ah) + av * (bv + 0.5 * av);
                } else if (reg == 1) {
                    const double d2 = ah * (ah + 2.0 * bh) + av * (av + 2.0 * bv);
                    const double q2 = bh * bh + bv * bv;
                    dtv += d2 / (sqrt(q2 + d2 + e2) + sqrt(q2 + e2));
                } else {
                    ds2 += ah * (ah + 2.0 * bh) + av * (av + 2.0 * bv);
                    s2 += bh * bh + bv * bv;
                }
            }
            if (reg == 2) dtv += ds2;
            else if (reg == 0) dtv += ds2 / (sqrt(s2 + ds2 + e2) + sqrt(s2 + e2));
        }
    }

    // ---- data part, and the new iterate
    double ddat = 0.0;
    for (int ch = 0; ch < C; ++ch) {
        const T* Gc = G + ch * HW;
        __syncthreads();
        load_tile<CR, CP, CP>(s_c, ti0 - c0, tj0 - c0, H, W, [&](int64_t g) { return Gc[g] * ninvL; });
        __syncthreads();
        T acc[R];
#pragma unroll
        for (int o = 0; o < R; ++o) acc[o] = T(0);
        correlate<T, K, R>(s_c, CP, I.thf, li0, tx, acc);
        const T* V = s_v + ch * VR * VP;
#pragma unroll
        for (int o = 0; o < R; ++o) {
            const int li = li0 + o, gi = ti0 + li;
            if (gi < H && gj < W) {
                const int64_t e = ch * HW + (int64_t)gi * W + gj;
                const T kx = KX[e];
                const T kv = dfma(m, kx - KXP[e], kx);
                const T d = acc[o];
                const double rv = (double)kv - (double)Y[e];
                ddat += (double)d * (rv + 0.5 * (double)d);
                const int idx = (li + 1) * VP + tx + 1;
                XN[e] = V[idx] + s_d[ch * VR * VP + idx];
                KXN[e] = kv + d;
            }
        }
    }
    block_partial(ddat + I.pr.alpha * dtv, I.pB, lb);
}

// xout = v = x + m (x - x_prev): the point that passed the stop test
// (instances whose solve failed are left untouched).
template <typename T>
__global__ __launch_bounds__(kNT) void k_apg_final(const Inst<T>* __restrict__ insts, const int* __restrict__ blk,
                                                   const ApgState* __restrict__ sin) {
    MAID_EW_PROLOGUE
    const ApgState st = sin[ii];
    if (st.status < 0 || !I.xout) return;
    const T* X = pick(I.X[0], I.X[1], I.X[2], st.cur);
    const T* XP = pick(I.X[0], I.X[1], I.X[2], st.prev);
    const T m = (T)st.m;
    T* out = I.xout;
    for (int64_t e = (int64_t)lb * kNT + threadIdx.x; e < I.N; e += (int64_t)I.nbe * kNT) {
        const T xv = X[e];
        out[e] = dfma(m, xv - XP[e], xv);
    }
}

// ------------------------------------------------------------------ conjugate gradients
// Direction pass.  Per instance: reads sin, block 0 writes sout.  Finishes
// gamma = ||r||^2 from the partials of the update (or set-up) pass, applies
// the stop tests (sqrt(gamma) <= tol; iteration cap), then forms
// p_new = r + beta p_old (p_new = r on the first iteration, beta =
// gamma / gamma_prev) and Kp = theta*p_new.  init = 1: the set-up call that
// only copies r (holding q0) into p and forms theta*q0, without touching the
// state.
template <typename T, int K, int R>
__global__ __launch_bounds__(kNT) void k_cg_dir(const Inst<T>* __restrict__ insts, const int* __restrict__ blk,
                                                const CgState* __restrict__ sin, CgState* __restrict__ sout, int init) {
    MAID_STENCIL_PROLOGUE
    CgState st = sin[ii];
    const bool writer = lb == 0 && threadIdx.x == 0;
    if (st.done) {
        if (writer && !init) put_state(&sout[ii], st);
        return;
    }
    double beta = 0.0;
    if (!init) {
        const double g = reduce_partials(I.pR, I.nbe);
        if (st.first) {
            st.first = 0;
        } else {
            beta = g / st.gamma;
        }
        st.gamma = g;
        if (!finite_d(g)) {
            st.done = 1;
            st.status = ST_NONFINITE;
        } else if (sqrt(g) <= st.tol) {
            st.done = 1;
            st.status = ST_OK;
        } else if (st.iters >= st.max) {
            st.done = 1;
            st.status = ST_MAXITER;
        }
        if (writer) put_state(&sout[ii], st);
        if (st.done) return;
    }
    constexpr int TH = tile_h(R), c0 = (K - 1) / 2, CP = cv_pitch(K), CR = cv_rows(K, R);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* s = reinterpret_cast<T*>(smem_raw);
    const int C = I.pr.C, H = I.pr.H, W = I.pr.W;
    const int64_t HW = (int64_t)H * W;
    const int ntx = (W + kTW - 1) / kTW;
    const int tile = xcd_tile(lb, I.nb);
    const int ti0 = (tile / ntx) * TH, tj0 = (tile % ntx) * kTW;
    const int tx = threadIdx.x & 63, li0 = (threadIdx.x >> 6) * R;
    const int gj = tj0 + tx;
    const T bT = (T)beta;
    const T* __restrict__ Pold = pick(I.P[0], I.P[1], st.pc);
    T* __restrict__ Pnew = pick(I.P[0], I.P[1], st.pc ^ 1);
    for (int ch = 0; ch < C; ++ch) {
        const T* rc = I.r + ch * HW;
        const T* pc = Pold + ch * HW;
        __syncthreads();
        if (beta == 0.0)
            load_tile<CR, CP, CP>(s, ti0 - c0, tj0 - c0, H, W, [&](int64_t g) { return rc[g]; });
        else
            load_tile<CR, CP, CP>(s, ti0 - c0, tj0 - c0, H, W, [&](int64_t g) { return dfma(bT, pc[g], rc[g]); });
        __syncthreads();
        T acc[R];
#pragma unroll
        for (int o = 0; o < R; ++o) acc[o] = T(0);
        correlate<T, K, R>(s, CP, I.thf, li0, tx, acc);
#pragma unroll
        for (int o = 0; o < R; ++o) {
            const int li = li0 + o, gi = ti0 + li;
            if (gi < H && gj < W) {
                const int64_t e = ch * HW + (int64_t)gi * W + gj;
                Pnew[e] = s[(li + c0) * CP + tx + c0];
                I.Kp[e] = acc[o];
            }
        }
    }
}

// Hessian pass.  Per instance: reads sin, block 0 writes sout.
// Hp = theta . Kp + alpha grad^2 R(xt)[p] and per-block partials of <p,Hp>;
// grad^2 R(x)[p] = D^T (w Dp - w^3 m Dx), m = <Dx, Dp> over the coupled
// channels.  init = 1 computes H q0 only.
template <typename T, int K, int R>
__global__ __launch_bounds__(kNT) void k_cg_hvp(const Inst<T>* __restrict__ insts, const int* __restrict__ blk,
                                                const CgState* __restrict__ sin, CgState* __restrict__ sout, int init) {
    MAID_STENCIL_PROLOGUE
    const CgState st = sin[ii];
    if (!init && lb == 0 && threadIdx.x == 0) put_state(&sout[ii], st);
    if (st.done) return;
    constexpr int TH = tile_h(R), c0 = (K - 1) / 2, CP = cv_pitch(K), CR = cv_rows(K, R);
    constexpr int VP = tv_pitch(), VR = tv_rows(R), WP = fx_pitch(), WR = fx_rows(R);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* sm = reinterpret_cast<T*>(smem_raw);
    const int C = I.pr.C, H = I.pr.H, W = I.pr.W, reg = I.pr.reg;
    const int nw = reg == 1 ? C : 1;
    const int64_t HW = (int64_t)H * W;
    const int ntx = (W + kTW - 1) / kTW;
    const int tile = xcd_tile(lb, I.nb);
    const int ti0 = (tile / ntx) * TH, tj0 = (tile % ntx) * kTW;
    const int tx = threadIdx.x & 63, li0 = (threadIdx.x >> 6) * R;
    const int gj = tj0 + tx;
    const T alpha = (T)I.pr.alpha;
    const T* __restrict__ P = pick(I.P[0], I.P[1], st.pc ^ 1);

    T* s_x = sm;
    T* s_p = sm + C * VR * VP;
    T* s_w = sm + 2 * C * VR * VP;
    T* s_mw = s_w + nw * WR * WP;
    for (int ch = 0; ch < C; ++ch) {
        const T* xc = I.xt + ch * HW;
        const T* pc = P + ch * HW;
        load_tile<VR, VP, VP>(s_x + ch * VR * VP, ti0 - 1, tj0 - 1, H, W, [&](int64_t g) { return xc[g]; });
        load_tile<VR, VP, VP>(s_p + ch * VR * VP, ti0 - 1, tj0 - 1, H, W, [&](int64_t g) { return pc[g]; });
    }
    __syncthreads();
    const T eps2 = (T)(I.pr.eps_tv * I.pr.eps_tv);
    for (int idx = threadIdx.x; idx < WR * WP; idx += kNT) {
        const int r = idx / WP, cc = idx - r * WP;
        const int gi = ti0 - 1 + r, gj2 = tj0 - 1 + cc;
        const bool in = (gi >= 0 && gi < H && gj2 >= 0 && gj2 < W);
        const bool hx = gj2 < W - 1, vx = gi < H - 1;
        T s2 = T(0), mm = T(0);
        for (int ch = 0; ch < C; ++ch) {
            const T* Xv = s_x + ch * VR * VP;
            const T* Pv = s_p + ch * VR * VP;
            const int i0 = r * VP + cc;
            const T xh = hx ? Xv[i0 + 1] - Xv[i0] : T(0);
            const T xv = vx ? Xv[i0 + VP] - Xv[i0] : T(0);
            const T ph = hx ? Pv[i0 + 1] - Pv[i0] : T(0);
            const T pv = vx ? Pv[i0 + VP] - Pv[i0] : T(0);
            if (reg == 1) {
                const T w = in ? T(1) / dsqrt(xh * xh + xv * xv + eps2) : T(0);
                s_w[ch * WR * WP + idx] = w;
                s_mw[ch * WR * WP + idx] = w * w * w * (xh * ph + xv * pv);
            } else {
                s2 += xh * xh + xv * xv;
                mm += xh * ph + xv * pv;
            }
        }
        if (reg == 0) {
            const T w = in ? T(1) / dsqrt(s2 + eps2) : T(0);
            s_w[idx] = w;
            s_mw[idx] = w * w * w * mm;
        } else if (reg == 2) {
            s_w[idx] = in ? T(1) : T(0);
            s_mw[idx] = T(0);
        }
    }
    __syncthreads();
    T hv0[R], hv1[R], hv2[R], pp0[R], pp1[R], pp2[R];
#pragma unroll
    for (int o = 0; o < R; ++o) {
        const int li = li0 + o, gi = ti0 + li;
        const int r = li + 1, cc = tx + 1;
#pragma unroll
        for (int ch = 0; ch < kMaxC; ++ch) {
            T hv = T(0), pcen = T(0);
            if (ch < C) {
                const T* Xv = s_x + ch * VR * VP;
                const T* Pv = s_p + ch * VR * VP;
                const T* Wt = s_w + (reg == 1 ? ch * WR * WP : 0);
                const T* Mw = s_mw + (reg == 1 ? ch * WR * WP : 0);
                const int i0 = r * VP + cc;
                pcen = Pv[i0];
                const T xh_h = (gj < W - 1) ? Xv[i0 + 1] - Xv[i0] : T(0);
                const T ph_h = (gj < W - 1) ? Pv[i0 + 1] - Pv[i0] : T(0);
                const T xv_h = (gi < H - 1) ? Xv[i0 + VP] - Xv[i0] : T(0);
                const T pv_h = (gi < H - 1) ? Pv[i0 + VP] - Pv[i0] : T(0);
                const T xh_l = Xv[i0] - Xv[i0 - 1], ph_l = Pv[i0] - Pv[i0 - 1];
                const T xv_u = Xv[i0] - Xv[i0 - VP], pv_u = Pv[i0] - Pv[i0 - VP];
                const int f0 = r * WP + cc, fl = f0 - 1, fu = f0 - WP;
                const T fh_here = Wt[f0] * ph_h - Mw[f0] * xh_h;
                const T fv_here = Wt[f0] * pv_h - Mw[f0] * xv_h;
                const T fh_left = Wt[fl] * ph_l - Mw[fl] * xh_l;
                const T fv_up = Wt[fu] * pv_u - Mw[fu] * xv_u;
                hv = fh_left - fh_here + fv_up - fv_here;
            }
            if (ch == 0) { hv0[o] = hv; pp0[o] = pcen; }
            if (ch == 1) { hv1[o] = hv; pp1[o] = pcen; }
            if (ch == 2) { hv2[o] = hv; pp2[o] = pcen; }
        }
    }

    double kap = 0.0;
    for (int ch = 0; ch < C; ++ch) {
        const T* kc = I.Kp + ch * HW;
        __syncthreads();
        load_tile<CR, CP, CP>(sm, ti0 - c0, tj0 - c0, H, W, [&](int64_t g) { return kc[g]; });
        __syncthreads();
        T acc[R];
#pragma unroll
        for (int o = 0; o < R; ++o) acc[o] = T(0);
        correlate<T, K, R>(sm, CP, I.th, li0, tx, acc);
#pragma unroll
        for (int o = 0; o < R; ++o) {
            const int gi = ti0 + li0 + o;
            if (gi < H && gj < W) {
                const int64_t e = ch * HW + (int64_t)gi * W + gj;
                const T hp = dfma(alpha, pick3<T, R>(hv0, hv1, hv2, ch, o), acc[o]);
                I.Hp[e] = hp;
                kap += (double)pick3<T, R>(pp0, pp1, pp2, ch, o) * (double)hp;
            }
        }
    }
    if (!init) block_partial(kap, I.pK, lb);
}

// Update pass.  Per instance: reads sin, block 0 writes sout.  Finishes the
// curvature kappa = <p,Hp> (not positive: MAID_NOT_SPD), a = gamma/kappa,
// then q += a p, r -= a Hp and per-block partials of ||r||^2.
template <typename T>
__global__ __launch_bounds__(kNT) void k_cg_update(const Inst<T>* __restrict__ insts, const int* __restrict__ blk,
                                                   const CgState* __restrict__ sin, CgState* __restrict__ sout) {
    MAID_EW_PROLOGUE
    CgState st = sin[ii];
    const bool writer = lb == 0 && threadIdx.x == 0;
    if (st.done) {
        if (writer) put_state(&sout[ii], st);
        return;
    }
    const double kappa = reduce_partials(I.pK, I.nb);
    st.kappa = kappa;
    if (!(kappa > 0.0) || !finite_d(kappa)) {
        st.done = 1;
        st.status = finite_d(kappa) ? ST_NOT_SPD : ST_NONFINITE;
        if (writer) put_state(&sout[ii], st);
        return;
    }
    const T* __restrict__ P = pick(I.P[0], I.P[1], st.pc ^ 1);
    st.a = st.gamma / kappa;
    st.iters += 1;
    st.pc ^= 1;
    if (writer) put_state(&sout[ii], st);
    const T a = (T)st.a;
    T* __restrict__ q = I.q;
    T* __restrict__ r = I.r;
    const T* __restrict__ Hp = I.Hp;
    double rs = 0.0;
    for (int64_t e = (int64_t)lb * kNT + threadIdx.x; e < I.N; e += (int64_t)I.nbe * kNT) {
        const T pv = P[e];
        q[e] = dfma(a, pv, q[e]);
        const T rv = dfma(-a, Hp[e], r[e]);
        r[e] = rv;
        rs += (double)rv * (double)rv;
    }
    block_partial(rs, I.pR, lb);
}

// r = b - H q0 (Hp holds H q0) and per-block partials of ||r||^2.
template <typename T>
__global__ __launch_bounds__(kNT) void k_cg_init(const Inst<T>* __restrict__ insts, const int* __restrict__ blk,
                                                 const CgState* __restrict__ sin) {
    MAID_EW_PROLOGUE
    if (sin[ii].done) return;
    const T* __restrict__ b = I.b;
    const T* __restrict__ Hp = I.Hp;
    T* __restrict__ r = I.r;
    double rs = 0.0;
    for (int64_t e = (int64_t)lb * kNT + threadIdx.x; e < I.N; e += (int64_t)I.nbe * kNT) {
        const T rv = b[e] - Hp[e];
        r[e] = rv;
        rs += (double)rv * (double)rv;
    }
    block_partial(rs, I.pR, lb);
}

// ------------------------------------------------------------------ small kernels
// One block per instance: theta64 (double, KxK) -> th (correlation form) and
// thf (flipped, convolution form), both column-major in the compute type;
// with L_io, the l1 norm squared becomes the starting Lipschitz estimate
// when that is <= 0; red[slot_abs] receives the l1 norm when slot_abs >= 0.
template <typename T>
__global__ __launch_bounds__(1024) void k_prep_kernel(const Inst<T>* __restrict__ insts, ApgState* __restrict__ Lst,
                                                      int slot_abs) {
    __shared__ double s_abs[1024];
    const Inst<T>& I = insts[blockIdx.x];
    if (!I.theta64) return;
    const int K = I.K, KK = K * K;
    const int t = threadIdx.x;
    double a = 0.0;
    if (t < KK) {
        const int u = t / K, v = t - u * K;
        const double w = I.theta64[t];
        // column-major: out(u,v) at v*K+u; the flipped kernel f(u',v') = theta(K-1-u', K-1-v')
        I.th[v * K + u] = (T)w;
        I.thf[(K - 1 - v) * K + (K - 1 - u)] = (T)w;
        a = fabs(w);
    }
    s_abs[t] = a;
    __syncthreads();
    if (t == 0) {
        double s = 0.0;
        for (int i = 0; i < KK; ++i) s += s_abs[i];
        if (Lst && !(Lst[blockIdx.x].L > 0.0)) Lst[blockIdx.x].L = s * s;
        if (slot_abs >= 0) I.red[slot_abs] = s;
    }
}

// One block per instance: red[slot] = sum of the instance's cv_part partials.
template <typename T>
__global__ __launch_bounds__(kNT) void k_reduce(const Inst<T>* __restrict__ insts, int slot) {
    const Inst<T>& I = insts[blockIdx.x];
    if (!I.cv_part) return;
    const double s = reduce_partials(I.cv_part, I.nb);
    if (threadIdx.x == 0) I.red[slot] = s;
}

// ------------------------------------------------------------------ hypergradient
// Z(u,v) = sum_{c,i',j} A(i'-c0+u, j) B(i', j+c0-v) for (A,B) = (rho, q) and
// (theta*q, x_tilde): a [K x P] . [P x K] contraction over all pixels, on
// the FP64 matrix cores (v_mfma_f64_16x16x4: u on the M axis, v on the N
// axis, four pixels per instruction on the K axis).  FP32 operands are
// widened exactly, so the whole sum is accumulated in double.  KT = 16 or 32
// is K rounded up to the MFMA tile; padded taps read as zero.
typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int kHgTI = 16, kHgTJ = 64;

template <typename T, int KT>
__global__ __launch_bounds__(kNT) void k_hg_corr(int C, int H, int W, int K, const T* __restrict__ rho, const T* __restrict__ q,
                                                 const T* __restrict__ wq, const T* __restrict__ xt, double* __restrict__ part) {
    constexpr int NO = KT / 16;
    constexpr int AP = kHgTJ + 1;            // A tile: rows TI+K-1, cols TJ
    constexpr int BP = kHgTJ + kMaxK;        // B tile: rows TI, cols TJ+K-1
    __shared__ T sA[(kHgTI + kMaxK - 1) * AP];
    __shared__ T sB[kHgTI * BP];
    __shared__ double s_red[4][KT * KT];
    const int c0 = (K - 1) / 2;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int kk = lane >> 4, nn = lane & 15;
    const int64_t HW = (int64_t)H * W;
    const int ntj = (W + kHgTJ - 1) / kHgTJ, nti = (H + kHgTI - 1) / kHgTI;
    const int nitems = ntj * nti * C * 2;
    d4_t acc[NO][NO];
#pragma unroll
    for (int a = 0; a < NO; ++a)
#pragma unroll
        for (int bq = 0; bq < NO; ++bq) acc[a][bq] = d4_t{0.0, 0.0, 0.0, 0.0};

    const int arows = kHgTI + K - 1, bcols = kHgTJ + K - 1;
    for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
        const int term = item & 1;
        const int ch = (item >> 1) % C;
        const int sp = (item >> 1) / C;
        const int ti0 = (sp / ntj) * kHgTI, tj0 = (sp % ntj) * kHgTJ;
        const T* Asrc = (term ? wq : rho) + ch * HW;
        const T* Bsrc = (term ? xt : q) + ch * HW;
        __syncthreads();
        for (int idx = threadIdx.x; idx < arows * kHgTJ; idx += kNT) {
            const int r = idx / kHgTJ, cc = idx - r * kHgTJ;
            const int gi = ti0 - c0 + r, gj = tj0 + cc;
            sA[r * AP + cc] = (gi >= 0 && gi < H && gj < W) ? Asrc[(int64_t)gi * W + gj] : T(0);
        }
        for (int idx = threadIdx.x; idx < kHgTI * bcols; idx += kNT) {
            const int r = idx / bcols, cc = idx - r * bcols;
            const int gi = ti0 + r, gj = tj0 - c0 + cc;
            sB[r * BP + cc] = (gi < H && gj >= 0 && gj < W) ? Bsrc[(int64_t)gi * W + gj] : T(0);
        }
        __syncthreads();
        for (int li = wid; li < kHgTI; li += 4) {
#pragma unroll 4
            for (int g = 0; g < kHgTJ / 4; ++g) {
                const int jj = 4 * g + kk;
                double av[NO], bv[NO];
#pragma unroll
                for (int t = 0; t < NO; ++t) {
                    const int u = 16 * t + nn;
                    av[t] = (u < K) ? (double)sA[(li + u) * AP + jj] : 0.0;
                    bv[t] = (u < K) ? (double)sB[li * BP + jj + 2 * c0 - u] : 0.0;
                }
#pragma unroll
                for (int a = 0; a < NO; ++a)
#pragma unroll
                    for (int bq = 0; bq < NO; ++bq)
                        acc[a][bq] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[bq], acc[a][bq], 0, 0, 0);
            }
        }
    }
    // D layout of the 16x16 f64 result (measured on gfx950): register r of
    // lane l holds row (l/16) + 4r, column l%16
#pragma unroll
    for (int a = 0; a < NO; ++a)
#pragma unroll
        for (int bq = 0; bq < NO; ++bq)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int u = 16 * a + kk + 4 * r, v = 16 * bq + nn;
                s_red[wid][u * KT + v] = acc[a][bq][r];
            }
    __syncthreads();
    for (int i = threadIdx.x; i < KT * KT; i += kNT)
        part[(size_t)blockIdx.x * KT * KT + i] = ((s_red[0][i] + s_red[1][i]) + s_red[2][i]) + s_red[3][i];
}

// z = -sum_blocks Z + with_r * grad r(theta); ||z||^2 into *znorm2.
template <int KT>
__global__ __launch_bounds__(1024) void k_hg_final(double beta, double h1_w0, const double* __restrict__ part, int nblk, int K,
                                                   const double* __restrict__ th, const double* __restrict__ a, int with_r,
                                                   double* __restrict__ z, double* __restrict__ znorm2) {
    __shared__ double s_e[1024];
    __shared__ double s_z[1024];
    const int t = threadIdx.x, KK = K * K;
    if (t < KK) s_e[t] = (with_r && a) ? th[t] - a[t] : 0.0;
    __syncthreads();
    double zz = 0.0;
    if (t < KK) {
        const int u = t / K, v = t - u * K;
        double s = 0.0;
#pragma unroll 8
        for (int bidx = 0; bidx < nblk; ++bidx) s += part[(size_t)bidx * KT * KT + u * KT + v];
        double gr = 0.0;
        if (with_r && a) {
            // D^T D e with Neumann differences = sum over in-grid neighbours of (e - e_nb)
            const double e = s_e[t];
            double lap = 0.0;
            if (u > 0) lap += e - s_e[t - K];
            if (u < K - 1) lap += e - s_e[t + K];
            if (v > 0) lap += e - s_e[t - 1];
            if (v < K - 1) lap += e - s_e[t + 1];
            gr = 2.0 * beta * (h1_w0 * e + lap);
        }
        zz = -s + gr;
        z[t] = zz;
    }
    s_z[t] = zz * zz;
    __syncthreads();
    if (t == 0) {
        double s = 0.0;
        for (int i = 0; i < KK; ++i) s += s_z[i];
        *znorm2 = s;
    }
}

}  // namespace maid
