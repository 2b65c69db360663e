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
// then the four waves in a fixed order, then the per-block partials are
// combined by the last block to finish (agent-scope acquire/release
// counter), in a fixed order.  That last block also takes the solver's
// scalar decisions (stop tests, backtracking, CG coefficients) and writes
// them to the device-resident DevCtx, so no host round trip is needed
// between passes.
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

// Grid-wide sum of NV doubles per thread.  Returns true in the block that
// finishes last; there tot[k] (shared) holds the totals for every thread.
// The counter is reset to zero by that block for the next launch.
template <int NV>
__device__ bool grid_reduce(const double (&v)[NV], double* partials, unsigned* counter, double* tot) {
    __shared__ double s_w[NV][4];
    __shared__ int s_last;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nb = gridDim.x;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double w = wave_sum(v[k]);
        if (lane == 0) s_w[k][wid] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const double s = ((s_w[k][0] + s_w[k][1]) + s_w[k][2]) + s_w[k][3];
            __hip_atomic_store(&partials[(size_t)k * nb + blockIdx.x], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __threadfence();
        const unsigned prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_last = (prev == (unsigned)(nb - 1));
    }
    __syncthreads();
    if (!s_last) return false;
    __threadfence();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nb; b += kNT)
            s += __hip_atomic_load(&partials[(size_t)k * nb + b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const double w = wave_sum(s);
        if (lane == 0) s_w[k][wid] = w;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        const int k = threadIdx.x;
        tot[k] = ((s_w[k][0] + s_w[k][1]) + s_w[k][2]) + s_w[k][3];
    }
    if (threadIdx.x == 0) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    return true;
}

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

// ------------------------------------------------------------------ generic convolution pass
// out = ker (x) in  [- sub]   (correlation with ker; pass the flipped kernel
// for the true convolution), optional grid total of out^2 into c->red[slot].
template <typename T, int K, int R>
__global__ __launch_bounds__(kNT) void k_conv(DevCtx* __restrict__ c, const T* __restrict__ ker, const T* __restrict__ in,
                                              const T* __restrict__ sub, T* __restrict__ out, int slot,
                                              double* partials, unsigned* counter) {
    constexpr int TH = tile_h(R), c0 = (K - 1) / 2, CP = cv_pitch(K), CR = cv_rows(K, R);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* s = reinterpret_cast<T*>(smem_raw);
    const int C = c->C, H = c->H, W = c->W;
    const int64_t HW = (int64_t)H * W;
    const int ntx = (W + kTW - 1) / kTW, nty = (H + TH - 1) / TH;
    const int tile = xcd_tile(blockIdx.x, ntx * nty);
    const int ti0 = (tile / ntx) * TH, tj0 = (tile % ntx) * kTW;
    const int tx = threadIdx.x & 63, li0 = (threadIdx.x >> 6) * R;
    double sq = 0.0;
    for (int ch = 0; ch < C; ++ch) {
        const T* src = in + ch * HW;
        __syncthreads();
        load_tile<CR, CP, CP>(s, ti0 - c0, tj0 - c0, H, W, [&](int64_t g) { return src[g]; });
        __syncthreads();
        T acc[R];
#pragma unroll
        for (int o = 0; o < R; ++o) acc[o] = T(0);
        correlate<T, K, R>(s, CP, ker, li0, tx, acc);
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
    if (slot >= 0) {
        __shared__ double tot[1];
        const double v[1] = {sq};
        if (grid_reduce<1>(v, partials, counter, tot) && threadIdx.x == 0) c->red[slot] = tot[0];
    }
}

// ------------------------------------------------------------------ lower level: FISTA
// Pass A: at the extrapolated point v = x + m (x - x_prev), with
// theta*v = Kx + m (Kx - Kx_prev) by linearity,
//   G = theta . (theta*v - y) + alpha grad R(v),  and ||G||^2 (grid total);
// the last block applies the stop test ||G|| <= tol.
template <typename T, int K, int R>
__global__ __launch_bounds__(kNT) void k_apg_grad(DevCtx* __restrict__ c, ApgBufs<T> b) {
    if (c->done | (c->phase != 0)) return;
    constexpr int TH = tile_h(R), c0 = (K - 1) / 2, CP = cv_pitch(K), CR = cv_rows(K, R);
    constexpr int VP = tv_pitch(), VR = tv_rows(R);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* sm = reinterpret_cast<T*>(smem_raw);
    const int C = c->C, H = c->H, W = c->W, reg = c->reg;
    const int64_t HW = (int64_t)H * W;
    const int ntx = (W + kTW - 1) / kTW, nty = (H + TH - 1) / TH;
    const int tile = xcd_tile(blockIdx.x, ntx * nty);
    const int ti0 = (tile / ntx) * TH, tj0 = (tile % ntx) * kTW;
    const int tx = threadIdx.x & 63, li0 = (threadIdx.x >> 6) * R;
    const int gj = tj0 + tx;
    const T m = (T)c->m;
    const T alpha = (T)c->alpha;
    const T* __restrict__ X = b.X[c->cur];
    const T* __restrict__ XP = b.X[c->prev];
    const T* __restrict__ KX = b.KX[c->cur];
    const T* __restrict__ KXP = b.KX[c->prev];
    const T* __restrict__ Y = b.y;

    // ---- TV gradient at v (all channels staged: the magnitude couples them)
    T* s_v = sm;
    T* s_w = sm + C * VR * VP;
    for (int ch = 0; ch < C; ++ch) {
        const T* Xc = X + ch * HW;
        const T* XPc = XP + ch * HW;
        load_tile<VR, VP, VP>(s_v + ch * VR * VP, ti0 - 1, tj0 - 1, H, W,
                              [&](int64_t g) { const T xv = Xc[g]; return dfma(m, xv - XPc[g], xv); });
    }
    __syncthreads();
    tv_weights<T, R>(s_v, s_w, C, reg, (T)(c->eps_tv * c->eps_tv), ti0, tj0, H, W);
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
        correlate<T, K, R>(sm, CP, b.th, li0, tx, acc);
#pragma unroll
        for (int o = 0; o < R; ++o) {
            const int gi = ti0 + li0 + o;
            if (gi < H && gj < W) {
                const T gv = dfma(alpha, pick3<T, R>(tg0, tg1, tg2, ch, o), acc[o]);
                b.G[ch * HW + (int64_t)gi * W + gj] = gv;
                gsq += (double)gv * (double)gv;
            }
        }
    }

    __shared__ double tot[1];
    const double v[1] = {gsq};
    if (grid_reduce<1>(v, b.partials, b.counter, tot) && threadIdx.x == 0) {
        const double gn2 = tot[0];
        c->gn2 = gn2;
        c->nb_iter = 0;
        if (!(gn2 <= 1.0e300)) {
            c->done = 1;
            c->status = ST_NONFINITE;
        } else if (sqrt(gn2) <= c->tol) {
            c->done = 1;
            c->status = ST_OK;
        } else if (c->iters >= c->max_iter) {
            c->done = 1;
            c->status = ST_MAXITER;
        } else {
            c->phase = 1;
        }
    }
}

// Pass B: trial x+ = v + dl with dl = -G/L.  Writes x+ and theta*x+ =
// theta*v + theta*dl into the spare buffers and forms the decrease
// h(x+) - h(v) through the increment (no cancellation of objective values):
//   data: sum d (r_v + d/2), d = theta*dl;
//   TV:   sum_sites (s'^2 - s^2) / (sqrt(s'^2+eps^2) + sqrt(s^2+eps^2)),
//         s'^2 - s^2 = sum a (a + 2 b), a = D dl, b = D v,
// all per-element products in double.  The last block accepts the step
// (h(x+) - h(v) <= -||G||^2 / (2L)) and rotates the buffers, or doubles L.
template <typename T, int K, int R>
__global__ __launch_bounds__(kNT) void k_apg_trial(DevCtx* __restrict__ c, ApgBufs<T> b) {
    if (c->done | (c->phase != 1)) return;
    constexpr int TH = tile_h(R), c0 = (K - 1) / 2, CP = cv_pitch(K), CR = cv_rows(K, R);
    constexpr int VP = tv_pitch(), VR = tv_rows(R);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* sm = reinterpret_cast<T*>(smem_raw);
    const int C = c->C, H = c->H, W = c->W, reg = c->reg;
    const int64_t HW = (int64_t)H * W;
    const int ntx = (W + kTW - 1) / kTW, nty = (H + TH - 1) / TH;
    const int tile = xcd_tile(blockIdx.x, ntx * nty);
    const int ti0 = (tile / ntx) * TH, tj0 = (tile % ntx) * kTW;
    const int tx = threadIdx.x & 63, li0 = (threadIdx.x >> 6) * R;
    const int gj = tj0 + tx;
    const double L = c->L;
    const T m = (T)c->m;
    const T ninvL = (T)(-1.0 / L);
    const int cur = c->cur, prv = c->prev, nxt = c->nxt;
    const T* __restrict__ X = b.X[cur];
    const T* __restrict__ XP = b.X[prv];
    const T* __restrict__ KX = b.KX[cur];
    const T* __restrict__ KXP = b.KX[prv];
    T* __restrict__ XN = b.X[nxt];
    T* __restrict__ KXN = b.KX[nxt];
    const T* __restrict__ G = b.G;
    const T* __restrict__ Y = b.y;

    T* s_v = sm;
    T* s_d = sm + C * VR * VP;
    T* s_c = sm + 2 * C * VR * VP;
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
    const double e2 = c->eps_tv * c->eps_tv;
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
        correlate<T, K, R>(s_c, CP, b.thf, li0, tx, acc);
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

    __shared__ double tot[1];
    const double v[1] = {ddat + c->alpha * dtv};
    if (grid_reduce<1>(v, b.partials, b.counter, tot) && threadIdx.x == 0) {
        const double delta = tot[0];
        c->delta_last = delta;
        if (!(delta <= 1.0e300 && delta >= -1.0e300)) {
            c->done = 1;
            c->status = ST_NONFINITE;
        } else if (delta <= -c->gn2 / (2.0 * L)) {
            if (b.trace && c->iters < c->trace_cap) b.trace[c->iters] = c->nb_iter;
            c->iters += 1;
            const int p = c->prev;
            c->prev = c->cur;
            c->cur = c->nxt;
            c->nxt = p;
            const double t = c->t;
            const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
            c->t_prev = t;
            c->t = tn;
            c->m = (t - 1.0) / tn;
            c->phase = 0;
        } else {
            c->L = 2.0 * L;
            c->bt += 1;
            c->nb_iter += 1;
            if (c->nb_iter > 200) {
                c->done = 1;
                c->status = ST_NONFINITE;
            }
        }
    }
}

// x_out = v = x + m (x - x_prev): the point that passed the stop test
template <typename T>
__global__ __launch_bounds__(kNT) void k_apg_final(const DevCtx* __restrict__ c, const T* __restrict__ X0, const T* __restrict__ X1,
                                                   const T* __restrict__ X2, T* __restrict__ out, int64_t n) {
    const T* X = c->cur == 0 ? X0 : (c->cur == 1 ? X1 : X2);
    const T* XP = c->prev == 0 ? X0 : (c->prev == 1 ? X1 : X2);
    const T m = (T)c->m;
    for (int64_t e = (int64_t)blockIdx.x * kNT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kNT) {
        const T xv = X[e];
        out[e] = dfma(m, xv - XP[e], xv);
    }
}

// ------------------------------------------------------------------ conjugate gradients
// Pass 1: p_new = r + beta p_old (p_new = r when beta = 0) and Kp = theta*p_new.
template <typename T, int K, int R>
__global__ __launch_bounds__(kNT) void k_cg_dir(DevCtx* __restrict__ c, CgBufs<T> b) {
    if (c->cg_done) return;
    constexpr int TH = tile_h(R), c0 = (K - 1) / 2, CP = cv_pitch(K), CR = cv_rows(K, R);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* s = reinterpret_cast<T*>(smem_raw);
    const int C = c->C, H = c->H, W = c->W;
    const int64_t HW = (int64_t)H * W;
    const int ntx = (W + kTW - 1) / kTW, nty = (H + TH - 1) / TH;
    const int tile = xcd_tile(blockIdx.x, ntx * nty);
    const int ti0 = (tile / ntx) * TH, tj0 = (tile % ntx) * kTW;
    const int tx = threadIdx.x & 63, li0 = (threadIdx.x >> 6) * R;
    const int gj = tj0 + tx;
    const double beta = c->cg_b;
    const T bT = (T)beta;
    const T* __restrict__ Pold = b.P[c->pc];
    T* __restrict__ Pnew = b.P[c->pc ^ 1];
    for (int ch = 0; ch < C; ++ch) {
        const T* rc = b.r + ch * HW;
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
        correlate<T, K, R>(s, CP, b.thf, li0, tx, acc);
#pragma unroll
        for (int o = 0; o < R; ++o) {
            const int li = li0 + o, gi = ti0 + li;
            if (gi < H && gj < W) {
                const int64_t e = ch * HW + (int64_t)gi * W + gj;
                Pnew[e] = s[(li + c0) * CP + tx + c0];
                b.Kp[e] = acc[o];
            }
        }
    }
}

// Pass 2: Hp = theta . Kp + alpha grad^2 R(xt)[p] and the curvature <p,Hp>.
// grad^2 R(x)[p] = D^T (w Dp - w^3 m Dx), m = <Dx, Dp> over the coupled
// channels.  init = 1 computes H q0 only (no solver decisions).
template <typename T, int K, int R>
__global__ __launch_bounds__(kNT) void k_cg_hvp(DevCtx* __restrict__ c, CgBufs<T> b, int init) {
    if (c->cg_done) return;
    constexpr int TH = tile_h(R), c0 = (K - 1) / 2, CP = cv_pitch(K), CR = cv_rows(K, R);
    constexpr int VP = tv_pitch(), VR = tv_rows(R), WP = fx_pitch(), WR = fx_rows(R);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* sm = reinterpret_cast<T*>(smem_raw);
    const int C = c->C, H = c->H, W = c->W, reg = c->reg;
    const int nw = reg == 1 ? C : 1;
    const int64_t HW = (int64_t)H * W;
    const int ntx = (W + kTW - 1) / kTW, nty = (H + TH - 1) / TH;
    const int tile = xcd_tile(blockIdx.x, ntx * nty);
    const int ti0 = (tile / ntx) * TH, tj0 = (tile % ntx) * kTW;
    const int tx = threadIdx.x & 63, li0 = (threadIdx.x >> 6) * R;
    const int gj = tj0 + tx;
    const T alpha = (T)c->alpha;
    const T* __restrict__ P = b.P[c->pc ^ 1];

    T* s_x = sm;
    T* s_p = sm + C * VR * VP;
    T* s_w = sm + 2 * C * VR * VP;
    T* s_mw = s_w + nw * WR * WP;
    for (int ch = 0; ch < C; ++ch) {
        const T* xc = b.xt + ch * HW;
        const T* pc = P + ch * HW;
        load_tile<VR, VP, VP>(s_x + ch * VR * VP, ti0 - 1, tj0 - 1, H, W, [&](int64_t g) { return xc[g]; });
        load_tile<VR, VP, VP>(s_p + ch * VR * VP, ti0 - 1, tj0 - 1, H, W, [&](int64_t g) { return pc[g]; });
    }
    __syncthreads();
    const T eps2 = (T)(c->eps_tv * c->eps_tv);
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
        const T* kc = b.Kp + ch * HW;
        __syncthreads();
        load_tile<CR, CP, CP>(sm, ti0 - c0, tj0 - c0, H, W, [&](int64_t g) { return kc[g]; });
        __syncthreads();
        T acc[R];
#pragma unroll
        for (int o = 0; o < R; ++o) acc[o] = T(0);
        correlate<T, K, R>(sm, CP, b.th, li0, tx, acc);
#pragma unroll
        for (int o = 0; o < R; ++o) {
            const int gi = ti0 + li0 + o;
            if (gi < H && gj < W) {
                const int64_t e = ch * HW + (int64_t)gi * W + gj;
                const T hp = dfma(alpha, pick3<T, R>(hv0, hv1, hv2, ch, o), acc[o]);
                b.Hp[e] = hp;
                kap += (double)pick3<T, R>(pp0, pp1, pp2, ch, o) * (double)hp;
            }
        }
    }
    if (init) return;
    __shared__ double tot[1];
    const double v[1] = {kap};
    if (grid_reduce<1>(v, b.partials, b.counter, tot) && threadIdx.x == 0) {
        const double kappa = tot[0];
        c->kappa = kappa;
        if (!(kappa > 0.0) || !(kappa <= 1.0e300)) {
            c->cg_done = 1;
            c->cg_status = (kappa <= 1.0e300) ? ST_NOT_SPD : ST_NONFINITE;
        } else {
            c->cg_a = c->gamma / kappa;
        }
    }
}

// Pass 3: q += a p, r -= a Hp, gamma+ = ||r||^2; the last block forms
// beta = gamma+/gamma and applies the stop test sqrt(gamma) <= tol.
template <typename T>
__global__ __launch_bounds__(kNT) void k_cg_update(DevCtx* __restrict__ c, CgBufs<T> b, int64_t n) {
    if (c->cg_done) return;
    const T a = (T)c->cg_a;
    const T* __restrict__ P = b.P[c->pc ^ 1];
    double rs = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * kNT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kNT) {
        const T pv = P[e];
        b.q[e] = dfma(a, pv, b.q[e]);
        const T rv = dfma(-a, b.Hp[e], b.r[e]);
        b.r[e] = rv;
        rs += (double)rv * (double)rv;
    }
    __shared__ double tot[1];
    const double v[1] = {rs};
    if (grid_reduce<1>(v, b.partials, b.counter, tot) && threadIdx.x == 0) {
        const double g = tot[0];
        c->cg_iters += 1;
        c->pc ^= 1;
        if (!(g <= 1.0e300)) {
            c->cg_done = 1;
            c->cg_status = ST_NONFINITE;
            return;
        }
        c->cg_b = g / c->gamma;
        c->gamma = g;
        if (sqrt(g) <= c->cg_tol) {
            c->cg_done = 1;
            c->cg_status = ST_OK;
        } else if (c->cg_iters >= c->cg_max) {
            c->cg_done = 1;
            c->cg_status = ST_MAXITER;
        }
    }
}

// r = b - H q0 (Hp holds H q0), gamma = ||r||^2, initial stop test.
template <typename T>
__global__ __launch_bounds__(kNT) void k_cg_init(DevCtx* __restrict__ c, CgBufs<T> b, int64_t n) {
    double rs = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * kNT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kNT) {
        const T rv = b.b[e] - b.Hp[e];
        b.r[e] = rv;
        rs += (double)rv * (double)rv;
    }
    __shared__ double tot[1];
    const double v[1] = {rs};
    if (grid_reduce<1>(v, b.partials, b.counter, tot) && threadIdx.x == 0) {
        const double g = tot[0];
        c->gamma = g;
        c->cg_b = 0.0;
        c->cg_iters = 0;
        if (!(g <= 1.0e300)) {
            c->cg_done = 1;
            c->cg_status = ST_NONFINITE;
        } else if (sqrt(g) <= c->cg_tol) {
            c->cg_done = 1;
            c->cg_status = ST_OK;
        } else if (c->cg_max <= 0) {
            c->cg_done = 1;
            c->cg_status = ST_MAXITER;
        }
    }
}

// ------------------------------------------------------------------ small kernels
// theta (double, KxK) -> compute type, plain and flipped; optionally its
// l1 norm squared into c->L when c->L <= 0 (starting Lipschitz estimate).
template <typename T>
__global__ __launch_bounds__(1024) void k_prep_kernel(DevCtx* __restrict__ c, const double* __restrict__ th, T* __restrict__ out, T* __restrict__ outf,
                              int K, int set_L, int red_slot) {
    __shared__ double s_abs[1024];
    const int KK = K * K;
    const int t = threadIdx.x;
    double a = 0.0;
    if (t < KK) {
        const int u = t / K, v = t - u * K;
        const double w = th[t];
        // column-major: out(u,v) at v*K+u; the flipped kernel f(u',v') = theta(K-1-u', K-1-v')
        out[v * K + u] = (T)w;
        outf[(K - 1 - v) * K + (K - 1 - u)] = (T)w;
        a = fabs(w);
    }
    s_abs[t] = a;
    __syncthreads();
    if (t == 0) {
        double s = 0.0;
        for (int i = 0; i < KK; ++i) s += s_abs[i];
        if (set_L && !(c->L > 0.0)) c->L = s * s;
        if (red_slot >= 0) c->red[red_slot] = s;
    }
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

// z = -sum_blocks Z + with_r * grad r(theta); ||z||^2 into c->red[slot].
template <int KT>
__global__ __launch_bounds__(1024) void k_hg_final(DevCtx* __restrict__ c, const double* __restrict__ part, int nblk, int K, const double* __restrict__ th,
                           const double* __restrict__ a, int with_r, double* __restrict__ z, int slot) {
    __shared__ double s_e[1024];
    __shared__ double s_z[1024];
    const int t = threadIdx.x, KK = K * K;
    if (t < KK) s_e[t] = (with_r && a) ? th[t] - a[t] : 0.0;
    __syncthreads();
    double zz = 0.0;
    if (t < KK) {
        const int u = t / K, v = t - u * K;
        double s = 0.0;
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
            gr = 2.0 * c->beta * (c->h1_w0 * e + lap);
        }
        zz = -s + gr;
        z[t] = zz;
    }
    s_z[t] = zz * zz;
    __syncthreads();
    if (t == 0) {
        double s = 0.0;
        for (int i = 0; i < KK; ++i) s += s_z[i];
        c->red[slot] = s;
    }
}

}  // namespace maid
