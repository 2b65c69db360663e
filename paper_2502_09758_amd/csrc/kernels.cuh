// kernels.cuh -- gfx950 kernels of libmaid (templated on storage type T,
// kernel size K and rows per thread R).
//
// Layout: images are planar [C][H][W]; a block of 256 threads (four wave64s)
// owns a 64-wide, 4R-tall tile of output pixels of one channel (the TV terms,
// which couple the channels, stage every channel's small halo tile).  Lane tx
// of wave wy computes the R pixels in rows wy*R .. wy*R+R-1 of column tx.
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
// The total is needed only after the pass has staged its own inputs, so the
// partial loads are issued first and summed after the tile loads: the two
// latencies overlap.  A pass whose decision may discard its work (a
// rejected trial step) computes speculatively and gates only its stores.
//
// Every pass serves a batch: block b belongs to instance blk[b] of the
// instance table (a plain solve is a batch of one; a launch over a single
// instance passes its index as `only` and skips the map); the instance's
// blocks start at a multiple of 8 so that the XCD-major tile order holds
// within each instance.  Solver states are arrays over instances, read
// through one copy and written by the instance's block 0 into the next.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "devctx.h"
#include "mfconv.cuh"

namespace maid {

// ------------------------------------------------------------------ helpers
template <typename T> __device__ __forceinline__ T dfma(T a, T b, T c);
template <> __device__ __forceinline__ float dfma<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <> __device__ __forceinline__ double dfma<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T> __device__ __forceinline__ T dsqrt(T v);
template <> __device__ __forceinline__ float dsqrt<float>(float v) { return sqrtf(v); }
template <> __device__ __forceinline__ double dsqrt<double>(double v) { return sqrt(v); }
// 1/sqrt: the hardware reciprocal square root for FP32 (1 ulp), the
// correctly rounded quotient for FP64
// c ? v : 0 with v evaluated whatever c is: where v reads LDS at addresses
// that lie inside the tile for every lane, the reads are then issued
// together instead of each under a branch of its own.
template <typename T> __device__ __forceinline__ T keep(bool c, T v) { return c ? v : T(0); }

template <typename T> __device__ __forceinline__ T drsqrt(T v);
template <> __device__ __forceinline__ float drsqrt<float>(float v) { return rsqrtf(v); }
template <> __device__ __forceinline__ double drsqrt<double>(double v) { return 1.0 / sqrt(v); }

// Element i of a channel plane: the byte offset is formed in 32 bits (a
// plane holds < 4 GiB), so global loads and stores take the uniform 64-bit
// plane base in SGPRs plus a 32-bit VGPR offset.
template <typename T> __device__ __forceinline__ T& at(T* p, unsigned i) {
    return *reinterpret_cast<T*>(reinterpret_cast<char*>(p) + (size_t)(i * (unsigned)sizeof(T)));
}
template <typename T> __device__ __forceinline__ const T& at(const T* p, unsigned i) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + (size_t)(i * (unsigned)sizeof(T)));
}
// Load of element i under a load policy: CO = false is a plain load; CO =
// true (the team loops, where the data were written by other blocks of the
// same XCD during the kernel) is a relaxed device-scope atomic load, which
// misses in the CU's L1 and so reads what the writers left in the XCD's L2.
template <bool CO, typename T> __device__ __forceinline__ T ld(const T* p, unsigned i) {
    if constexpr (CO) return __hip_atomic_load(&at(p, i), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return at(p, i);
}

template <bool CO, typename T> __device__ __forceinline__ T ld64(const T* p, int64_t e) {
    if constexpr (CO) return __hip_atomic_load(p + e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return p[e];
}

// blockIdx -> tile id, XCD-major: the hardware hands block b to XCD b % 8;
// this bijection gives every XCD a contiguous run of tile ids.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int q = nb >> 3, r = nb & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// A lane permutation of a double through the DPP crossbar (two 32-bit
// moves; CTRL is a pattern in which every lane reads an active lane).
template <int CTRL> __device__ __forceinline__ double dpp_f64(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, true);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over the wave (all 64 lanes active), the same value in every lane:
// butterflies within each row of 16 lanes on the DPP crossbar (partners
// lane^1 and lane^2, then the half-row and the row mirror, each of which
// pairs two lanes holding sums over disjoint lane sets, so both partners
// form the same sum), then the four row sums in a fixed order.  The lane
// crossbar takes a few cycles per step where a shuffle through the LDS
// unit takes a round trip.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);  // row_half_mirror
    v += dpp_f64<0x140>(v);  // row_mirror
    return ((readlane_f64(v, 0) + readlane_f64(v, 16)) + readlane_f64(v, 32)) + readlane_f64(v, 48);
}

// Sum of one double per thread over the block, returned to every thread
// (wave sums, then the four waves in a fixed order).
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double s_w[4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) s_w[wid] = v;
    __syncthreads();
    return ((s_w[0] + s_w[1]) + s_w[2]) + s_w[3];
}
// Two such sums with one pair of barriers, for blocks of NW waves (the wave
// sums added in wave order).
template <int NW = 4> __device__ __forceinline__ void block_sum2(double& a, double& b) {
    __shared__ double s_w2[2 * NW];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    a = wave_sum(a);
    b = wave_sum(b);
    __syncthreads();
    if (lane == 0) {
        s_w2[wid] = a;
        s_w2[NW + wid] = b;
    }
    __syncthreads();
    a = s_w2[0];
    b = s_w2[NW];
#pragma unroll
    for (int w = 1; w < NW; ++w) {
        a += s_w2[w];
        b += s_w2[NW + w];
    }
}

// Two grid-wide sums at the consumer, for blocks of any number of waves:
// wave 0 alone has loaded and added the partials (lane l those at l, l + 64,
// ..., with partials_issue / partials_local at 64 threads) and passes a, b
// here; the wave sums go to every thread through LDS (one barrier).
__device__ __forceinline__ void wave0_share2(double& a, double& b) {
    __shared__ double s_sh[2];
    if ((threadIdx.x >> 6) == 0) {
        a = wave_sum(a);
        b = wave_sum(b);
        if (threadIdx.x == 0) {
            s_sh[0] = a;
            s_sh[1] = b;
        }
    }
    __syncthreads();
    a = s_sh[0];
    b = s_sh[1];
}
// Two partials of a block of NW waves; only thread 0 needs the totals (it
// stores them), so one barrier: the wave sums meet in LDS and thread 0 adds
// them in wave order.
template <int NW>
__device__ __forceinline__ void block_partial2_1(double va, double* pa, double vb, double* pb, int lb) {
    __shared__ double s_p2[2 * NW];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    va = wave_sum(va);
    vb = wave_sum(vb);
    if (lane == 0) {
        s_p2[wid] = va;
        s_p2[NW + wid] = vb;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = s_p2[0], b = s_p2[NW];
#pragma unroll
        for (int w = 1; w < NW; ++w) {
            a += s_p2[w];
            b += s_p2[NW + w];
        }
        pa[lb] = a;
        pb[lb] = b;
    }
}

// Producer side of a grid-wide sum: one partial per block (index lb within
// its instance), plain store.
__device__ __forceinline__ void block_partial(double v, double* part, int lb) {
    const double s = block_sum(v);
    if (threadIdx.x == 0) part[lb] = s;
}
// Two partials of the same block.
template <int NW = 4>
__device__ __forceinline__ void block_partial2(double va, double* pa, double vb, double* pb, int lb) {
    block_sum2<NW>(va, vb);
    if (threadIdx.x == 0) {
        pa[lb] = va;
        pb[lb] = vb;
    }
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

// The same sum in two steps: partials_issue loads the thread's first four
// partials into registers (the loads stay in flight while the caller stages
// its tiles), partials_finish adds them and any further ones in the same
// order as reduce_partials and sums over the block.
struct Partials {
    double v[4];
};
template <bool CO = false, int NT = kNT>
__device__ __forceinline__ Partials partials_issue(const double* __restrict__ part, int nb) {
    Partials p;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int b = threadIdx.x + k * NT;
        p.v[k] = b < nb ? ld<CO>(part, b) : 0.0;
    }
    return p;
}
// The thread's share of partials_finish (before the sum over the block).
template <bool CO = false, int NT = kNT>
__device__ __forceinline__ double partials_local(const double* __restrict__ part, int nb, const Partials& p) {
    double s = ((p.v[0] + p.v[1]) + p.v[2]) + p.v[3];
    for (int b = threadIdx.x + 4 * NT; b < nb; b += NT) s += ld<CO>(part, b);
    return s;
}
template <bool CO = false>
__device__ __forceinline__ double partials_finish(const double* __restrict__ part, int nb, const Partials& p) {
    return block_sum(partials_local<CO>(part, nb, p));
}

__device__ __forceinline__ bool finite_d(double v) { return v == v && v <= 1.0e300 && v >= -1.0e300; }

// Field-by-field state stores (no whole-struct copy, so the local state stays
// in scalar registers) and select-based buffer picks (no runtime indexing
// into by-value argument arrays, which would go through scratch memory).
__device__ __forceinline__ void put_state(ApgState* __restrict__ o, const ApgState& s) {
    o->L = s.L; o->t = s.t; o->t_prev = s.t_prev; o->m = s.m; o->gn2 = s.gn2; o->tol = s.tol;
    o->delta_last = s.delta_last; o->max_iter = s.max_iter; o->iters = s.iters; o->bt = s.bt;
    o->nb_iter = s.nb_iter; o->status = s.status; o->done = s.done; o->phase = s.phase; o->cur = s.cur;
    o->prev = s.prev; o->nxt = s.nxt; o->trace_cap = s.trace_cap; o->resync = s.resync;
    o->resync_full = s.resync_full; o->pp = s.pp; o->fixed = s.fixed;
}
__device__ __forceinline__ void put_state(CgState* __restrict__ o, const CgState& s) {
    o->gamma = s.gamma; o->kappa = s.kappa; o->a = s.a; o->tol = s.tol; o->max = s.max; o->iters = s.iters;
    o->status = s.status; o->done = s.done; o->pc = s.pc; o->first = s.first;
}
template <typename P>
__device__ __forceinline__ P pick(P a0, P a1, P a2, int i) { return i == 0 ? a0 : (i == 1 ? a1 : a2); }
template <typename P>
__device__ __forceinline__ P pick(P a0, P a1, int i) { return i == 0 ? a0 : a1; }

// inside [0,H) x [0,W), with one unsigned compare per axis
__device__ __forceinline__ bool inside(int gi, int gj, int H, int W) { return (unsigned)gi < (unsigned)H && (unsigned)gj < (unsigned)W; }
__device__ __forceinline__ int clampi(int v, int hi) { return v < 0 ? 0 : (v > hi ? hi : v); }

// Stage f(global flat index) into an LDS tile s[ROWS][PITCH] covering rows
// gi0.., columns gj0..; zero outside [0,H) x [0,W).  Each thread issues the
// global loads of up to eight of its elements before it writes any of them
// to LDS, so their latencies overlap instead of adding up.
template <int ROWS, int COLS, int PITCH, int NT = kNT, typename T, typename F>
__device__ __forceinline__ void load_tile(T* s, int gi0, int gj0, int H, int W, F f) {
    constexpr int NE = ROWS * COLS, IT = (NE + NT - 1) / NT, B = IT < 8 ? IT : 8;
#pragma unroll 1
    for (int k0 = 0; k0 < IT; k0 += B) {
        T val[B];
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int idx = threadIdx.x + (k0 + k) * NT;
            const int r = idx / COLS, cc = idx - r * COLS;
            const int gi = gi0 + r, gj = gj0 + cc;
            // every lane loads from a valid (clamped) address and zeroes what
            // lies outside afterwards: no branch around the loads, so all of
            // them are in flight before the first is used
            const T v = f(clampi(gi, H - 1) * W + clampi(gj, W - 1));
            val[k] = (idx < NE && inside(gi, gj, H, W)) ? v : T(0);
        }
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int idx = threadIdx.x + (k0 + k) * NT;
            const int r = idx / COLS, cc = idx - r * COLS;
            if (idx < NE) s[r * PITCH + cc] = val[k];
        }
    }
}

// acc[o] += sum_{u,v} ker(u,v) * s[li0+o+u][tx+v]  (a KxK correlation of
// the staged tile; with the flipped kernel it is the true convolution).
// Taps are stored column-major, kT[v*K + u] = ker(u,v), so the K taps of one
// column arrive in a few wide scalar loads.  The column loop stays rolled
// for large K to bound register pressure (R+K-1 staged values, R
// accumulators, K taps in SGPRs per iteration).
// The taps are read through the constant address space: they are uniform and
// nothing in the kernel writes them, so they arrive by scalar loads.
#if defined(__HIP_DEVICE_COMPILE__)
#define MAID_CONST __attribute__((address_space(4)))
#else
#define MAID_CONST
#endif
// Warms the scalar cache with the lines of two tap arrays (K*K taps each):
// scalar loads of one word per 64-byte line, folded into one value that only
// an empty asm statement consumes (so all loads are issued before the one
// wait).  Called while a pass's global loads are in flight, it takes the
// taps' memory latency off the correlations, whose scalar loads of the taps
// then hit the cache.
template <typename T, int K> __device__ __forceinline__ void warm_taps(const T* ka, const T* kb) {
#if defined(__HIP_DEVICE_COMPILE__)
    using U = unsigned;
    const U MAID_CONST* a = (const U MAID_CONST*)ka;
    const U MAID_CONST* b = (const U MAID_CONST*)kb;
    constexpr int NW = K * K * (int)(sizeof(T) / sizeof(U)), L = 16;
    U x = a[NW - 1] ^ b[NW - 1];
#pragma unroll
    for (int i = 0; i < NW - 1; i += L) x ^= a[i] ^ b[i];
    asm volatile("" ::"s"(x));
#endif
}

template <typename T, int K, int R>
__device__ __forceinline__ void correlate_col(const T* s, int pitch, const T* __restrict__ kT, int li0, int tx, int v, T (&acc)[R]) {
    const T MAID_CONST* kc = (const T MAID_CONST*)kT;
    T col[R + K - 1];
#pragma unroll
    for (int t = 0; t < R + K - 1; ++t) col[t] = s[(li0 + t) * pitch + tx + v];
#pragma unroll
    for (int u = 0; u < K; ++u) {
        const T w = kc[v * K + u];
#pragma unroll
        for (int o = 0; o < R; ++o) acc[o] = dfma(w, col[o + u], acc[o]);
    }
}

// Small kernels with short columns unroll the column loop too, so that the
// LDS reads of the next columns are in flight during this column's FMAs (a
// pass of a small image has few waves per SIMD to hide that latency).  Tiles
// of 8 rows per thread unroll it only up to K = 5: at K = 7 and 9 the
// unrolled loop held 136-168 VGPRs (3 waves per SIMD, and the trial pass
// spilled at K = 9) and ran slower than the rolled K = 11 one.
template <typename T, int K, int R> __host__ __device__ constexpr bool corr_unrolled() {
    return K <= 5 || (R <= 4 && K <= 11 && K * (R + K - 1) <= (sizeof(T) == 4 ? 160 : 96));
}

template <typename T, int K, int R>
__device__ __forceinline__ void correlate(const T* s, int pitch, const T* __restrict__ kT, int li0, int tx, T (&acc)[R]) {
    if constexpr (corr_unrolled<T, K, R>()) {
#pragma unroll
        for (int v = 0; v < K; ++v) correlate_col<T, K, R>(s, pitch, kT, li0, tx, v, acc);
    } else {
#pragma unroll 1
        for (int v = 0; v < K; ++v) correlate_col<T, K, R>(s, pitch, kT, li0, tx, v, acc);
    }
}

// The correlation of a staged tile on the matrix cores where the tile shape
// allows it and the instance carries the kernel's operand layout (mf,
// nullable), else on the vector ALUs.  Every thread of the block calls it.
// MF = false leaves the matrix-core path out of the kernel (the team loops,
// which serve instances too small to need it).
// kp: the kernel plane (0 for a kernel shared by the channels, the image
// channel for per-channel kernels): taps kT + kp K^2, operand layouts
// mf + kp (the size of one kernel's), exponent mfsh[kp].
// On the matrix cores the staged tile s is overwritten (its LDS region of
// lds_conv(K, R, sizeof(T)) elements is the correlation's work space):
// callers read what they need of the tile before the call.
template <typename T, int K, int R, bool MF = true>
__device__ __forceinline__ void correlate_sel(T* s, int pitch, const T* __restrict__ kT, const uint4* mf,
                                              const int* mfsh, int kp, int li0, int tx, T (&acc)[R]) {
    if constexpr (MF && mf_ok<T, K, R>()) {
        if (mf) {
            correlate_mfma<K, R>(s, pitch, mf + kp * (mf_frag_bytes(K) / 16), *(const int MAID_CONST*)(mfsh + kp),
                                 li0, tx, acc);
            return;
        }
    }
    correlate<T, K, R>(s, pitch, kT + kp * K * K, li0, tx, acc);
}

// The kernel plane of image channel ch: per-channel kernels (kc > 1) hold
// one KxK plane per channel, a shared kernel one plane.
template <typename T> __device__ __forceinline__ int kplane(const Inst<T>& I, int ch) { return I.kc > 1 ? ch : 0; }

// acc[o] += sum_{u,v} ker(u,v) s[(li0+o+u) pitch + tx+v] in FP64, the taps
// read as doubles from the row-major KxK array th: ker(u,v) = th[u K + v],
// or th[(K-1-u) K + (K-1-v)] with `flip`.  Both tap loops stay rolled and
// the staged values are read per tap (few registers: the solver passes
// call it rarely, next to register-hungry code).
template <typename T, int K, int R>
__device__ __forceinline__ void correlate64(const T* s, int pitch, const double* __restrict__ th, bool flip, int li0,
                                            int tx, double (&acc)[R]) {
    const double MAID_CONST* kc = (const double MAID_CONST*)th;
#pragma unroll 1
    for (int u = 0; u < K; ++u) {
#pragma unroll 1
        for (int v = 0; v < K; ++v) {
            const double w = kc[flip ? (K - 1 - u) * K + (K - 1 - v) : u * K + v];
            const T* col = s + (li0 + u) * pitch + tx + v;
#pragma unroll
            for (int o = 0; o < R; ++o) acc[o] = __builtin_fma(w, (double)col[o * pitch], acc[o]);
        }
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
// TH: rows of the tile the weights serve (flux sites of TH + 1 rows from a
// v tile of TH + 2 rows); NT: threads of the block.
template <typename T, int TH, int NT>
__device__ __forceinline__ void tv_weights_h(const T* s_v, T* s_w, int C, int reg, T eps2, int ti0, int tj0, int H, int W) {
    constexpr int VP = tv_pitch(), VR = TH + 2, WP = fx_pitch(), WR = TH + 1;
    constexpr int NS = WR * WP, IT = (NS + NT - 1) / NT;
    if (reg == 1 && C > 1) {
        // channelwise weights, one set per channel
        for (int idx = threadIdx.x; idx < NS; idx += NT) {
            const int r = idx / WP, cc = idx - r * WP;
            const int gi = ti0 - 1 + r, gj = tj0 - 1 + cc;
            const bool in = (gi >= 0 && gi < H && gj >= 0 && gj < W);
            const bool hx = gj < W - 1, vx = gi < H - 1;
            for (int ch = 0; ch < C; ++ch) {
                const T* V = s_v + ch * VR * VP;
                const T v0 = V[r * VP + cc];
                const T dh = keep(hx, V[r * VP + cc + 1] - v0);
                const T dv = keep(vx, V[(r + 1) * VP + cc] - v0);
                s_w[ch * WR * WP + idx] = in ? drsqrt(dh * dh + dv * dv + eps2) : T(0);
            }
        }
        return;
    }
    // one weight per site (coupled channels; with one channel the
    // channelwise weight is the same number): the thread's sites unrolled,
    // all reads (at a clamped site index) before all stores, so that no LDS
    // read waits behind an LDS store the compiler cannot tell apart from it
    T wk[IT];
#pragma unroll
    for (int k = 0; k < IT; ++k) {
        const int idx = threadIdx.x + k * NT;
        const int ic = idx < NS ? idx : NS - 1;
        const int r = ic / WP, cc = ic - r * WP;
        const int gi = ti0 - 1 + r, gj = tj0 - 1 + cc;
        const bool in = (gi >= 0 && gi < H && gj >= 0 && gj < W);
        const bool hx = gj < W - 1, vx = gi < H - 1;
        T s2 = T(0);
        for (int ch = 0; ch < C; ++ch) {
            const T* V = s_v + ch * VR * VP;
            const T v0 = V[r * VP + cc];
            const T dh = keep(hx, V[r * VP + cc + 1] - v0);
            const T dv = keep(vx, V[(r + 1) * VP + cc] - v0);
            s2 += dh * dh + dv * dv;
        }
        wk[k] = in ? (reg == 2 ? T(1) : drsqrt(s2 + eps2)) : T(0);
    }
#pragma unroll
    for (int k = 0; k < IT; ++k) {
        const int idx = threadIdx.x + k * NT;
        if (idx < NS) s_w[idx] = wk[k];
    }
}
template <typename T, int R>
__device__ __forceinline__ void tv_weights(const T* s_v, T* s_w, int C, int reg, T eps2, int ti0, int tj0, int H, int W) {
    tv_weights_h<T, tile_h(R), kNT>(s_v, s_w, C, reg, eps2, ti0, tj0, H, W);
}

// grad R at the thread's pixel (li, tx) of channel ch:
// fh(i,j-1) - fh(i,j) + fv(i-1,j) - fv(i,j), flux f = w * (forward difference)
template <typename T, int TH>
__device__ __forceinline__ T tv_grad_px_h(const T* s_v, const T* s_w, int ch, int reg, int li, int tx, int gi, int gj, int H, int W) {
    constexpr int VP = tv_pitch(), VR = TH + 2, WP = fx_pitch(), WR = TH + 1;
    const T* V = s_v + ch * VR * VP;
    const T* Wt = s_w + (reg == 1 ? ch * WR * WP : 0);
    const int r = li + 1, cc = tx + 1;
    const T v0 = V[r * VP + cc];
    const T dh_here = keep(gj < W - 1, V[r * VP + cc + 1] - v0);
    const T dv_here = keep(gi < H - 1, V[(r + 1) * VP + cc] - v0);
    const T dh_left = v0 - V[r * VP + cc - 1];
    const T dv_up = v0 - V[(r - 1) * VP + cc];
    const T w0 = Wt[r * WP + cc];
    return Wt[r * WP + cc - 1] * dh_left - w0 * dh_here + Wt[(r - 1) * WP + cc] * dv_up - w0 * dv_here;
}
template <typename T, int R>
__device__ __forceinline__ T tv_grad_px(const T* s_v, const T* s_w, int ch, int reg, int li, int tx, int gi, int gj, int H, int W) {
    return tv_grad_px_h<T, tile_h(R)>(s_v, s_w, ch, reg, li, tx, gi, gj, H, W);
}

// Occupancy floor (waves per SIMD) the compiler must keep for the
// large-kernel passes with tall tiles (FP32 storage only; the FP64
// instantiations keep the compiler's choice).  With the matrix-core
// correlation's LDS these passes hold 2-4 blocks per CU, so a higher floor
// would only cap their registers (and made the trial pass spill).
template <typename T> __host__ __device__ constexpr int min_waves(int K, int R) {
    return sizeof(T) == 4 && seq_lds(K) && R >= 4 ? (R == 8 ? 3 : 4) : 1;
}

// Several tiles staged together: every tile's global loads are issued (held
// in registers) before any of them is written to LDS, so a pass that needs a
// few small tiles pays one memory latency instead of one per tile.
template <int ROWS, int COLS, int PITCH, typename T, typename F, int NT = kNT>
struct Stage {
    static constexpr int NE = ROWS * COLS, IT = (NE + NT - 1) / NT;
    T* s;
    int gi0, gj0;
    F f;
    T val[IT];
    __device__ __forceinline__ void fetch(int H, int W) {
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const int idx = threadIdx.x + k * NT;
            const int r = idx / COLS, cc = idx - r * COLS;
            const int gi = gi0 + r, gj = gj0 + cc;
            // every lane loads from a valid (clamped) address and zeroes what
            // lies outside afterwards: no branch around the loads, so all of
            // them are in flight before the first is used
            const T v = f(clampi(gi, H - 1) * W + clampi(gj, W - 1));
            val[k] = (idx < NE && inside(gi, gj, H, W)) ? v : T(0);
        }
    }
    __device__ __forceinline__ void put() const {
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const int idx = threadIdx.x + k * NT;
            const int r = idx / COLS, cc = idx - r * COLS;
            if (idx < NE) s[r * PITCH + cc] = val[k];
        }
    }
};
template <int ROWS, int COLS, int PITCH, int NT = kNT, typename T, typename F>
__device__ __forceinline__ Stage<ROWS, COLS, PITCH, T, F, NT> stage(T* s, int gi0, int gj0, F f) {
    return Stage<ROWS, COLS, PITCH, T, F, NT>{s, gi0, gj0, f, {}};
}

// ------------------------------------------------------------------ instance lookup
// Block -> (instance, local block).  Padding blocks (lb >= nb) return at once,
// and so would a block below its instance's range (one unsigned compare).
#define MAID_STENCIL_PROLOGUE                                         \
    const int ii = only >= 0 ? only : blk[blockIdx.x];                \
    const Inst<T>& I = insts[ii];                                     \
    const int lb = (int)blockIdx.x - I.base;                          \
    if ((unsigned)lb >= (unsigned)I.nb) return;

#define MAID_EW_PROLOGUE                                              \
    const int ii = only >= 0 ? only : blk[blockIdx.x];                \
    const Inst<T>& I = insts[ii];                                     \
    const int lb = (int)blockIdx.x - I.base_e;                        \
    if ((unsigned)lb >= (unsigned)I.nbe) return;

// Local block -> tile origin and channel.  The C channel blocks of one tile
// are adjacent in the XCD-major order (they share halo loads in L2).
template <int R>
__device__ __forceinline__ void tile_pos(const Params& pr, int lb, int nb, int& ti0, int& tj0, int& ch) {
    const int t = xcd_tile(lb, nb);
    const int tile = t / pr.C;
    ch = t - tile * pr.C;
    const int ntx = (pr.W + kTW - 1) / kTW;
    ti0 = (tile / ntx) * tile_h(R);
    tj0 = (tile % ntx) * kTW;
}

// ------------------------------------------------------------------ generic convolution pass
// cv_out = cv_ker (x) cv_in  [- cv_sub]   (correlation with cv_ker; the
// flipped kernel gives the true convolution); with cv_part, per-block
// partials of sum cv_out^2; optionally a second copy of the result and up to
// two copies of the input (the set-up of a solve).  Instances without cv_out
// take no part.
template <typename T, int K, int R>
__global__ __launch_bounds__(kNT) void k_conv(const Inst<T>* __restrict__ insts, const int* __restrict__ blk, int only) {
    MAID_STENCIL_PROLOGUE
    if (!I.cv_out) return;
    if (I.cv_prev_part && lb == 0) {
        const double t = reduce_partials(I.cv_prev_part, I.nb);
        if (threadIdx.x == 0) I.red[I.cv_prev_slot] = t;
    }
    constexpr int c0 = (K - 1) / 2, CP = cv_pitch(K), CR = cv_rows(K, R);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* s = reinterpret_cast<T*>(smem_raw);
    const int H = I.pr.H, W = I.pr.W;
    const int64_t HW = (int64_t)H * W;
    int ti0, tj0, ch;
    tile_pos<R>(I.pr, lb, I.nb, ti0, tj0, ch);
    const int tx = threadIdx.x & 63, li0 = (threadIdx.x >> 6) * R;
    const T* __restrict__ src = I.cv_in + ch * HW;
    // channel planes (64-bit base once per block; 32-bit offsets inside)
    const T* __restrict__ sub = I.cv_sub ? I.cv_sub + ch * HW : nullptr;
    T* __restrict__ out = I.cv_out + ch * HW;
    T* __restrict__ out2 = I.cv_out2 ? I.cv_out2 + ch * HW : nullptr;
    T* __restrict__ out3 = I.cv_out3 ? I.cv_out3 + ch * HW : nullptr;
    T* __restrict__ cp0 = I.cv_cp[0] ? I.cv_cp[0] + ch * HW : nullptr;
    T* __restrict__ cp1 = I.cv_cp[1] ? I.cv_cp[1] + ch * HW : nullptr;
    T* __restrict__ cp2 = I.cv_cp[2] ? I.cv_cp[2] + ch * HW : nullptr;
    load_tile<CR, CP, CP>(s, ti0 - c0, tj0 - c0, H, W, [&](int g) { return at(src, g); });
    __syncthreads();
    const int gj = tj0 + tx;
    if constexpr (sizeof(T) == 4) {
        if (I.cv_ker64) {
            // FP64 taps and sums; one rounding to the storage type at the
            // store, none where the job keeps the result in FP64 (cv_out64)
            double* __restrict__ out64 = I.cv_out64 ? I.cv_out64 + ch * HW : nullptr;
            double acc[R];
#pragma unroll
            for (int o = 0; o < R; ++o) acc[o] = 0.0;
            correlate64<T, K, R>(s, CP, I.cv_ker64 + kplane(I, ch) * K * K, I.cv_flip64 != 0, li0, tx, acc);
            double sq = 0.0;
#pragma unroll
            for (int o = 0; o < R; ++o) {
                const int gi = ti0 + li0 + o;
                if (gi < H && gj < W) {
                    const int e = gi * W + gj;
                    double val = acc[o];
                    if (sub) val -= (double)at(sub, e);
                    if (out64) {
                        at(out64, e) = val;
                    } else {
                        at(out, e) = (T)val;
                    }
                    if (out2) at(out2, e) = (T)val;
                    if (out3) at(out3, e) = (T)val;
                    if (cp0) {
                        const T xin = s[(li0 + o + c0) * CP + tx + c0];
                        at(cp0, e) = xin;
                        if (cp1) at(cp1, e) = xin;
                        if (cp2) at(cp2, e) = xin;
                    }
                    sq += val * val;
                }
            }
            if (I.cv_part) block_partial(sq, I.cv_part, lb);
            return;
        }
    }
    T acc[R];
#pragma unroll
    for (int o = 0; o < R; ++o) acc[o] = T(0);
    // the tile's centre values (the input copies) are read before the
    // correlation, which may overwrite the tile
    T ctr[R];
#pragma unroll
    for (int o = 0; o < R; ++o) ctr[o] = cp0 ? s[(li0 + o + c0) * CP + tx + c0] : T(0);
    correlate_sel<T, K, R>(s, CP, I.cv_ker, I.cv_mf, I.cv_mfsh, kplane(I, ch), li0, tx, acc);
    double sq = 0.0;
#pragma unroll
    for (int o = 0; o < R; ++o) {
        const int gi = ti0 + li0 + o;
        if (gi < H && gj < W) {
            const int e = gi * W + gj;
            T val = acc[o];
            if (sub) val -= at(sub, e);
            at(out, e) = val;
            if (out2) at(out2, e) = val;
            if (out3) at(out3, e) = val;
            if (cp0) {
                const T xin = ctr[o];
                at(cp0, e) = xin;
                if (cp1) at(cp1, e) = xin;
                if (cp2) at(cp2, e) = xin;
            }
            sq += (double)val * (double)val;
        }
    }
    if (I.cv_part) block_partial(sq, I.cv_part, lb);
}

// ------------------------------------------------------------------ lower level: FISTA
// Gradient pass.  Per instance: reads sin, block 0 writes sout.  After a
// trial pass, the decrease h(x+) - h(v) is finished from the partials and
// decides: accept (rotate buffers, advance the momentum sequence, then
// evaluate the new gradient) or reject (double L, no gradient work).  The
// gradient at v = x + m (x - x_prev), with theta*v = Kx + m (Kx - Kx_prev) by
// linearity, is
//   G = theta . (theta*v - y) + alpha grad R(v),
// and its per-block partials of ||G||^2 go to pA.  The gradient at the point
// an acceptance would move to is computed while the partials are in flight;
// a rejection drops it before any store.
template <typename T, int K, int R, bool CO>
__device__ __forceinline__ void apg_grad_body(const Inst<T>& I, int lb, ApgState& st, ApgState* __restrict__ sout,
                                              bool writer) {
    const bool trialed = st.phase == PH_TRIALED;
    Partials pv;
    if (trialed) pv = partials_issue<CO>(I.pB, I.nb);
    // the point of the next gradient if the trial is accepted (at the start: the current one)
    int cur = st.cur, prev = st.prev;
    double mnext = st.m, tnext = st.t;
    if (trialed) {
        cur = st.nxt;
        prev = st.cur;
        tnext = st.fixed ? 1.0 : 0.5 * (1.0 + sqrt(1.0 + 4.0 * st.t * st.t));
        mnext = st.fixed ? 0.0 : (st.t - 1.0) / tnext;
    }

    constexpr int c0 = (K - 1) / 2, CP = cv_pitch(K), CR = cv_rows(K, R);
    constexpr int VP = tv_pitch(), VR = tv_rows(R), WP = fx_pitch(), WR = fx_rows(R);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* sm = reinterpret_cast<T*>(smem_raw);
    const int C = I.pr.C, H = I.pr.H, W = I.pr.W, reg = I.pr.reg;
    const int nw = reg == 1 ? C : 1;
    const int64_t HW = (int64_t)H * W;
    int ti0, tj0, ch;
    tile_pos<R>(I.pr, lb, I.nb, ti0, tj0, ch);
    const int tx = threadIdx.x & 63, li0 = (threadIdx.x >> 6) * R;
    const int gj = tj0 + tx;
    const T m = (T)mnext;
    const T alpha = (T)I.pr.alpha;
    const T* __restrict__ X = pick(I.X[0], I.X[1], I.X[2], cur);
    const T* __restrict__ XP = pick(I.X[0], I.X[1], I.X[2], prev);
    const T* __restrict__ KX = pick(I.KX[0], I.KX[1], I.KX[2], cur) + ch * HW;
    const T* __restrict__ KXP = pick(I.KX[0], I.KX[1], I.KX[2], prev) + ch * HW;

    // stage v for every channel (the TV magnitude couples them) and the data
    // residual theta*v - y of this block's channel
    constexpr bool SEQ = seq_lds(K);
    T* s_v = sm;
    T* s_w = s_v + C * VR * VP;
    T* s_c = SEQ ? sm : s_w + nw * WR * WP;
    auto stage_residual = [&]() {
        load_tile<CR, CP, CP>(s_c, ti0 - c0, tj0 - c0, H, W, [&](int g) {
            const T kx = ld<CO>(KX, g);
            return dfma(m, kx - ld<CO>(KXP, g), kx);
        });
    };
    auto vfun = [&](int c) {
        const T* Xc = X + c * HW;
        const T* XPc = XP + c * HW;
        return [=](int g) { const T xv = ld<CO>(Xc, g); return dfma(m, xv - ld<CO>(XPc, g), xv); };
    };
    if constexpr (!SEQ) {
        // all of this pass's tiles in one round of loads
        auto v0 = stage<VR, VP, VP>(s_v, ti0 - 1, tj0 - 1, vfun(0));
        auto v1 = stage<VR, VP, VP>(s_v + VR * VP, ti0 - 1, tj0 - 1, vfun(C > 1 ? 1 : 0));
        auto v2 = stage<VR, VP, VP>(s_v + 2 * VR * VP, ti0 - 1, tj0 - 1, vfun(C > 2 ? 2 : 0));
        auto rs = stage<CR, CP, CP>(s_c, ti0 - c0, tj0 - c0, [&](int g) {
            const T kx = ld<CO>(KX, g);
            return dfma(m, kx - ld<CO>(KXP, g), kx);
        });
        v0.fetch(H, W);
        if (C > 1) v1.fetch(H, W);
        if (C > 2) v2.fetch(H, W);
        rs.fetch(H, W);
        v0.put();
        if (C > 1) v1.put();
        if (C > 2) v2.put();
        rs.put();
    } else {
        // every channel's v tile in one round of loads (one memory latency
        // instead of one per channel; the residual tile follows later in the
        // same LDS region)
        auto v0 = stage<VR, VP, VP>(s_v, ti0 - 1, tj0 - 1, vfun(0));
        auto v1 = stage<VR, VP, VP>(s_v + VR * VP, ti0 - 1, tj0 - 1, vfun(C > 1 ? 1 : 0));
        auto v2 = stage<VR, VP, VP>(s_v + 2 * VR * VP, ti0 - 1, tj0 - 1, vfun(C > 2 ? 2 : 0));
        v0.fetch(H, W);
        if (C > 1) v1.fetch(H, W);
        if (C > 2) v2.fetch(H, W);
        v0.put();
        if (C > 1) v1.put();
        if (C > 2) v2.put();
    }
    // the backtracking decision; large kernels take it before their
    // convolution (occupancy first), small ones after it (latency first)
    bool compute = true;
    auto decide = [&]() {
        if (trialed) {
            const double delta = partials_finish<CO>(I.pB, I.nb, pv);
            st.delta_last = delta;
            if (!finite_d(delta)) {
                st.done = 1;
                st.status = ST_NONFINITE;
                compute = false;
            } else if (st.fixed || delta <= -st.gn2 / (2.0 * st.L)) {
                if (writer && I.trace && st.iters < st.trace_cap) I.trace[st.iters] = st.nb_iter;
                st.iters += 1;
                st.nxt = st.prev;
                st.prev = st.cur;
                st.cur = cur;
                st.t_prev = st.t;
                st.t = tnext;
                st.m = mnext;
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
        if (writer && sout) put_state(sout, st);
    };
    __syncthreads();
    if (SEQ) {
        decide();
        if (!compute) return;
    }
    tv_weights<T, R>(s_v, s_w, C, reg, (T)(I.pr.eps_tv * I.pr.eps_tv), ti0, tj0, H, W);
    T acc[R];
#pragma unroll
    for (int o = 0; o < R; ++o) acc[o] = T(0);
    if (!SEQ) correlate<T, K, R>(s_c, CP, I.th + kplane(I, ch) * K * K, li0, tx, acc);
    __syncthreads();
    // SEQ: the TV gradient waits in LDS past the tile region while the
    // convolution tile reuses it (registers stay with the convolution)
    T* s_park = sm + cmax(C * VR * VP + nw * WR * WP, lds_conv(K, R, sizeof(T)));
    T tg[SEQ ? 1 : R];
#pragma unroll
    for (int o = 0; o < R; ++o) {
        const int li = li0 + o, gi = ti0 + li;
        const T g = tv_grad_px<T, R>(s_v, s_w, ch, reg, li, tx, gi, gj, H, W);
        if constexpr (SEQ) s_park[o * kNT + threadIdx.x] = g;
        else tg[o] = g;
    }
    if (SEQ) {
        __syncthreads();
        stage_residual();
        __syncthreads();
        correlate_sel<T, K, R, !CO>(s_c, CP, I.th, I.mf_th, I.mf_sh, kplane(I, ch), li0, tx, acc);
    }
    T gv[R];
#pragma unroll
    for (int o = 0; o < R; ++o) gv[o] = dfma(alpha, SEQ ? s_park[o * kNT + threadIdx.x] : tg[SEQ ? 0 : o], acc[o]);

    if (!SEQ) {
        decide();
        if (!compute) return;
    }
    double gsq = 0.0;
    T* __restrict__ G = I.G + ch * HW;
#pragma unroll
    for (int o = 0; o < R; ++o) {
        const int gi = ti0 + li0 + o;
        if (gi < H && gj < W) {
            at(G, gi * W + gj) = gv[o];
            gsq += (double)gv[o] * (double)gv[o];
        }
    }
    block_partial(gsq, I.pA, lb);
}

template <typename T, int K, int R>
__global__ __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(min_waves<T>(K, R)))) void k_apg_grad(const Inst<T>* __restrict__ insts, const int* __restrict__ blk, int only,
                                                  const ApgState* __restrict__ sin, ApgState* __restrict__ sout) {
    MAID_STENCIL_PROLOGUE
    ApgState st = sin[ii];
    const bool writer = lb == 0 && threadIdx.x == 0;
    if (st.done) {
        if (writer) put_state(&sout[ii], st);
        return;
    }
    apg_grad_body<T, K, R, false>(I, lb, st, &sout[ii], writer);
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
// with every per-element product in double.  The TV part couples the
// channels; each of a tile's channel blocks takes a share of its rows.
// theta*x+ by linearity accumulates the rounding of the x and theta*x
// recurrences (the momentum makes it grow faster than a random walk), so on
// two consecutive iterations of every `resync` it is recomputed exactly as
// the convolution of the stored x+ (two consecutive, so that both theta*x
// and theta*x_prev, i.e. the momentum term, are exact again).
template <typename T, int K, int R, bool CO>
__device__ __forceinline__ void apg_trial_body(const Inst<T>& I, int lb, ApgState& st, ApgState* __restrict__ sout,
                                               bool writer) {
    const bool fresh = st.phase == PH_GRAD_READY;
    Partials pv;
    if (fresh) pv = partials_issue<CO>(I.pA, I.nb);

    constexpr int c0 = (K - 1) / 2, CP = cv_pitch(K), CR = cv_rows(K, R);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* sm = reinterpret_cast<T*>(smem_raw);
    const int C = I.pr.C, H = I.pr.H, W = I.pr.W, reg = I.pr.reg;
    const int64_t HW = (int64_t)H * W;
    int ti0, tj0, ch;
    tile_pos<R>(I.pr, lb, I.nb, ti0, tj0, ch);
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

    constexpr bool SEQ = seq_lds(K);
    constexpr int VP = tv_pitch(), VR = tv_rows(R);
    T* s_c = sm;
    T* s_v = sm + lds_conv(K, R, sizeof(T));   // small kernels: v and dl of every channel, one-pixel halo
    T* s_d = s_v + C * VR * VP;
    const T* Gc = G + ch * HW;
    auto sfun_v = [&](int c) {
        const T* Xc = X + c * HW;
        const T* XPc = XP + c * HW;
        return [=](int g) { const T xv = ld<CO>(Xc, g); return dfma(m, xv - ld<CO>(XPc, g), xv); };
    };
    auto sfun_d = [&](int c) {
        const T* Gcc = G + c * HW;
        return [=](int g) { return ld<CO>(Gcc, g) * ninvL; };
    };
    if constexpr (!SEQ) {
        auto sg = stage<CR, CP, CP>(s_c, ti0 - c0, tj0 - c0, [&](int g) { return ld<CO>(Gc, g) * ninvL; });
        auto v0 = stage<VR, VP, VP>(s_v, ti0 - 1, tj0 - 1, sfun_v(0));
        auto v1 = stage<VR, VP, VP>(s_v + VR * VP, ti0 - 1, tj0 - 1, sfun_v(C > 1 ? 1 : 0));
        auto v2 = stage<VR, VP, VP>(s_v + 2 * VR * VP, ti0 - 1, tj0 - 1, sfun_v(C > 2 ? 2 : 0));
        auto d0 = stage<VR, VP, VP>(s_d, ti0 - 1, tj0 - 1, sfun_d(0));
        auto d1 = stage<VR, VP, VP>(s_d + VR * VP, ti0 - 1, tj0 - 1, sfun_d(C > 1 ? 1 : 0));
        auto d2 = stage<VR, VP, VP>(s_d + 2 * VR * VP, ti0 - 1, tj0 - 1, sfun_d(C > 2 ? 2 : 0));
        sg.fetch(H, W);
        v0.fetch(H, W);
        d0.fetch(H, W);
        if (C > 1) { v1.fetch(H, W); d1.fetch(H, W); }
        if (C > 2) { v2.fetch(H, W); d2.fetch(H, W); }
        sg.put();
        v0.put();
        d0.put();
        if (C > 1) { v1.put(); d1.put(); }
        if (C > 2) { v2.put(); d2.put(); }
    } else {
        load_tile<CR, CP, CP>(s_c, ti0 - c0, tj0 - c0, H, W, [&](int g) { return ld<CO>(Gc, g) * ninvL; });
    }
    __syncthreads();

    bool trial = true;
    if (fresh) {
        const double gn2 = partials_finish<CO>(I.pA, I.nb, pv);
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
    if (writer && sout) put_state(sout, st);
    if (!trial) return;

    // ---- TV part of the decrease, per site: the tile's rows are dealt to its
    // channel blocks in turn; v and dl come from LDS (small kernels) or from
    // global memory (L1/L2; large kernels keep their LDS for the convolution)
    const double e2 = I.pr.eps_tv * I.pr.eps_tv;
    double dtv = 0.0;
    auto tv_site = [&](double bh, double bv, double ah, double av, double& ds2, double& s2) {
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
    };
    if constexpr (!SEQ) {
#pragma unroll
        for (int o = 0; o < R; ++o) {
            const int li = li0 + o, gi = ti0 + li;
            if (li % C == ch && gi < H && gj < W) {
                const int idx = (li + 1) * VP + tx + 1;
                const bool hx = gj < W - 1, vx = gi < H - 1;
                double ds2 = 0.0, s2 = 0.0;
                for (int c = 0; c < C; ++c) {
                    const T* V = s_v + c * VR * VP;
                    const T* D = s_d + c * VR * VP;
                    const double bh = hx ? (double)(V[idx + 1] - V[idx]) : 0.0;
                    const double bv = vx ? (double)(V[idx + VP] - V[idx]) : 0.0;
                    const double ah = hx ? (double)(D[idx + 1] - D[idx]) : 0.0;
                    const double av = vx ? (double)(D[idx + VP] - D[idx]) : 0.0;
                    tv_site(bh, bv, ah, av, ds2, s2);
                }
                if (reg == 2) dtv += ds2;
                else if (reg == 0) dtv += ds2 / (sqrt(s2 + ds2 + e2) + sqrt(s2 + e2));
            }
        }
    } else {
        // v and dl of every channel at the site and at its right and lower
        // neighbours, all loaded before any is used: clamped addresses and a
        // clamped channel index, so no branch separates the loads and a row
        // costs one memory round trip instead of one per channel and term
#pragma unroll
        for (int o = 0; o < R; ++o) {
            const int li = li0 + o, gi = ti0 + li;
            if (li % C != ch) continue;
            const bool in = gi < H && gj < W;
            const int e = clampi(gi, H - 1) * W + clampi(gj, W - 1);
            const bool hx = in && gj < W - 1, vx = in && gi < H - 1;
            const int eh = hx ? e + 1 : e, ev = vx ? e + W : e;
            T xa[kMaxC][3], xb[kMaxC][3], ga[kMaxC][3];
#pragma unroll
            for (int c = 0; c < kMaxC; ++c) {
                const int64_t co = (int64_t)(c < C ? c : 0) * HW;
                const T* Xc = X + co;
                const T* XPc = XP + co;
                const T* Gcc = G + co;
                xa[c][0] = ld<CO>(Xc, e);
                xa[c][1] = ld<CO>(Xc, eh);
                xa[c][2] = ld<CO>(Xc, ev);
                xb[c][0] = ld<CO>(XPc, e);
                xb[c][1] = ld<CO>(XPc, eh);
                xb[c][2] = ld<CO>(XPc, ev);
                ga[c][0] = ld<CO>(Gcc, e);
                ga[c][1] = ld<CO>(Gcc, eh);
                ga[c][2] = ld<CO>(Gcc, ev);
            }
            if (!in) continue;
            double ds2 = 0.0, s2 = 0.0;
#pragma unroll
            for (int c = 0; c < kMaxC; ++c) {
                if (c >= C) break;
                auto vat = [&](int k) { return dfma(m, xa[c][k] - xb[c][k], xa[c][k]); };
                const T v0 = vat(0), d0 = ga[c][0] * ninvL;
                const double bh = hx ? (double)(vat(1) - v0) : 0.0;
                const double bv = vx ? (double)(vat(2) - v0) : 0.0;
                const double ah = hx ? (double)(ga[c][1] * ninvL - d0) : 0.0;
                const double av = vx ? (double)(ga[c][2] * ninvL - d0) : 0.0;
                tv_site(bh, bv, ah, av, ds2, s2);
            }
            if (reg == 2) dtv += ds2;
            else if (reg == 0) dtv += ds2 / (sqrt(s2 + ds2 + e2) + sqrt(s2 + e2));
        }
    }

    // ---- data part of this block's channel, and the new iterate
    const bool exact = st.resync > 0 && (st.iters % st.resync) < 2;
    const T* __restrict__ KXc = KX + ch * HW;
    const T* __restrict__ KXPc = KXP + ch * HW;
    const T* __restrict__ Xc0 = X + ch * HW;
    const T* __restrict__ XPc0 = XP + ch * HW;
    T* __restrict__ XNc = XN + ch * HW;
    T* __restrict__ KXNc = KXN + ch * HW;
    T acc[R];
#pragma unroll
    for (int o = 0; o < R; ++o) acc[o] = T(0);
    // the step dl at the outputs, read before the correlation (which may
    // overwrite the tile)
    T dlc[R];
#pragma unroll
    for (int o = 0; o < R; ++o) dlc[o] = s_c[(li0 + o + c0) * CP + tx + c0];
    correlate_sel<T, K, R, !CO>(s_c, CP, I.thf, I.mf_thf, I.mf_sh, kplane(I, ch), li0, tx, acc);
    double ddat = 0.0;
    // small kernels: every row's loads in flight before any is used (clamped
    // addresses, no branch); large kernels keep their registers
    constexpr int RL = SEQ ? 1 : R;
    T kxr[RL], kxpr[RL], xr[RL], xpr[RL];
    if constexpr (!SEQ) {
#pragma unroll
        for (int o = 0; o < R; ++o) {
            const int e = clampi(ti0 + li0 + o, H - 1) * W + clampi(gj, W - 1);
            kxr[o] = ld<CO>(KXc, e);
            kxpr[o] = ld<CO>(KXPc, e);
            xr[o] = ld<CO>(Xc0, e);
            xpr[o] = ld<CO>(XPc0, e);
        }
    }
#pragma unroll
    for (int o = 0; o < R; ++o) {
        const int li = li0 + o, gi = ti0 + li;
        if (gi < H && gj < W) {
            const int e = gi * W + gj;
            const int q = SEQ ? 0 : o;
            if constexpr (SEQ) {
                kxr[0] = ld<CO>(KXc, e);
                kxpr[0] = ld<CO>(KXPc, e);
                xr[0] = ld<CO>(Xc0, e);
                xpr[0] = ld<CO>(XPc0, e);
            }
            // the residual at v by linearity, and its increment d = theta*dl
            const T kv = dfma(m, kxr[q] - kxpr[q], kxr[q]);
            const T d = acc[o];
            ddat += (double)d * ((double)kv + 0.5 * (double)d);
            const T xn = dfma(m, xr[q] - xpr[q], xr[q]) + dlc[o];
            at(XNc, e) = xn;
            if (I.hist) {
                T* __restrict__ hp = I.hist + (int64_t)st.iters * I.N + ch * HW;
                at(hp, e) = xn;
            }
            if (!exact) at(KXNc, e) = kv + d;
        }
    }
    if (exact) {
        // the residual at x+ = v + dl recomputed from x+ (staged with its
        // halo): in full, theta*x+ - y with FP64 taps and sums, and x+ with
        // that residual become the base point; otherwise relative to the
        // base, r_base + theta*(x+ - x_base), whose small difference the
        // storage type convolves accurately
        const bool full = st.resync_full > 0 && (st.iters % st.resync_full) == 0;
        const T* Xc = X + ch * HW;
        const T* XPc = XP + ch * HW;
        const T* XBc = I.xb + ch * HW;
        const T* RBc = I.rb + ch * HW;
        __syncthreads();
        if (full) {
            load_tile<CR, CP, CP>(s_c, ti0 - c0, tj0 - c0, H, W, [&](int g) {
                const T xv = ld<CO>(Xc, g);
                return dfma(m, xv - ld<CO>(XPc, g), xv) + ld<CO>(Gc, g) * ninvL;
            });
        } else {
            load_tile<CR, CP, CP>(s_c, ti0 - c0, tj0 - c0, H, W, [&](int g) {
                const T xv = ld<CO>(Xc, g);
                return (dfma(m, xv - ld<CO>(XPc, g), xv) + ld<CO>(Gc, g) * ninvL) - ld<CO>(XBc, g);
            });
        }
        __syncthreads();
        if (full) {
            double a64[R];
#pragma unroll
            for (int o = 0; o < R; ++o) a64[o] = 0.0;
            correlate64<T, K, R>(s_c, CP, I.theta64 + kplane(I, ch) * K * K, true, li0, tx, a64);
            T* __restrict__ XBw = I.xb + ch * HW;
            T* __restrict__ RBw = I.rb + ch * HW;
            const T* __restrict__ Yc = Y + ch * HW;
#pragma unroll
            for (int o = 0; o < R; ++o) {
                const int gi = ti0 + li0 + o;
                if (gi < H && gj < W) {
                    const int e = gi * W + gj;
                    const T r = (T)(a64[o] - (double)ld<CO>(Yc, e));
                    at(KXNc, e) = r;
                    at(RBw, e) = r;
                    at(XBw, e) = s_c[(li0 + o + c0) * CP + tx + c0];
                }
            }
        } else {
#pragma unroll
            for (int o = 0; o < R; ++o) acc[o] = T(0);
            correlate_sel<T, K, R, !CO>(s_c, CP, I.thf, I.mf_thf, I.mf_sh, kplane(I, ch), li0, tx, acc);
#pragma unroll
            for (int o = 0; o < R; ++o) {
                const int gi = ti0 + li0 + o;
                if (gi < H && gj < W) {
                    const int e = gi * W + gj;
                    at(KXNc, e) = ld<CO>(RBc, e) + acc[o];
                }
            }
        }
    }
    block_partial(ddat + I.pr.alpha * dtv, I.pB, lb);
}

template <typename T, int K, int R>
__global__ __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(min_waves<T>(K, R)))) void k_apg_trial(const Inst<T>* __restrict__ insts, const int* __restrict__ blk, int only,
                                                   const ApgState* __restrict__ sin, ApgState* __restrict__ sout) {
    MAID_STENCIL_PROLOGUE
    ApgState st = sin[ii];
    const bool writer = lb == 0 && threadIdx.x == 0;
    if (st.done) {
        if (writer) put_state(&sout[ii], st);
        return;
    }
    apg_trial_body<T, K, R, false>(I, lb, st, &sout[ii], writer);
}

// xout = v = x + m (x - x_prev): the point that passed the stop test
// (instances whose solve failed are left untouched).
template <typename T, bool CO>
__device__ __forceinline__ void apg_final_body(const Inst<T>& I, int lb, const ApgState& st) {
    if (st.status < 0 || !I.xout) return;
    const T* X = pick(I.X[0], I.X[1], I.X[2], st.cur);
    const T* XP = pick(I.X[0], I.X[1], I.X[2], st.prev);
    const T m = (T)st.m;
    T* out = I.xout;
    for (int64_t e = (int64_t)lb * kNT + threadIdx.x; e < I.N; e += (int64_t)I.nbe * kNT) {
        const T xv = ld64<CO>(X, e);
        out[e] = dfma(m, xv - ld64<CO>(XP, e), xv);
    }
}
template <typename T>
__global__ __launch_bounds__(kNT) void k_apg_final(const Inst<T>* __restrict__ insts, const int* __restrict__ blk, int only,
                                                   const ApgState* __restrict__ sin) {
    MAID_EW_PROLOGUE
    const ApgState st = sin[ii];
    apg_final_body<T, false>(I, lb, st);
}

// ------------------------------------------------------------------ conjugate gradients
// Direction pass.  Per instance: reads sin, block 0 writes sout.  Finishes
// gamma = ||r||^2 from the partials of the update (or set-up) pass, applies
// the stop tests (sqrt(gamma) <= tol; iteration cap), then forms
// p_new = r + beta p_old (p_new = r on the first iteration, beta =
// gamma / gamma_prev) and Kp = theta*p_new.  r and p_old are staged while the
// partials are in flight and combined once beta is known.  init = 1: the
// set-up call that copies the caller's q0 into q and p and forms theta*q0,
// without touching the state.
template <typename T, int K, int R, bool CO>
__device__ __forceinline__ void cg_dir_body(const Inst<T>& I, int lb, CgState& st, CgState* __restrict__ sout, bool writer,
                                            int init) {
    Partials pv;
    if (!init) pv = partials_issue<CO>(I.pR, I.nbe);
    constexpr int c0 = (K - 1) / 2, CP = cv_pitch(K), CR = cv_rows(K, R);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* s = reinterpret_cast<T*>(smem_raw);
    constexpr bool SEQ = seq_lds(K);   // SEQ: stage r + beta p once beta is known
    T* s_p = s + lds_conv(K, R, sizeof(T));
    const int H = I.pr.H, W = I.pr.W;
    const int64_t HW = (int64_t)H * W;
    int ti0, tj0, ch;
    tile_pos<R>(I.pr, lb, I.nb, ti0, tj0, ch);
    const int tx = threadIdx.x & 63, li0 = (threadIdx.x >> 6) * R;
    const int gj = tj0 + tx;
    const T* __restrict__ Pold = pick(I.P[0], I.P[1], st.pc) + ch * HW;
    T* __restrict__ Pnew = pick(I.P[0], I.P[1], st.pc ^ 1) + ch * HW;
    const T* __restrict__ rc = (init ? I.q0 : I.r) + ch * HW;
    const bool with_p = !init && !st.first;
    if constexpr (!SEQ) {
        auto sr = stage<CR, CP, CP>(s, ti0 - c0, tj0 - c0, [&](int g) { return ld<CO>(rc, g); });
        auto sp = stage<CR, CP, CP>(s_p, ti0 - c0, tj0 - c0, [&](int g) { return ld<CO>(Pold, g); });
        sr.fetch(H, W);
        if (with_p) sp.fetch(H, W);
        sr.put();
        if (with_p) sp.put();
    }
    double beta = 0.0;
    if (!init) {
        const double g = partials_finish<CO>(I.pR, I.nbe, pv);
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
        if (writer && sout) put_state(sout, st);
        if (st.done) return;
    }
    if (SEQ) {
        const T bT = (T)beta;
        if (with_p)
            load_tile<CR, CP, CP>(s, ti0 - c0, tj0 - c0, H, W, [&](int g) { return dfma(bT, ld<CO>(Pold, g), ld<CO>(rc, g)); });
        else
            load_tile<CR, CP, CP>(s, ti0 - c0, tj0 - c0, H, W, [&](int g) { return ld<CO>(rc, g); });
    } else if (with_p) {
        __syncthreads();
        const T bT = (T)beta;
        for (int idx = threadIdx.x; idx < CR * CP; idx += kNT) s[idx] = dfma(bT, s_p[idx], s[idx]);
    }
    __syncthreads();
    T acc[R];
#pragma unroll
    for (int o = 0; o < R; ++o) acc[o] = T(0);
    // the new direction at the outputs, read before the correlation (which
    // may overwrite the tile)
    T pn[R];
#pragma unroll
    for (int o = 0; o < R; ++o) pn[o] = s[(li0 + o + c0) * CP + tx + c0];
    correlate_sel<T, K, R, !CO>(s, CP, I.thf, I.mf_thf, I.mf_sh, kplane(I, ch), li0, tx, acc);
    T* __restrict__ Kp = I.Kp + ch * HW;
    T* __restrict__ qc = I.q + ch * HW;
#pragma unroll
    for (int o = 0; o < R; ++o) {
        const int li = li0 + o, gi = ti0 + li;
        if (gi < H && gj < W) {
            const int e = gi * W + gj;
            const T pv = pn[o];
            at(Pnew, e) = pv;
            at(Kp, e) = acc[o];
            if (init) at(qc, e) = pv;
        }
    }
}

template <typename T, int K, int R>
__global__ __launch_bounds__(kNT) void k_cg_dir(const Inst<T>* __restrict__ insts, const int* __restrict__ blk, int only,
                                                const CgState* __restrict__ sin, CgState* __restrict__ sout, int init) {
    MAID_STENCIL_PROLOGUE
    CgState st = sin[ii];
    const bool writer = lb == 0 && threadIdx.x == 0;
    if (st.done) {
        if (writer && !init) put_state(&sout[ii], st);
        return;
    }
    cg_dir_body<T, K, R, false>(I, lb, st, &sout[ii], writer, init);
}

// Hessian pass.  Per instance: reads sin, block 0 writes sout.
// Hp = theta . Kp + alpha grad^2 R(xt)[p] and per-block partials of <p,Hp>;
// grad^2 R(x)[p] = D^T (w Dp - w^3 m Dx), m = <Dx, Dp> over the coupled
// channels.  init = 1 computes H q0 only.
template <typename T, int K, int R, bool CO>
__device__ __forceinline__ void cg_hvp_body(const Inst<T>& I, int lb, const CgState& st, int init) {
    constexpr int c0 = (K - 1) / 2, CP = cv_pitch(K), CR = cv_rows(K, R);
    constexpr int VP = tv_pitch(), VR = tv_rows(R), WP = fx_pitch(), WR = fx_rows(R);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* sm = reinterpret_cast<T*>(smem_raw);
    const int C = I.pr.C, H = I.pr.H, W = I.pr.W, reg = I.pr.reg;
    const int64_t HW = (int64_t)H * W;
    int ti0, tj0, ch;
    tile_pos<R>(I.pr, lb, I.nb, ti0, tj0, ch);
    const int tx = threadIdx.x & 63, li0 = (threadIdx.x >> 6) * R;
    const int gj = tj0 + tx;
    const T alpha = (T)I.pr.alpha;
    const T* __restrict__ P = pick(I.P[0], I.P[1], st.pc ^ 1);

    // LDS: x and p with a one-pixel halo (small kernels: every channel, all
    // staged with the Kp tile in one round; large kernels: this block's
    // channel only, the coupled weights then formed from global memory, so
    // the footprint does not grow with C), and the weight planes w, w^3 m of
    // the flux sites (one each: reg 1 needs only this channel's).
    constexpr bool SEQ = seq_lds(K);
    const int nx = SEQ ? 1 : C;
    T* s_c = sm;
    T* s_x = SEQ ? sm : s_c + lds_conv(K, R, sizeof(T));
    T* s_p = s_x + nx * VR * VP;
    T* s_w = s_p + nx * VR * VP;
    T* s_mw = s_w + WR * WP;
    const T* kc = I.Kp + ch * HW;
    auto stage_kp = [&]() { load_tile<CR, CP, CP>(s_c, ti0 - c0, tj0 - c0, H, W, [&](int g) { return ld<CO>(kc, g); }); };
    auto xfun = [&](int c) { const T* xc = I.xt + c * HW; return [=](int g) { return ld<CO>(xc, g); }; };
    auto pfun = [&](int c) { const T* pc = P + c * HW; return [=](int g) { return ld<CO>(pc, g); }; };
    const T eps2 = (T)(I.pr.eps_tv * I.pr.eps_tv);
    if constexpr (!SEQ) {
        auto sk = stage<CR, CP, CP>(s_c, ti0 - c0, tj0 - c0, [&](int g) { return ld<CO>(kc, g); });
        auto x0 = stage<VR, VP, VP>(s_x, ti0 - 1, tj0 - 1, xfun(0));
        auto x1 = stage<VR, VP, VP>(s_x + VR * VP, ti0 - 1, tj0 - 1, xfun(C > 1 ? 1 : 0));
        auto x2 = stage<VR, VP, VP>(s_x + 2 * VR * VP, ti0 - 1, tj0 - 1, xfun(C > 2 ? 2 : 0));
        auto p0 = stage<VR, VP, VP>(s_p, ti0 - 1, tj0 - 1, pfun(0));
        auto p1 = stage<VR, VP, VP>(s_p + VR * VP, ti0 - 1, tj0 - 1, pfun(C > 1 ? 1 : 0));
        auto p2 = stage<VR, VP, VP>(s_p + 2 * VR * VP, ti0 - 1, tj0 - 1, pfun(C > 2 ? 2 : 0));
        sk.fetch(H, W);
        x0.fetch(H, W);
        p0.fetch(H, W);
        if (C > 1) { x1.fetch(H, W); p1.fetch(H, W); }
        if (C > 2) { x2.fetch(H, W); p2.fetch(H, W); }
        sk.put();
        x0.put();
        p0.put();
        if (C > 1) { x1.put(); p1.put(); }
        if (C > 2) { x2.put(); p2.put(); }
        __syncthreads();
        for (int idx = threadIdx.x; idx < WR * WP; idx += kNT) {
            const int r = idx / WP, cc = idx - r * WP;
            const int gi = ti0 - 1 + r, gj2 = tj0 - 1 + cc;
            const bool in = inside(gi, gj2, H, W);
            const bool hx = gj2 < W - 1, vx = gi < H - 1;
            const int i0 = r * VP + cc;
            T s2 = T(0), mm = T(0);
            const int c_lo = reg == 1 ? ch : 0, c_hi = reg == 1 ? ch + 1 : C;
            for (int c = c_lo; c < c_hi; ++c) {
                const T* Xv = s_x + c * VR * VP;
                const T* Pv = s_p + c * VR * VP;
                const T xh = hx ? Xv[i0 + 1] - Xv[i0] : T(0);
                const T xv = vx ? Xv[i0 + VP] - Xv[i0] : T(0);
                const T ph = hx ? Pv[i0 + 1] - Pv[i0] : T(0);
                const T pv = vx ? Pv[i0 + VP] - Pv[i0] : T(0);
                s2 += xh * xh + xv * xv;
                mm += xh * ph + xv * pv;
            }
            if (reg == 2) {
                s_w[idx] = in ? T(1) : T(0);
                s_mw[idx] = T(0);
            } else {
                const T w = in ? drsqrt(s2 + eps2) : T(0);
                s_w[idx] = w;
                s_mw[idx] = w * w * w * mm;
            }
        }
    } else {
        auto sx = stage<VR, VP, VP>(s_x, ti0 - 1, tj0 - 1, xfun(ch));
        auto sp = stage<VR, VP, VP>(s_p, ti0 - 1, tj0 - 1, pfun(ch));
        sx.fetch(H, W);
        sp.fetch(H, W);
        sx.put();
        sp.put();
        for (int idx = threadIdx.x; idx < WR * WP; idx += kNT) {
            const int r = idx / WP, cc = idx - r * WP;
            const int gi = ti0 - 1 + r, gj2 = tj0 - 1 + cc;
            const bool in = inside(gi, gj2, H, W);
            // clamped neighbours: outside the image a difference reads zero
            const int gic = clampi(gi, H - 1), gjc = clampi(gj2, W - 1);
            const int e = gic * W + gjc;
            const int eh = gjc < W - 1 ? e + 1 : e, ev = gic < H - 1 ? e + W : e;
            T s2 = T(0), mm = T(0);
            if (reg != 2) {
                // every coupled channel's loads before any is used (a clamped
                // channel index: no branch separates them)
                const int c_lo = reg == 1 ? ch : 0, c_n = reg == 1 ? 1 : C;
                T xa[kMaxC][3], pa[kMaxC][3];
#pragma unroll
                for (int k = 0; k < kMaxC; ++k) {
                    const int64_t co = (int64_t)(c_lo + (k < c_n ? k : 0)) * HW;
                    const T* xc = I.xt + co;
                    const T* pc = P + co;
                    xa[k][0] = ld<CO>(xc, e);
                    xa[k][1] = ld<CO>(xc, eh);
                    xa[k][2] = ld<CO>(xc, ev);
                    pa[k][0] = ld<CO>(pc, e);
                    pa[k][1] = ld<CO>(pc, eh);
                    pa[k][2] = ld<CO>(pc, ev);
                }
#pragma unroll
                for (int k = 0; k < kMaxC; ++k) {
                    if (k >= c_n) break;
                    const T xh = xa[k][1] - xa[k][0], xv = xa[k][2] - xa[k][0];
                    const T ph = pa[k][1] - pa[k][0], pv = pa[k][2] - pa[k][0];
                    s2 += xh * xh + xv * xv;
                    mm += xh * ph + xv * pv;
                }
            }
            if (reg == 2) {
                s_w[idx] = in ? T(1) : T(0);
                s_mw[idx] = T(0);
            } else {
                const T w = in ? drsqrt(s2 + eps2) : T(0);
                s_w[idx] = w;
                s_mw[idx] = w * w * w * mm;
            }
        }
    }
    __syncthreads();
    T acc[R];
#pragma unroll
    for (int o = 0; o < R; ++o) acc[o] = T(0);
    if (!SEQ) correlate<T, K, R>(s_c, CP, I.th + kplane(I, ch) * K * K, li0, tx, acc);
    const T* Xv = s_x + (SEQ ? 0 : ch) * VR * VP;
    const T* Pv = s_p + (SEQ ? 0 : ch) * VR * VP;
    const T* Wt = s_w;
    const T* Mw = s_mw;
    // SEQ: the TV term and p of each output wait in LDS past the tile region
    // while the convolution tile reuses it (registers stay with the convolution)
    T* s_park = sm + cmax(2 * VR * VP + 2 * WR * WP, lds_conv(K, R, sizeof(T)));
    T hvv[SEQ ? 1 : R], pc[SEQ ? 1 : R];
#pragma unroll
    for (int o = 0; o < R; ++o) {
        const int li = li0 + o, gi = ti0 + li;
        const int r = li + 1, cc = tx + 1;
        const int i0 = r * VP + cc;
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
        const T hv = fh_left - fh_here + fv_up - fv_here;
        if constexpr (SEQ) {
            s_park[o * kNT + threadIdx.x] = hv;
            s_park[(R + o) * kNT + threadIdx.x] = Pv[i0];
        } else {
            hvv[o] = hv;
            pc[o] = Pv[i0];
        }
    }
    if (SEQ) {
        __syncthreads();
        stage_kp();
        __syncthreads();
        correlate_sel<T, K, R, !CO>(s_c, CP, I.th, I.mf_th, I.mf_sh, kplane(I, ch), li0, tx, acc);
    }
    double kap = 0.0;
    T* __restrict__ Hp = I.Hp + ch * HW;
#pragma unroll
    for (int o = 0; o < R; ++o) {
        const int gi = ti0 + li0 + o;
        if (gi < H && gj < W) {
            const T hv = SEQ ? s_park[o * kNT + threadIdx.x] : hvv[SEQ ? 0 : o];
            const T pp = SEQ ? s_park[(R + o) * kNT + threadIdx.x] : pc[SEQ ? 0 : o];
            const T hp = dfma(alpha, hv, acc[o]);
            at(Hp, gi * W + gj) = hp;
            kap += (double)pp * (double)hp;
        }
    }
    if (!init) block_partial(kap, I.pK, lb);
}

template <typename T, int K, int R>
__global__ __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(min_waves<T>(K, R)))) void k_cg_hvp(const Inst<T>* __restrict__ insts, const int* __restrict__ blk, int only,
                                                const CgState* __restrict__ sin, CgState* __restrict__ sout, int init) {
    MAID_STENCIL_PROLOGUE
    const CgState st = sin[ii];
    if (!init && lb == 0 && threadIdx.x == 0) put_state(&sout[ii], st);
    if (st.done) return;
    cg_hvp_body<T, K, R, false>(I, lb, st, init);
}

// Update pass.  Per instance: reads sin, block 0 writes sout.  Finishes the
// curvature kappa = <p,Hp> (not positive: MAID_NOT_SPD), a = gamma/kappa,
// then q += a p, r -= a Hp and per-block partials of ||r||^2.  The first
// element of every thread is loaded while the partials are in flight.
template <typename T, bool CO>
__device__ __forceinline__ void cg_update_body(const Inst<T>& I, int lb, CgState& st, CgState* __restrict__ sout,
                                               bool writer) {
    const Partials pv = partials_issue<CO>(I.pK, I.nb);
    const T* __restrict__ P = pick(I.P[0], I.P[1], st.pc ^ 1);
    T* __restrict__ q = I.q;
    T* __restrict__ r = I.r;
    const T* __restrict__ Hp = I.Hp;
    const int64_t e0 = (int64_t)lb * kNT + threadIdx.x, stride = (int64_t)I.nbe * kNT;
    T p0 = T(0), q0 = T(0), r0 = T(0), h0 = T(0);
    if (e0 < I.N) {
        p0 = ld64<CO>(P, e0);
        q0 = ld64<CO>(q, e0);
        r0 = ld64<CO>(r, e0);
        h0 = ld64<CO>(Hp, e0);
    }
    const double kappa = partials_finish<CO>(I.pK, I.nb, pv);
    st.kappa = kappa;
    if (!(kappa > 0.0) || !finite_d(kappa)) {
        st.done = 1;
        st.status = finite_d(kappa) ? ST_NOT_SPD : ST_NONFINITE;
        if (writer && sout) put_state(sout, st);
        return;
    }
    st.a = st.gamma / kappa;
    st.iters += 1;
    st.pc ^= 1;
    if (writer && sout) put_state(sout, st);
    const T a = (T)st.a;
    double rs = 0.0;
    if (e0 < I.N) {
        q[e0] = dfma(a, p0, q0);
        const T rv = dfma(-a, h0, r0);
        r[e0] = rv;
        rs += (double)rv * (double)rv;
    }
    // the rest four at a time, every load in flight before any is used
    for (int64_t e = e0 + stride; e < I.N; e += 4 * stride) {
        T pv[4], qv[4], rv[4], hv[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t ek = e + k * stride;
            const int64_t el = ek < I.N ? ek : 0;
            pv[k] = ld64<CO>(P, el);
            qv[k] = ld64<CO>(q, el);
            rv[k] = ld64<CO>(r, el);
            hv[k] = ld64<CO>(Hp, el);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t ek = e + k * stride;
            if (ek < I.N) {
                q[ek] = dfma(a, pv[k], qv[k]);
                const T rn = dfma(-a, hv[k], rv[k]);
                r[ek] = rn;
                rs += (double)rn * (double)rn;
            }
        }
    }
    block_partial(rs, I.pR, lb);
}

template <typename T>
__global__ __launch_bounds__(kNT) void k_cg_update(const Inst<T>* __restrict__ insts, const int* __restrict__ blk, int only,
                                                   const CgState* __restrict__ sin, CgState* __restrict__ sout) {
    MAID_EW_PROLOGUE
    // instances on the one-pass CG form have their own state sequence
    if (I.cg1) return;
    CgState st = sin[ii];
    const bool writer = lb == 0 && threadIdx.x == 0;
    if (st.done) {
        if (writer) put_state(&sout[ii], st);
        return;
    }
    cg_update_body<T, false>(I, lb, st, &sout[ii], writer);
}

// r = b - H q0 (Hp holds H q0) and per-block partials of ||r||^2.
template <typename T>
__global__ __launch_bounds__(kNT) void k_cg_init(const Inst<T>* __restrict__ insts, const int* __restrict__ blk, int only,
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
// One block per instance: the initial solver states of the table entry go
// into the state arrays (Lst, Cst: nullable), then theta64 (double, kc KxK
// planes) -> th (correlation form) and thf (flipped, convolution form), both
// column-major in the compute type, plane by plane; with Lst, the largest
// plane l1 norm squared (a bound of ||theta*.||^2: Young's inequality per
// channel, the channels do not mix) becomes the starting Lipschitz estimate
// when the initial one is <= 0; red[slot_abs] receives that l1 norm when
// slot_abs >= 0.
template <typename T>
__global__ __launch_bounds__(1024) void k_prep_kernel(const Inst<T>* insts, ApgState* __restrict__ Lst,
                                                      CgState* __restrict__ Cst, int slot_abs,
                                                      const unsigned* __restrict__ up_src, unsigned* up_dst,
                                                      int up_roles) {
    __shared__ double s_abs[1024];
    if (up_src) {
        // the table upload: block b copies entry b of each of up_roles
        // adjacent role tables (gridDim.x entries each) from mapped host
        // memory; insts is the first of those tables on the device
        constexpr int IW = (int)(sizeof(Inst<T>) / 4);
        static_assert(sizeof(Inst<T>) % 4 == 0, "instance entries are whole words");
        for (int w = threadIdx.x; w < up_roles * IW; w += 1024) {
            const int r = w / IW, k = w - r * IW;
            const size_t o = ((size_t)r * gridDim.x + blockIdx.x) * IW + k;
            up_dst[o] = up_src[o];
        }
        __syncthreads();
    }
    const Inst<T>& I = insts[blockIdx.x];
    if (threadIdx.x == 0) {
        if (Lst) put_state(&Lst[blockIdx.x], I.st0);
        if (Cst) put_state(&Cst[blockIdx.x], I.cg0);
    }
    if (!I.theta64) return;
    const int K = I.K, KK = K * K, KP = I.kc > 1 ? I.kc : 1;
    const int t = threadIdx.x;
    __shared__ int s_sh[kMaxC];
    double l1max = 0.0;
    for (int p = 0; p < KP; ++p) {
        const double* th64 = I.theta64 + p * KK;
        double a = 0.0;
        if (t < KK) {
            const int u = t / K, v = t - u * K;
            const double w = th64[t];
            // column-major: out(u,v) at v*K+u; the flipped kernel f(u',v') = theta(K-1-u', K-1-v')
            I.th[p * KK + v * K + u] = (T)w;
            I.thf[p * KK + (K - 1 - v) * K + (K - 1 - u)] = (T)w;
            a = fabs(w);
        }
        __syncthreads();   // s_abs of the previous plane has been read
        s_abs[t] = a;
        __syncthreads();
        if (t == 0) {
            double s = 0.0, mx = 0.0;
            for (int i = 0; i < KK; ++i) {
                s += s_abs[i];
                mx = fmax(mx, s_abs[i]);
            }
            l1max = fmax(l1max, s);
            // the matrix-core layouts: each plane scaled by a power of two
            // that brings its largest tap into [2^14, 2^15)
            const float mxf = (float)mx;
            s_sh[p] = mxf >= 1.0e-30f ? mf_shift(mxf) : 0;
            if (I.mf_th) I.mf_sh[p] = s_sh[p];
        }
    }
    if (t == 0) {
        if (Lst && !(I.st0.L > 0.0)) Lst[blockIdx.x].L = l1max * l1max;
        if (slot_abs >= 0) I.red[slot_abs] = l1max;
    }
    if (!I.mf_th) return;
    __syncthreads();
    const int fw = mf_frag_bytes(K) / 16;   // one plane's layout, in uint4
    for (int p = 0; p < KP; ++p) {
        mf_fragments(I.theta64 + p * KK, K, false, s_sh[p], I.mf_th + p * fw, t, 1024);
        mf_fragments(I.theta64 + p * KK, K, true, s_sh[p], I.mf_thf + p * fw, t, 1024);
    }
}

// One block per instance: red[slot] = sum of the instance's cv_part partials;
// with sob_th, also red[sob_slot] = r(theta) = beta (w0 ||e||^2 + ||D_h e||^2
// + ||D_v e||^2), e = theta - a, Neumann forward differences on the KxK grid.
template <typename T>
__global__ __launch_bounds__(kNT) void k_finish(const Inst<T>* __restrict__ insts, int slot, int sob_slot) {
    const Inst<T>& I = insts[blockIdx.x];
    if (I.cv_part) {
        const double s = reduce_partials(I.cv_part, I.nb);
        if (threadIdx.x == 0) I.red[slot] = s;
    }
    if (I.sob_th) {
        // every plane's own KxK grid (no difference across planes)
        const int K = I.K, KK = K * K, KP = I.kc > 1 ? I.kc : 1;
        const double* th = I.sob_th;
        const double* a = I.sob_a;
        double v = 0.0;
        for (int t = threadIdx.x; t < KP * KK; t += kNT) {
            const int tp = t % KK, u = tp / K, w = tp - u * K;
            const double e = th[t] - a[t];
            const double dh = w < K - 1 ? (th[t + 1] - a[t + 1]) - e : 0.0;
            const double dv = u < K - 1 ? (th[t + K] - a[t + K]) - e : 0.0;
            v += I.h1_w0 * e * e + dh * dh + dv * dv;
        }
        const double s = block_sum(v);
        if (threadIdx.x == 0) I.red[sob_slot] = I.beta * s;
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

// One block's share: items b0, b0 + nb, ... of the instance; its K x K
// partial sum goes to part[b0].
template <typename T, int KT>
__device__ __forceinline__ void hg_corr_blk(int C, int H, int W, int K, const double* __restrict__ rho,
                                            const T* __restrict__ q, const double* __restrict__ wq,
                                            const T* __restrict__ xt, double* __restrict__ part, int b0, int nb) {
    constexpr int NO = KT / 16;
    constexpr int AP = kHgTJ + 1;            // A tile: rows TI+K-1, cols TJ
    constexpr int BP = kHgTJ + kMaxK;        // B tile: rows TI, cols TJ+K-1
    __shared__ double sA[(kHgTI + kMaxK - 1) * AP];
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
    for (int item = b0; item < nitems; item += nb) {
        const int term = item & 1;
        const int ch = (item >> 1) % C;
        const int sp = (item >> 1) / C;
        const int ti0 = (sp / ntj) * kHgTI, tj0 = (sp % ntj) * kHgTJ;
        const double* Asrc = (term ? wq : rho) + ch * HW;
        const T* Bsrc = (term ? xt : q) + ch * HW;
        __syncthreads();
        for (int idx = threadIdx.x; idx < arows * kHgTJ; idx += kNT) {
            const int r = idx / kHgTJ, cc = idx - r * kHgTJ;
            const int gi = ti0 - c0 + r, gj = tj0 + cc;
            sA[r * AP + cc] = (gi >= 0 && gi < H && gj < W) ? Asrc[gi * W + gj] : 0.0;
        }
        for (int idx = threadIdx.x; idx < kHgTI * bcols; idx += kNT) {
            const int r = idx / bcols, cc = idx - r * bcols;
            const int gi = ti0 + r, gj = tj0 - c0 + cc;
            sB[r * BP + cc] = (gi < H && gj >= 0 && gj < W) ? Bsrc[gi * W + gj] : T(0);
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
        part[(size_t)b0 * KT * KT + i] = ((s_red[0][i] + s_red[1][i]) + s_red[2][i]) + s_red[3][i];
}

// The correlations of a batch (a plain solve is a batch of one) in one
// launch per tile class KT: the
// instances of the class (K <= 16 for KT = 16) with hg_nblk > 0 own
// consecutive block ranges [hg_base, hg_base + hg_nblk) and each range
// runs exactly as a launch of its own would (so the partial sums, and z,
// are bitwise those of the per-instance form).  With per-channel kernels
// (kc > 1) the range splits into kc equal parts, part p correlating channel
// p alone into its own partial sums.
template <typename T, int KT>
__global__ __launch_bounds__(kNT) void k_hg_corr_batch(const Inst<T>* __restrict__ insts, int n) {
    const int b = (int)blockIdx.x;
    for (int i = 0; i < n; ++i) {
        const Inst<T>& I = insts[i];
        if ((I.K <= 16) != (KT == 16) || b < I.hg_base || b >= I.hg_base + I.hg_nblk) continue;
        if (I.kc > 1) {
            const int nbp = I.hg_nblk / I.kc, lb = b - I.hg_base, p = lb / nbp;
            const int64_t o = (int64_t)p * I.pr.H * I.pr.W;
            hg_corr_blk<T, KT>(1, I.pr.H, I.pr.W, I.K, I.hg_rho + o, I.hg_q + o, I.hg_w + o, I.cv_in + o,
                               I.hg_part + (size_t)p * nbp * KT * KT, lb - p * nbp, nbp);
            return;
        }
        hg_corr_blk<T, KT>(I.pr.C, I.pr.H, I.pr.W, I.K, I.hg_rho, I.hg_q, I.hg_w, I.cv_in, I.hg_part, b - I.hg_base,
                           I.hg_nblk);
        return;
    }
}

// z = -sum_blocks Z + with_r * grad r(theta) for one KxK plane; returns
// ||z||^2 to thread 0 (a block of 1024 threads).
template <int KT>
__device__ __forceinline__ double hg_final_blk(double beta, double h1_w0, const double* __restrict__ part, int nblk,
                                               int K, const double* __restrict__ th, const double* __restrict__ a,
                                               int with_r, double* __restrict__ z) {
    __shared__ double s_e[1024];
    __shared__ double s_z[1024];
    __shared__ double s_g[1024];
    const int t = threadIdx.x, KK = K * K;
    __syncthreads();   // the previous plane's reads of the shared arrays are done
    if (t < KK) s_e[t] = (with_r && a) ? th[t] - a[t] : 0.0;
    // the sum over the correlation blocks: G = 1024 / K^2 threads per tap,
    // thread (g, tap) adds blocks g, g + G, ... in order, then the tap's
    // thread adds the G sums in order (a fixed order for every launch)
    const int G = KK <= 1024 ? 1024 / KK : 1;
    if (t < G * KK) {
        const int g = t / KK, tap = t - g * KK;
        const int u = tap / K, v = tap - u * K;
        double sg = 0.0;
#pragma unroll 4
        for (int bidx = g; bidx < nblk; bidx += G) sg += part[(size_t)bidx * KT * KT + u * KT + v];
        s_g[t] = sg;
    }
    __syncthreads();
    double zz = 0.0;
    if (t < KK) {
        const int u = t / K, v = t - u * K;
        double s = s_g[t];
        for (int g = 1; g < G; ++g) s += s_g[g * KK + t];
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
    double s = 0.0;
    if (t == 0)
        for (int i = 0; i < KK; ++i) s += s_z[i];
    return s;
}

// block i finishes instance i of a batched correlation launch (if it was in it)
template <typename T, int KT>
__global__ __launch_bounds__(1024) void k_hg_final_batch(const Inst<T>* __restrict__ insts) {
    const Inst<T>& I = insts[blockIdx.x];
    if (I.hg_nblk <= 0 || (I.K <= 16) != (KT == 16)) return;
    // ||z||^2: the planes' sums added in plane order
    const int KP = I.kc > 1 ? I.kc : 1, KK = I.K * I.K, nbp = I.hg_nblk / KP;
    double zn2 = 0.0;
    for (int p = 0; p < KP; ++p)
        zn2 += hg_final_blk<KT>(I.beta, I.h1_w0, I.hg_part + (size_t)p * nbp * KT * KT, nbp, I.K,
                                I.theta64 + p * KK, I.hg_a ? I.hg_a + p * KK : nullptr, I.hg_with_r, I.hg_z + p * KK);
    if (threadIdx.x == 0) *I.hg_zn2 = zn2;
}

}  // namespace maid
