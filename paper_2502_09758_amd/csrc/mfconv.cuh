// mfconv.cuh -- the K x K correlation of a staged FP32 tile on the matrix
// cores (FP32 storage, K >= 13: the range where the vector ALUs bound the
// passes).
//
// The correlation out(i,j) = sum_{u,v} ker(u,v) s(i+u, j+v) of a 64-wide,
// 4R-row output tile (R = 4 or 8) is a sum over the tap rows u of banded
// (Toeplitz) products: for a 16 x 16 output block at (i0, j0),
//   out(i0+i, j0+jl) = sum_u sum_m S_u(i, m) T_u(m, jl),
//   S_u(i, m) = s(i0+i+u, j0+m),  T_u(m, jl) = ker(u, m-jl) (0 outside [0,K)),
// with m over Lm = 16+K-1 columns rounded up to a multiple of 8.  Stacking
// the tap rows along the contraction gives one [16 x K Lm] . [K Lm x 16]
// product per block, cut into 32-deep chunks for v_mfma_f32_16x16x32_f16
// (FP32 accumulation).  T depends only on the kernel: it is laid out once
// per kernel, in the exact register order of the instruction's B operand,
// by the preparation pass (mf_fragments below), and read from global memory
// (it stays in L2); S is read from LDS, 8 consecutive columns of one row per
// lane per chunk (one 16-byte read).  A K = 31 block spends 31 of 48 columns
// of each chunk on nonzero taps.
//
// Precision: FP16 has 11 significant bits, so each FP32 operand is split
// into two FP16 parts, v = hi + lo, and the product is formed from three
// FP16 products (hi.hi + hi.lo + lo.hi; the dropped lo.lo and the split's
// own rounding are below 2^-22 of the product).  To keep both parts inside
// FP16's range, the tile is scaled by a power of two that brings its largest
// magnitude into [2^14, 2^15), and the kernel likewise (its exponent comes
// with the fragments); the accumulated sums are scaled back exactly.
//
// Work split: the four waves of a block take every fourth chunk each and
// accumulate every output block of the tile; their partial sums are
// combined through LDS in a fixed order ((w0 + w2) + (w1 + w3)), so the
// result is deterministic.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace maid {

typedef _Float16 mf_h8 __attribute__((ext_vector_type(8)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));

// Geometry of the banded product for kernel size K.
template <int K> struct MfGeom {
    static constexpr int Lm = ((K + 15) + 7) / 8 * 8;   // columns per tap row (multiple of 8)
    static constexpr int NC = (K * Lm + 31) / 32;       // 32-deep chunks
    static constexpr int W16 = 48 + Lm;                 // staged columns the blocks read
    static constexpr int P16 = W16 + 8;                 // LDS pitch of the FP16 tiles (halfs)
};

// The tiles the matrix-core path applies to.
template <typename T, int K, int R> __host__ __device__ constexpr bool mf_ok() {
    return sizeof(T) == 4 && K >= 13 && K <= 31 && (R == 4 || R == 8);
}

// Bytes of the B-operand layout of one kernel (hi and lo parts).
__host__ __device__ constexpr int mf_frag_bytes(int K) { return ((K * (((K + 15) + 7) / 8 * 8) + 31) / 32) * 2 * 64 * 16; }

// row pitch (floats) of the wave partial sums
constexpr int kMfPP = 68;

// The correlation works in the staged tile's own LDS region: it writes the
// tile's FP16 halves (two tiles of P16 halfs per row) over the FP32 tile,
// then the waves' partial sums (two planes of 4R rows of kMfPP floats).
// lds_conv(K, R, 4) floats cover all three (checked here).
static_assert(kMfPP == 68, "partial-sum pitch of the LDS region sizing");
template <int K, int R> __host__ __device__ constexpr bool mf_region_fits() {
    constexpr int CR = 4 * R + K - 1;
    return MfGeom<K>::P16 == mf_p16(K) && CR * MfGeom<K>::P16 <= lds_conv(K, R, 4) &&
           2 * 4 * R * kMfPP <= lds_conv(K, R, 4) && CR * (64 + K - 1) <= lds_conv(K, R, 4);
}

// 2^e as a float (|e| < 127)
__device__ __forceinline__ float mf_pow2(int e) { return __int_as_float((e + 127) << 23); }

// Exponent that brings a largest magnitude mx > 0 into [2^14, 2^15).
__device__ __forceinline__ int mf_shift(float mx) {
    const int e = ((__float_as_int(mx) >> 23) & 255) - 127;   // floor(log2 mx) for normal mx
    return 14 - e;
}

// Columns per tap row and 32-deep chunks of kernel size K (runtime form of
// MfGeom, for the preparation pass).
__host__ __device__ constexpr int mf_lm(int K) { return ((K + 15) + 7) / 8 * 8; }
__host__ __device__ constexpr int mf_nc(int K) { return (K * mf_lm(K) + 31) / 32; }

// B-operand fragments of one kernel: entry (c, part, lane) holds the 8 FP16
// values of lane `lane` for chunk c (part 0: hi, 1: lo):
//   k = 32 c + 8 (lane / 16) + t, u = k / Lm, m = k mod Lm, jl = lane mod 16,
//   value = ker(u, m - jl) * 2^sh   (0 outside the kernel or for u >= K),
// ker(u, v) = theta[u K + v], or theta[(K-1-u) K + (K-1-v)] with `flip`.
// Written by the threads t0, t0 + nt, ... of a block.
__device__ __forceinline__ void mf_fragments(const double* __restrict__ theta, int K, bool flip, int sh,
                                             uint4* __restrict__ out, int t0, int nt) {
    const int Lm = mf_lm(K), NC = mf_nc(K);
    const float scale = mf_pow2(sh);
    for (int e = t0; e < NC * 64; e += nt) {
        const int c = e >> 6, lane = e & 63, jl = lane & 15;
        union { _Float16 h[8]; uint4 v; } hi, lo;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int k = 32 * c + 8 * (lane >> 4) + t;
            const int u = k / Lm, m = k - u * Lm, v = m - jl;
            float w = 0.0f;
            if (u < K && v >= 0 && v < K) {
                const int uu = flip ? K - 1 - u : u, vv = flip ? K - 1 - v : v;
                w = (float)theta[uu * K + vv] * scale;
            }
            const _Float16 h = (_Float16)w;
            hi.h[t] = h;
            lo.h[t] = (_Float16)(w - (float)h);
        }
        out[(2 * c) * 64 + lane] = hi.v;
        out[(2 * c + 1) * 64 + lane] = lo.v;
    }
}

// acc[o] += sum_{u,v} ker(u,v) s[(li0+o+u) pitch + tx+v] for the tile layout
// of the stencil passes (lane tx of wave wy holds rows wy R .. wy R+R-1 of
// column tx), ker given by its fragments `frag` and the power of two
// `ksh` they were scaled by.  s: the staged FP32 tile (4R+K-1 rows, 64+K-1
// columns, 16-byte aligned) at the start of an LDS region of
// lds_conv(K, R, 4) floats, which the correlation overwrites (the tile is
// gone when it returns).  Every thread of the block must call it (it has
// barriers).
template <int K, int R>
__device__ __forceinline__ void correlate_mfma(float* s, int pitch, const uint4* __restrict__ frag, int ksh, int li0,
                                               int tx, float (&acc)[R]) {
    using G = MfGeom<K>;
    constexpr int TH = 4 * R, CR = TH + K - 1, CP = 64 + K - 1, NB = R, P16 = G::P16, PP = kMfPP;
    static_assert(mf_region_fits<K, R>(), "the LDS region holds the FP16 tiles and the partial sums");
    __shared__ float s_mx[4];
    _Float16* Sh = reinterpret_cast<_Float16*>(s);
    _Float16* Sl = Sh + CR * P16;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;

    // the tile's largest magnitude (max is exact: any order gives the same),
    // read as float2 over the flat tile (rows are whole pairs: CP is even)
    static_assert(CP % 2 == 0 && P16 % 8 == 0, "tile shapes");
    float mx = 0.0f;
    {
        constexpr int N2 = CR * CP / 2;
        const float2* s2 = reinterpret_cast<const float2*>(s);
        for (int e = t; e < N2; e += 256) {
            const float2 v = s2[e];
            mx = fmaxf(mx, fmaxf(fabsf(v.x), fabsf(v.y)));
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
    if (lane == 0) s_mx[w] = mx;
    __syncthreads();
    mx = fmaxf(fmaxf(s_mx[0], s_mx[1]), fmaxf(s_mx[2], s_mx[3]));
    // a tile of zeros (or one below the normal range) keeps shift 0
    const int sh = mx >= 1.0e-30f ? mf_shift(mx) : 0;
    const float scale = mf_pow2(sh);
    // the split, in place: each thread converts runs of 8 columns of one row
    // (float2 reads; columns past the tile are zero), all of its runs read
    // before the barrier and written after it (one 16-byte write per part)
    {
        constexpr int NS = P16 / 8, IT = (CR * NS + 255) / 256;
        union H8 { _Float16 h[8]; uint4 v; };
        H8 hi[IT], lo[IT];
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int e = t + 256 * it;
            const int r = e / NS, c = 8 * (e - r * NS);
#pragma unroll
            for (int k = 0; k < 8; k += 2) {
                float2 v = make_float2(0.0f, 0.0f);
                if (e < CR * NS && c + k < CP) v = *reinterpret_cast<const float2*>(s + r * pitch + c + k);
                const float a = v.x * scale, b = v.y * scale;
                const _Float16 ha = (_Float16)a, hb = (_Float16)b;
                hi[it].h[k] = ha;
                hi[it].h[k + 1] = hb;
                lo[it].h[k] = (_Float16)(a - (float)ha);
                lo[it].h[k + 1] = (_Float16)(b - (float)hb);
            }
        }
        __syncthreads();   // every thread has read the FP32 tile
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int e = t + 256 * it;
            if (e < CR * NS) {
                const int r = e / NS, c = 8 * (e - r * NS);
                *reinterpret_cast<uint4*>(Sh + r * P16 + c) = hi[it].v;
                *reinterpret_cast<uint4*>(Sl + r * P16 + c) = lo[it].v;
            }
        }
    }
    __syncthreads();

    mf_f4 d[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) d[b] = mf_f4{0.0f, 0.0f, 0.0f, 0.0f};
    const int r16 = lane & 15, g = lane >> 4;
    // chunks dealt round-robin to the waves (c = w, w+4, ...); the B
    // fragments of the next chunk are loaded while this chunk's products
    // run (the last prefetch re-reads the last chunk: no branch in the loop)
    const uint4* __restrict__ F = frag + lane;
    const int nw = (G::NC - w + 3) >> 2;
    uint4 bh4 = F[(2 * w) * 64], bl4 = F[(2 * w + 1) * 64];
#pragma unroll 1
    for (int i = 0; i < nw; ++i) {
        const int c = w + 4 * i;
        const mf_h8 bh = __builtin_bit_cast(mf_h8, bh4), bl = __builtin_bit_cast(mf_h8, bl4);
        const int cn = c + 4 < G::NC ? c + 4 : G::NC - 1;
        bh4 = F[(2 * cn) * 64];
        bl4 = F[(2 * cn + 1) * 64];
        const int k0 = 32 * c + 8 * g;
        int u = k0 / G::Lm;
        const int m0 = k0 - u * G::Lm;
        u = u < K ? u : K - 1;               // padding rows: the fragments are zero there
        const int base = (r16 + u) * P16 + m0;
        mf_h8 ah[NB], al[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int off = base + 16 * (b >> 2) * P16 + 16 * (b & 3);
            ah[b] = *reinterpret_cast<const mf_h8*>(Sh + off);
            al[b] = *reinterpret_cast<const mf_h8*>(Sl + off);
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            d[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[b], bh, d[b], 0, 0, 0);
            d[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[b], bl, d[b], 0, 0, 0);
            d[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[b], bh, d[b], 0, 0, 0);
        }
    }
    __syncthreads();   // every wave is done with the FP16 tiles

    // wave partials: lane (g, r16) holds rows 4g..4g+3, column r16 of each
    // block; rows padded to PP floats so that the four rows a write covers
    // fall in different LDS banks
    float* P = s;   // [2][TH][PP], over the FP16 tiles
    auto at_p = [&](int half, int b, int k) -> float& {
        return P[(half * TH + 16 * (b >> 2) + 4 * g + k) * PP + 16 * (b & 3) + r16];
    };
    if (w >= 2) {
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int k = 0; k < 4; ++k) at_p(w - 2, b, k) = d[b][k];
    }
    __syncthreads();
    if (w < 2) {
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                float& p = at_p(w, b, k);
                p = d[b][k] + p;
            }
    }
    __syncthreads();
    const float unscale_x = mf_pow2(-sh), unscale_k = mf_pow2(-ksh);
#pragma unroll
    for (int o = 0; o < R; ++o) {
        const int row = li0 + o;
        const float v = P[row * PP + tx] + P[(TH + row) * PP + tx];
        acc[o] += (v * unscale_x) * unscale_k;
    }
    __syncthreads();   // the LDS region may be reused by the caller
}

}  // namespace maid
