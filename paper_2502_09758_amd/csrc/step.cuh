// step.cuh -- one-pass FISTA iterations (Algorithm 1, lower level) for
// single-channel images and small kernels (3 <= K <= 11).
//
// The two-pass form needs a grid-wide sum between the gradient and the trial
// step only for the stop test, and a halo exchange only because the trial
// convolves the step dl = -G/L, whose values near the tile edge belong to
// other blocks.  Here every block computes G itself on its tile grown by the
// convolution halo c0 = (K-1)/2 (an extended region E of 64 columns; the
// output tile is the 64 - 2 c0 columns inside it), so the trial follows in
// the same pass: one launch and one memory round trip per iteration instead
// of two.  The stop test on ||G_k|| and the decrease test of trial k are
// taken at the start of the next pass, before any store, in the order the
// two-pass form takes them; a rejected trial recomputes G at the same point
// (the same values) with the doubled L.
//
// Per-pixel formulas are those of the two-pass kernels (the same staging,
// correlation order, TV terms and trial increments), so the iterates agree
// with the two-pass form to rounding: the partial sums run over this pass's
// own tiles, and the compiler may contract products differently here.
#pragma once
#include "kernels.cuh"

namespace maid {

template <int K> __host__ __device__ constexpr int step_c0() { return (K - 1) / 2; }
// output tile width and the rows per thread of the extended region
template <int K> __host__ __device__ constexpr int step_tw() { return kTW - 2 * step_c0<K>(); }
template <int K, int R> __host__ __device__ constexpr int step_re() { return R + (2 * step_c0<K>() + 3) / 4; }
template <int K, int R> __host__ __device__ constexpr int lds_apg_step() {
    return tv_rows(step_re<K, R>()) * tv_pitch() + fx_rows(step_re<K, R>()) * fx_pitch() +
           lds_conv(K, step_re<K, R>()) + tile_h(step_re<K, R>()) * cv_pitch(K);
}

// One FISTA iteration on the output tile of local block lb (see above).
// Per instance: reads sin, block 0 writes sout; partials pA (||G||^2) and pB
// (the decrease) have two halves of nbf entries, alternating by pass.  CO: the load policy (true in the team
// loops, where other blocks wrote the data during the kernel).
template <typename T, int K, int R, bool CO>
__device__ __forceinline__ void apg_step_body(const Inst<T>& I, int lb, ApgState& st, ApgState* __restrict__ sout,
                                              bool writer) {
    constexpr int c0 = step_c0<K>(), TWF = step_tw<K>(), RE = step_re<K, R>();
    constexpr int CP = cv_pitch(K), CRE = cv_rows(K, RE);
    constexpr int VP = tv_pitch(), VRE = tv_rows(RE), WP = fx_pitch(), WRE = fx_rows(RE);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* sm = reinterpret_cast<T*>(smem_raw);
    T* s_v = sm;                          // v on E grown by one pixel
    T* s_w = s_v + VRE * VP;              // TV weights of the flux sites of E
    T* s_r = s_w + WRE * WP;              // residual theta*v - y on E grown by c0 (later: x+ on E)
    T* s_g = s_r + CRE * CP;              // the step dl = -G/L on E

    const int H = I.pr.H, W = I.pr.W, reg = I.pr.reg;
    const int nbf = I.nbf;
    const int ntx = (W + TWF - 1) / TWF;
    const int t = xcd_tile(lb, nbf);
    const int ti0 = (t / ntx) * tile_h(R), tj0 = (t % ntx) * TWF;
    const int ei0 = ti0 - c0, ej0 = tj0 - c0;          // origin of E
    const int tx = threadIdx.x & 63, wv = threadIdx.x >> 6;

    // ---- decisions about the previous pass's gradient and trial; the
    // tiles of the point an acceptance moves to are loaded meanwhile
    // The pass reads the partials of the previous pass from one half of pA /
    // pB and writes its own to the other half (blocks that finish early
    // must not overwrite what later blocks still read).
    const bool start = st.phase == PH_START;
    const bool fresh = st.phase == PH_STEP_NEW;
    const double* __restrict__ rA = I.pA + (st.pp ? nbf : 0);
    const double* __restrict__ rB = I.pB + (st.pp ? nbf : 0);
    double* __restrict__ wA = I.pA + (st.pp ? 0 : nbf);
    double* __restrict__ wB = I.pB + (st.pp ? 0 : nbf);
    Partials pa, pb;
    if (fresh) pa = partials_issue<CO>(rA, nbf);
    if (!start) pb = partials_issue<CO>(rB, nbf);
    int cur = st.cur, prev = st.prev;
    double mnext = st.m, tnext = st.t;
    if (!start) {
        cur = st.nxt;
        prev = st.cur;
        tnext = 0.5 * (1.0 + sqrt(1.0 + 4.0 * st.t * st.t));
        mnext = (st.t - 1.0) / tnext;
    }
    // tile pixels of this thread: theta*x, theta*x_prev and y for the data part
    T kxr[R], kxpr[R], yr[R];
    auto stage_point = [&](int ci, int pi, T m) {
        const T* __restrict__ X = pick(I.X[0], I.X[1], I.X[2], ci);
        const T* __restrict__ XP = pick(I.X[0], I.X[1], I.X[2], pi);
        const T* __restrict__ KX = pick(I.KX[0], I.KX[1], I.KX[2], ci);
        const T* __restrict__ KXP = pick(I.KX[0], I.KX[1], I.KX[2], pi);
        const T* __restrict__ Y = I.y;
        auto rs = stage<CRE, CP, CP>(s_r, ei0 - c0, ej0 - c0, [&](int g) {
            const T kx = ld<CO>(KX, g);
            return dfma(m, kx - ld<CO>(KXP, g), kx) - ld<CO>(Y, g);
        });
        auto vs = stage<VRE, VP, VP>(s_v, ei0 - 1, ej0 - 1, [&](int g) {
            const T xv = ld<CO>(X, g);
            return dfma(m, xv - ld<CO>(XP, g), xv);
        });
        rs.fetch(H, W);
        vs.fetch(H, W);
#pragma unroll
        for (int o = 0; o < R; ++o) {
            const int e = clampi(ti0 + wv * R + o, H - 1) * W + clampi(tj0 + tx, W - 1);
            kxr[o] = ld<CO>(KX, e);
            kxpr[o] = ld<CO>(KXP, e);
            yr[o] = ld<CO>(Y, e);
        }
        rs.put();
        vs.put();
    };
    stage_point(cur, prev, (T)mnext);

    if (fresh) {
        const double gn2 = partials_finish<CO>(rA, nbf, pa);
        st.gn2 = gn2;
        st.nb_iter = 0;
        if (!finite_d(gn2)) {
            st.done = 1;
            st.status = ST_NONFINITE;
        } else if (sqrt(gn2) <= st.tol) {
            st.done = 1;
            st.status = ST_OK;
        } else if (st.iters >= st.max_iter) {
            st.done = 1;
            st.status = ST_MAXITER;
        }
    }
    bool moved = start;
    if (!st.done && !start) {
        const double delta = partials_finish<CO>(rB, nbf, pb);
        st.delta_last = delta;
        if (!finite_d(delta)) {
            st.done = 1;
            st.status = ST_NONFINITE;
        } else if (delta <= -st.gn2 / (2.0 * st.L)) {
            if (writer && I.trace && st.iters < st.trace_cap) I.trace[st.iters] = st.nb_iter;
            st.iters += 1;
            st.nxt = st.prev;
            st.prev = st.cur;
            st.cur = cur;
            st.t_prev = st.t;
            st.t = tnext;
            st.m = mnext;
            moved = true;
        } else {
            st.L = 2.0 * st.L;
            st.bt += 1;
            st.nb_iter += 1;
            if (st.nb_iter > 200) {
                st.done = 1;
                st.status = ST_NONFINITE;
            }
        }
    }
    if (!st.done) {
        st.phase = moved ? PH_STEP_NEW : PH_STEP_RETRY;
        st.pp ^= 1;
    }
    if (writer && sout) put_state(sout, st);
    if (st.done) return;
    if (!moved) {
        // rejected: the same point again (G is recomputed, the same values)
        __syncthreads();
        stage_point(st.cur, st.prev, (T)st.m);
    }
    __syncthreads();

    // ---- G on E: the gradient pass's arithmetic on a 64 x 4 RE tile at E
    const T alpha = (T)I.pr.alpha;
    const T ninvL = (T)(-1.0 / st.L);
    tv_weights<T, RE>(s_v, s_w, 1, reg, (T)(I.pr.eps_tv * I.pr.eps_tv), ei0, ej0, H, W);
    T acc[RE];
#pragma unroll
    for (int o = 0; o < RE; ++o) acc[o] = T(0);
    correlate<T, K, RE>(s_r, CP, I.th, wv * RE, tx, acc);
    __syncthreads();
    double gsq = 0.0;
    const int gj = ej0 + tx;
#pragma unroll
    for (int o = 0; o < RE; ++o) {
        const int li = wv * RE + o, gi = ei0 + li;
        const T g = dfma(alpha, tv_grad_px<T, RE>(s_v, s_w, 0, reg, li, tx, gi, gj, H, W), acc[o]);
        const bool in = inside(gi, gj, H, W);
        s_g[li * CP + tx] = in ? g * ninvL : T(0);
        // ||G||^2 over the output tile only (every pixel in exactly one tile)
        if (in && li >= c0 && li < c0 + tile_h(R) && tx >= c0 && tx < c0 + TWF) gsq += (double)g * (double)g;
    }
    __syncthreads();

    // ---- the trial step on the output tile (the trial pass's arithmetic)
    const T m = (T)st.m;
    const double e2 = I.pr.eps_tv * I.pr.eps_tv;
    const int li0 = wv * R, oj = tj0 + tx;
    const bool lane_in = tx < TWF;
    double dtv = 0.0;
#pragma unroll
    for (int o = 0; o < R; ++o) {
        const int gi = ti0 + li0 + o;
        if (lane_in && gi < H && oj < W) {
            const int iv = (li0 + o + c0 + 1) * VP + tx + c0 + 1;
            const int ig = (li0 + o + c0) * CP + tx + c0;
            const bool hx = oj < W - 1, vx = gi < H - 1;
            const double bh = hx ? (double)(s_v[iv + 1] - s_v[iv]) : 0.0;
            const double bv = vx ? (double)(s_v[iv + VP] - s_v[iv]) : 0.0;
            const double ah = hx ? (double)(s_g[ig + 1] - s_g[ig]) : 0.0;
            const double av = vx ? (double)(s_g[ig + CP] - s_g[ig]) : 0.0;
            if (reg == 2) {
                dtv += ah * (bh + 0.5 * ah) + av * (bv + 0.5 * av);
            } else {
                // one channel: the coupled and the channelwise magnitudes agree
                const double d2 = ah * (ah + 2.0 * bh) + av * (av + 2.0 * bv);
                const double q2 = bh * bh + bv * bv;
                dtv += d2 / (sqrt(q2 + d2 + e2) + sqrt(q2 + e2));
            }
        }
    }
    T dacc[R];
#pragma unroll
    for (int o = 0; o < R; ++o) dacc[o] = T(0);
    correlate<T, K, R>(s_g, CP, I.thf, li0, tx, dacc);
    const bool exact = st.resync > 0 && (st.iters % st.resync) < 2;
    T* __restrict__ XN = pick(I.X[0], I.X[1], I.X[2], st.nxt);
    T* __restrict__ KXN = pick(I.KX[0], I.KX[1], I.KX[2], st.nxt);
    double ddat = 0.0;
#pragma unroll
    for (int o = 0; o < R; ++o) {
        const int gi = ti0 + li0 + o;
        if (lane_in && gi < H && oj < W) {
            const int e = gi * W + oj;
            const T kv = dfma(m, kxr[o] - kxpr[o], kxr[o]);
            const T d = dacc[o];
            const double rv = (double)kv - (double)yr[o];
            ddat += (double)d * (rv + 0.5 * (double)d);
            at(XN, e) = s_v[(li0 + o + c0 + 1) * VP + tx + c0 + 1] + s_g[(li0 + o + c0) * CP + tx + c0];
            if (!exact) at(KXN, e) = kv + d;
        }
    }
    if (exact) {
        // theta*x+ from x+ = v + dl on E (zero outside the image)
        T* s_x = s_r;
        __syncthreads();
        for (int idx = threadIdx.x; idx < tile_h(RE) * kTW; idx += kNT) {
            const int r = idx / kTW, cc = idx - r * kTW;
            s_x[r * CP + cc] = s_v[(r + 1) * VP + cc + 1] + s_g[r * CP + cc];
        }
        __syncthreads();
#pragma unroll
        for (int o = 0; o < R; ++o) dacc[o] = T(0);
        correlate<T, K, R>(s_x, CP, I.thf, li0, tx, dacc);
#pragma unroll
        for (int o = 0; o < R; ++o) {
            const int gi = ti0 + li0 + o;
            if (lane_in && gi < H && oj < W) at(KXN, gi * W + oj) = dacc[o];
        }
    }
    block_partial(gsq, wA, lb);
    block_partial(ddat + I.pr.alpha * dtv, wB, lb);
}

// One-pass FISTA launch over a group: block b -> (instance, local block) via
// the group's step map (blocks of an instance start at a multiple of 8).
template <typename T, int K, int R>
__global__ __launch_bounds__(kNT) void k_apg_step(const Inst<T>* __restrict__ insts, const int* __restrict__ blk,
                                                  int only, const ApgState* __restrict__ sin,
                                                  ApgState* __restrict__ sout) {
    const int ii = only >= 0 ? only : blk[blockIdx.x];
    const Inst<T>& I = insts[ii];
    const int lb = (int)blockIdx.x - I.basef;
    if (lb >= I.nbf) return;
    ApgState st = sin[ii];
    const bool writer = lb == 0 && threadIdx.x == 0;
    if (st.done) {
        if (writer) put_state(&sout[ii], st);
        return;
    }
    apg_step_body<T, K, R, false>(I, lb, st, &sout[ii], writer);
}

}  // namespace maid
