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
// Blocks have kStepNW = 8 waves, one tile row per wave and row of a thread:
// an output tile of 8 R rows needs 8 R + 2 c0 rows of G, so the recomputed
// halo costs less per output pixel than with the 4-wave blocks of the
// two-pass kernels, and a 256 x 256 image takes 160 blocks (one per CU)
// instead of 320 (where a CU holding two blocks finishes last).
//
// Per-pixel formulas are those of the two-pass kernels (the same staging,
// correlation order, TV terms and trial increments), so the iterates agree
// with the two-pass form to rounding: the partial sums run over this pass's
// own tiles, and the compiler may contract products differently here.
#pragma once
#include "kernels.cuh"

namespace maid {

template <int K> __host__ __device__ constexpr int step_c0() { return (K - 1) / 2; }
// Blocks of kStepNW waves: a tile of r rows per thread is kStepNW r rows tall
// (the v tile two rows more, the flux sites one row more, a convolution
// input K - 1 rows more).
__host__ __device__ constexpr int step_th(int r) { return kStepNW * r; }
__host__ __device__ constexpr int step_tv_rows(int r) { return step_th(r) + 2; }
__host__ __device__ constexpr int step_fx_rows(int r) { return step_th(r) + 1; }
__host__ __device__ constexpr int step_cv_rows(int K, int r) { return step_th(r) + K - 1; }
// output tile width and the rows per thread of the extended region
template <int K> __host__ __device__ constexpr int step_tw() { return kTW - 2 * step_c0<K>(); }
template <int K, int R> __host__ __device__ constexpr int step_re() {
    return R + (2 * step_c0<K>() + kStepNW - 1) / kStepNW;
}
template <int K, int R> __host__ __device__ constexpr int lds_apg_step() {
    return step_tv_rows(step_re<K, R>()) * tv_pitch() + step_fx_rows(step_re<K, R>()) * fx_pitch() +
           step_cv_rows(K, step_re<K, R>()) * cv_pitch(K) + step_th(step_re<K, R>()) * cv_pitch(K);
}

// One FISTA iteration on the output tile of local block lb (see above).
// Per instance: reads sin, block 0 writes sout; partials pA (||G||^2) and pB
// (the decrease) have two halves of nbf entries, alternating by pass.  CO: the load policy (true in the team
// loops, where other blocks wrote the data during the kernel).
template <typename T, int K, int R, bool CO>
__device__ __forceinline__ void apg_step_body(const Inst<T>& I, int lb, ApgState& st, ApgState* __restrict__ sout,
                                              bool writer) {
    constexpr int c0 = step_c0<K>(), TWF = step_tw<K>(), RE = step_re<K, R>();
    constexpr int CP = cv_pitch(K), CRE = step_cv_rows(K, RE);
    constexpr int VP = tv_pitch(), VRE = step_tv_rows(RE), WP = fx_pitch(), WRE = step_fx_rows(RE);
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
    const int ti0 = (t / ntx) * step_th(R), tj0 = (t % ntx) * TWF;
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
    // wave 0 alone reads and adds the partials
    Partials pa, pb;
    if (wv == 0) {
        if (fresh) pa = partials_issue<CO, 64>(rA, nbf);
        if (!start) pb = partials_issue<CO, 64>(rB, nbf);
    }
    int cur = st.cur, prev = st.prev;
    double mnext = st.m, tnext = st.t;
    if (!start) {
        cur = st.nxt;
        prev = st.cur;
        tnext = st.fixed ? 1.0 : 0.5 * (1.0 + sqrt(1.0 + 4.0 * st.t * st.t));
        mnext = st.fixed ? 0.0 : (st.t - 1.0) / tnext;
    }
    // tile pixels of this thread: the residuals theta*x - y at x and x_prev
    T kxr[R], kxpr[R];
    auto stage_point = [&](int ci, int pi, T m) {
        const T* __restrict__ X = pick(I.X[0], I.X[1], I.X[2], ci);
        const T* __restrict__ XP = pick(I.X[0], I.X[1], I.X[2], pi);
        const T* __restrict__ KX = pick(I.KX[0], I.KX[1], I.KX[2], ci);
        const T* __restrict__ KXP = pick(I.KX[0], I.KX[1], I.KX[2], pi);
        auto rs = stage<CRE, CP, CP, kStepNT>(s_r, ei0 - c0, ej0 - c0, [&](int g) {
            const T kx = ld<CO>(KX, g);
            return dfma(m, kx - ld<CO>(KXP, g), kx);
        });
        auto vs = stage<VRE, VP, VP, kStepNT>(s_v, ei0 - 1, ej0 - 1, [&](int g) {
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
        }
        warm_taps<T, K>(I.th, I.thf);
        rs.put();
        vs.put();
    };
    stage_point(cur, prev, (T)mnext);

    // both sums of the previous pass with one pair of barriers
    double gn2 = 0.0, delta = 0.0;
    if (wv == 0) {
        gn2 = fresh ? partials_local<CO, 64>(rA, nbf, pa) : 0.0;
        delta = start ? 0.0 : partials_local<CO, 64>(rB, nbf, pb);
    }
    wave0_share2(gn2, delta);
    if (fresh) {
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
        st.delta_last = delta;
        if (!finite_d(delta)) {
            st.done = 1;
            st.status = ST_NONFINITE;
        } else if (st.fixed || delta <= -st.gn2 / (2.0 * st.L)) {
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

    // ---- G on E: the gradient pass's arithmetic on a 64 x (kStepNW RE) tile at E
    const T alpha = (T)I.pr.alpha;
    const T ninvL = (T)(-1.0 / st.L);
    tv_weights_h<T, step_th(RE), kStepNT>(s_v, s_w, 1, reg, (T)(I.pr.eps_tv * I.pr.eps_tv), ei0, ej0, H, W);
    T acc[RE];
#pragma unroll
    for (int o = 0; o < RE; ++o) acc[o] = T(0);
    correlate<T, K, RE>(s_r, CP, I.th, wv * RE, tx, acc);
    __syncthreads();
    double gsq = 0.0;
    const int gj = ej0 + tx;
    // all rows' LDS reads before the first LDS store
    T gv[RE];
#pragma unroll
    for (int o = 0; o < RE; ++o) {
        const int li = wv * RE + o, gi = ei0 + li;
        gv[o] = dfma(alpha, tv_grad_px_h<T, step_th(RE)>(s_v, s_w, 0, reg, li, tx, gi, gj, H, W), acc[o]);
    }
#pragma unroll
    for (int o = 0; o < RE; ++o) {
        const int li = wv * RE + o, gi = ei0 + li;
        const T g = gv[o];
        const bool in = inside(gi, gj, H, W);
        s_g[li * CP + tx] = in ? g * ninvL : T(0);
        // ||G||^2 over the output tile only (every pixel in exactly one tile)
        if (in && li >= c0 && li < c0 + step_th(R) && tx >= c0 && tx < c0 + TWF) gsq += (double)g * (double)g;
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
        // every lane reads (inside the staged tiles) and computes; lanes
        // outside the output tile or the image add nothing
        const int gi = ti0 + li0 + o;
        const bool px = lane_in && gi < H && oj < W;
        const int iv = (li0 + o + c0 + 1) * VP + tx + c0 + 1;
        const int ig = (li0 + o + c0) * CP + tx + c0;
        const bool hx = oj < W - 1, vx = gi < H - 1;
        const double bh = keep(hx, (double)(s_v[iv + 1] - s_v[iv]));
        const double bv = keep(vx, (double)(s_v[iv + VP] - s_v[iv]));
        const double ah = keep(hx, (double)(s_g[ig + 1] - s_g[ig]));
        const double av = keep(vx, (double)(s_g[ig + CP] - s_g[ig]));
        double term;
        if (reg == 2) {
            term = ah * (bh + 0.5 * ah) + av * (bv + 0.5 * av);
        } else {
            // one channel: the coupled and the channelwise magnitudes agree
            const double d2 = ah * (ah + 2.0 * bh) + av * (av + 2.0 * bv);
            const double q2 = bh * bh + bv * bv;
            term = d2 / (sqrt(q2 + d2 + e2) + sqrt(q2 + e2));
        }
        dtv = px ? dtv + term : dtv;
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
            ddat += (double)d * ((double)kv + 0.5 * (double)d);
            at(XN, e) = s_v[(li0 + o + c0 + 1) * VP + tx + c0 + 1] + s_g[(li0 + o + c0) * CP + tx + c0];
            if (!exact) at(KXN, e) = kv + d;
        }
    }
    if (exact) {
        // the residual at x+ = v + dl (formed on E, zero outside the image):
        // in full, theta*x+ - y with FP64 taps and sums, x+ becoming the base
        // point; otherwise r_base + theta*(x+ - x_base)
        const bool full = st.resync_full > 0 && (st.iters % st.resync_full) == 0;
        T* __restrict__ XB = I.xb;
        T* __restrict__ RB = I.rb;
        const T* __restrict__ Y = I.y;
        T* s_x = s_r;
        __syncthreads();
        for (int idx = threadIdx.x; idx < step_th(RE) * kTW; idx += kStepNT) {
            const int r = idx / kTW, cc = idx - r * kTW;
            const int gi = ei0 + r, gj = ej0 + cc;
            const T xb = (full || !inside(gi, gj, H, W)) ? T(0) : ld<CO>(XB, clampi(gi, H - 1) * W + clampi(gj, W - 1));
            s_x[r * CP + cc] = (s_v[(r + 1) * VP + cc + 1] + s_g[r * CP + cc]) - xb;
        }
        __syncthreads();
        if (full) {
            double a64[R];
#pragma unroll
            for (int o = 0; o < R; ++o) a64[o] = 0.0;
            correlate64<T, K, R>(s_x, CP, I.theta64, true, li0, tx, a64);
#pragma unroll
            for (int o = 0; o < R; ++o) {
                const int gi = ti0 + li0 + o;
                if (lane_in && gi < H && oj < W) {
                    const int e = gi * W + oj;
                    const T r = (T)(a64[o] - (double)ld<CO>(Y, e));
                    at(KXN, e) = r;
                    at(RB, e) = r;
                    at(XB, e) = s_x[(li0 + o + c0) * CP + tx + c0];
                }
            }
        } else {
#pragma unroll
            for (int o = 0; o < R; ++o) dacc[o] = T(0);
            correlate<T, K, R>(s_x, CP, I.thf, li0, tx, dacc);
#pragma unroll
            for (int o = 0; o < R; ++o) {
                const int gi = ti0 + li0 + o;
                if (lane_in && gi < H && oj < W) {
                    const int e = gi * W + oj;
                    at(KXN, e) = ld<CO>(RB, e) + dacc[o];
                }
            }
        }
    }
    block_partial2_1<kStepNW>(gsq, wA, ddat + I.pr.alpha * dtv, wB, lb);
}

// One-pass FISTA launch over a group: block b -> (instance, local block) via
// the group's step map (blocks of an instance start at a multiple of 8).
template <typename T, int K, int R>
__global__ __launch_bounds__(kStepNT) void k_apg_step(const Inst<T>* __restrict__ insts, const int* __restrict__ blk,
                                                  int only, const ApgState* __restrict__ sin,
                                                  ApgState* __restrict__ sout) {
    const int ii = only >= 0 ? only : blk[blockIdx.x];
    const Inst<T>& I = insts[ii];
    const int lb = (int)blockIdx.x - I.basef;
    if ((unsigned)lb >= (unsigned)I.nbf) return;
    ApgState st = sin[ii];
    const bool writer = lb == 0 && threadIdx.x == 0;
    if (st.done) {
        if (writer) put_state(&sout[ii], st);
        return;
    }
    apg_step_body<T, K, R, false>(I, lb, st, &sout[ii], writer);
}

// ------------------------------------------------------------------ one-pass CG
// The adjoint solve of Algorithm 1 in the Chronopoulos-Gear form of conjugate
// gradients: with w = H r kept next to r, the two inner products of an
// iteration (gamma = <r,r>, delta = <r,w>) come from one reduction, and
//   beta_i = gamma_i / gamma_{i-1},  a_i = gamma_i / (delta_i - beta_i gamma_i / a_{i-1}),
//   p_i = r_i + beta_i p_{i-1},  s_i = w_i + beta_i s_{i-1}  (s = H p),
//   q += a_i p_i,  r_{i+1} = r_i - a_i s_i,  w_{i+1} = H r_{i+1};
// in exact arithmetic these are the iterates of the Hestenes-Stiefel form
// (the denominator of a_i is <p_i, H p_i>, tested for positivity as there).
// One pass per iteration: every block forms r_{i+1} on its tile grown by 2 c0
// from r_i, w_i, s_{i-1} (the same arithmetic as the block that owns those
// pixels), the convolution u = theta*r_{i+1} on the tile grown by c0 (the
// region E of the one-pass FISTA form), and then H r_{i+1} = theta.u +
// alpha grad^2 R(xt)[r_{i+1}] on the tile.  r, w and s (FP64) alternate
// between two buffers (blocks read their neighbours' old values while
// writing new ones);
// the partials of gamma and delta alternate between the halves of pR and pK.
// st.first: 2 = the priming pass (w_0 = H r_0 and the first sums, nothing
// else), 1 = the first iteration (beta = 0), 0 after; st.pc: the buffer set
// the pass reads.
template <int K, int R> __host__ __device__ constexpr int lds_cg_step() {
    return step_cv_rows(K, step_re<K, R>()) * cv_pitch(K) + step_th(step_re<K, R>()) * cv_pitch(K) +
           2 * step_tv_rows(R) * tv_pitch() + 2 * step_fx_rows(R) * fx_pitch();
}

template <typename T, int K, int R, bool CO>
__device__ __forceinline__ void cg_step_body(const Inst<T>& I, int lb, CgState& st, CgState* __restrict__ sout,
                                             bool writer) {
    constexpr int c0 = step_c0<K>(), TWF = step_tw<K>(), RE = step_re<K, R>();
    constexpr int CP = cv_pitch(K), CRE = step_cv_rows(K, RE);
    constexpr int VP = tv_pitch(), VR = step_tv_rows(R), WP = fx_pitch(), WR = step_fx_rows(R);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* sm = reinterpret_cast<T*>(smem_raw);
    T* s_rn = sm;                         // r_{i+1} on the tile grown by 2 c0
    T* s_u = s_rn + CRE * CP;             // u = theta * r_{i+1} on E
    T* s_x = s_u + step_th(RE) * CP;       // xt, tile grown by one pixel
    T* s_p = s_x + VR * VP;               // r_{i+1}, tile grown by one pixel
    T* s_w = s_p + VR * VP;               // TV weights w and w^3 <Dx, Dr> of the flux sites
    T* s_mw = s_w + WR * WP;

    const int H = I.pr.H, W = I.pr.W, reg = I.pr.reg;
    const int nbf = I.nbf;
    const int ntx = (W + TWF - 1) / TWF;
    const int t = xcd_tile(lb, nbf);
    const int ti0 = (t / ntx) * step_th(R), tj0 = (t % ntx) * TWF;
    const int ei0 = ti0 - c0, ej0 = tj0 - c0;
    const int tx = threadIdx.x & 63, wv = threadIdx.x >> 6;

    const bool prime = st.first == 2, first = st.first == 1;
    const int par = st.pc;
    const T* __restrict__ Rb = pick(I.r, I.Kp, par);
    const T* __restrict__ Wb = pick(I.Hp, I.V[0], par);
    const double* __restrict__ Sb = pick(I.S64[0], I.S64[1], par);
    T* __restrict__ Pv = I.V[1];
    T* __restrict__ Qv = I.q;
    const T* __restrict__ Xt = I.xt;
    const double* __restrict__ rG = I.pR + (par ? nbf : 0);
    const double* __restrict__ rD = I.pK + (par ? nbf : 0);
    Partials pg, pd;
    if (!prime) {
        if (wv == 0) {
            pg = partials_issue<CO, 64>(rG, nbf);
            pd = partials_issue<CO, 64>(rD, nbf);
        }
    }
    // the tile pixels' own values, loaded with the staging
    T rr[R], wr[R], pr_[R], qr[R];
    double sr[R];
#pragma unroll
    for (int o = 0; o < R; ++o) {
        const int e = clampi(ti0 + wv * R + o, H - 1) * W + clampi(tj0 + tx, W - 1);
        rr[o] = ld<CO>(Rb, e);
        wr[o] = ld<CO>(Wb, e);
        sr[o] = ld<CO>(Sb, e);
        pr_[o] = ld<CO>((const T*)Pv, e);
        qr[o] = ld<CO>((const T*)Qv, e);
    }
    auto xs = stage<VR, VP, VP, kStepNT>(s_x, ti0 - 1, tj0 - 1, [&](int g) { return ld<CO>(Xt, g); });
    xs.fetch(H, W);
    warm_taps<T, K>(I.th, I.thf);

    double a = 0.0, beta = 0.0;
    if (!prime) {
        double g = 0.0, d = 0.0;
        if (wv == 0) {
            g = partials_local<CO, 64>(rG, nbf, pg);
            d = partials_local<CO, 64>(rD, nbf, pd);
        }
        wave0_share2(g, d);
        beta = first ? 0.0 : g / st.gamma;
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
        } else {
            const double den = first ? d : d - beta * g / st.a;
            st.kappa = den;
            if (!(den > 0.0) || !finite_d(den)) {
                st.done = 1;
                st.status = finite_d(den) ? ST_NOT_SPD : ST_NONFINITE;
            } else {
                a = g / den;
                st.a = a;
                st.iters += 1;
                st.first = 0;
                st.pc = par ^ 1;
            }
        }
    } else {
        st.first = 1;
    }
    if (writer && sout) put_state(sout, st);
    if (st.done) return;

    // r_{i+1} on the tile grown by 2 c0 (zero outside the image); s_i = w_i +
    // beta s_{i-1} and r_{i+1} = r_i - a s_i by the same expressions as below.
    // s is a recurrence (the Hestenes-Stiefel form recomputes Hp instead), so
    // it is carried in FP64 whatever the storage type: stored in FP32 its
    // rounding accumulates into r and the iterates drift from that form.
    const T aT = (T)a, bT = (T)beta;
    auto snext = [&](T w, double s) { return first ? (double)w : dfma(beta, s, (double)w); };
    auto rnext = [&](T r, T w, double s) { return (T)dfma(-a, snext(w, s), (double)r); };
    if (prime) {
        load_tile<CRE, CP, CP, kStepNT>(s_rn, ei0 - c0, ej0 - c0, H, W, [&](int g) { return ld<CO>(Rb, g); });
    } else {
        load_tile<CRE, CP, CP, kStepNT>(s_rn, ei0 - c0, ej0 - c0, H, W,
                               [&](int g) { return rnext(ld<CO>(Rb, g), ld<CO>(Wb, g), ld<CO>(Sb, g)); });
    }
    xs.put();
    __syncthreads();
    // u = theta * r_{i+1} on E (the direction pass's convolution), r_{i+1} on
    // the tile grown by one pixel for the TV term
    T acc[RE];
#pragma unroll
    for (int o = 0; o < RE; ++o) acc[o] = T(0);
    correlate<T, K, RE>(s_rn, CP, I.thf, wv * RE, tx, acc);
#pragma unroll
    for (int o = 0; o < RE; ++o) {
        const int li = wv * RE + o;
        s_u[li * CP + tx] = inside(ei0 + li, ej0 + tx, H, W) ? acc[o] : T(0);
    }
    for (int idx = threadIdx.x; idx < VR * VP; idx += kStepNT) {
        const int r = idx / VP, cc = idx - r * VP;
        s_p[idx] = s_rn[(r + 2 * c0 - 1) * CP + cc + 2 * c0 - 1];
    }
    __syncthreads();
    // TV weights of the flux sites (the Hessian pass's arithmetic, one channel)
    const T eps2 = (T)(I.pr.eps_tv * I.pr.eps_tv);
    constexpr int NS = WR * WP, ITS = (NS + kStepNT - 1) / kStepNT;
    // unrolled over the thread's sites with a clamped site index for the
    // reads, all reads before all stores
    T wk[ITS], mk[ITS];
#pragma unroll
    for (int k = 0; k < ITS; ++k) {
        const int idx = threadIdx.x + k * kStepNT;
        const int ic = idx < NS ? idx : NS - 1;
        const int r = ic / WP, cc = ic - r * WP;
        const int gi = ti0 - 1 + r, gj2 = tj0 - 1 + cc;
        const bool in = inside(gi, gj2, H, W);
        const bool hx = gj2 < W - 1, vx = gi < H - 1;
        const int i0 = r * VP + cc;
        const T xh = keep(hx, s_x[i0 + 1] - s_x[i0]);
        const T xv = keep(vx, s_x[i0 + VP] - s_x[i0]);
        const T ph = keep(hx, s_p[i0 + 1] - s_p[i0]);
        const T pv = keep(vx, s_p[i0 + VP] - s_p[i0]);
        const T s2 = xh * xh + xv * xv, mm = xh * ph + xv * pv;
        if (reg == 2) {
            wk[k] = in ? T(1) : T(0);
            mk[k] = T(0);
        } else {
            const T w = in ? drsqrt(s2 + eps2) : T(0);
            wk[k] = w;
            mk[k] = w * w * w * mm;
        }
    }
#pragma unroll
    for (int k = 0; k < ITS; ++k) {
        const int idx = threadIdx.x + k * kStepNT;
        if (idx < NS) {
            s_w[idx] = wk[k];
            s_mw[idx] = mk[k];
        }
    }
    T hacc[R];
#pragma unroll
    for (int o = 0; o < R; ++o) hacc[o] = T(0);
    correlate<T, K, R>(s_u, CP, I.th, wv * R, tx, hacc);
    __syncthreads();

    // w_{i+1} = theta.u + alpha grad^2 R(xt)[r_{i+1}] on the tile; the updates
    const T alpha = (T)I.pr.alpha;
    const int li0 = wv * R, oj = tj0 + tx;
    const bool lane_in = tx < TWF;
    const int wsel = prime ? par : par ^ 1;
    T* __restrict__ Rn = pick(I.r, I.Kp, wsel);
    T* __restrict__ Wn = pick(I.Hp, I.V[0], wsel);
    double* __restrict__ Sn = pick(I.S64[0], I.S64[1], wsel);
    double gs = 0.0, ds = 0.0;
#pragma unroll
    for (int o = 0; o < R; ++o) {
        const int gi = ti0 + li0 + o;
        // the Hessian term from LDS for every lane (the reads stay inside
        // the staged tiles), the stores for the output pixels only
        const int r = li0 + o + 1, cc = tx + 1;
        const int i0 = r * VP + cc;
        const T xh_h = keep(oj < W - 1, s_x[i0 + 1] - s_x[i0]);
        const T ph_h = keep(oj < W - 1, s_p[i0 + 1] - s_p[i0]);
        const T xv_h = keep(gi < H - 1, s_x[i0 + VP] - s_x[i0]);
        const T pv_h = keep(gi < H - 1, s_p[i0 + VP] - s_p[i0]);
        const T xh_l = s_x[i0] - s_x[i0 - 1], ph_l = s_p[i0] - s_p[i0 - 1];
        const T xv_u = s_x[i0] - s_x[i0 - VP], pv_u = s_p[i0] - s_p[i0 - VP];
        const int f0 = r * WP + cc, fl = f0 - 1, fu = f0 - WP;
        const T fh_here = s_w[f0] * ph_h - s_mw[f0] * xh_h;
        const T fv_here = s_w[f0] * pv_h - s_mw[f0] * xv_h;
        const T fh_left = s_w[fl] * ph_l - s_mw[fl] * xh_l;
        const T fv_up = s_w[fu] * pv_u - s_mw[fu] * xv_u;
        const T hv = fh_left - fh_here + fv_up - fv_here;
        const T rn = s_p[i0];
        if (lane_in && gi < H && oj < W) {
            const T wn = dfma(alpha, hv, hacc[o]);
            const int e = gi * W + oj;
            at(Wn, e) = wn;
            if (!prime) {
                const T pi = first ? rr[o] : dfma(bT, pr_[o], rr[o]);
                const double si = snext(wr[o], sr[o]);
                at(Pv, e) = pi;
                at(Sn, e) = si;
                at(Qv, e) = dfma(aT, pi, qr[o]);
                at(Rn, e) = rn;
            }
            gs += (double)rn * (double)rn;
            ds += (double)rn * (double)wn;
        }
    }
    double* __restrict__ wG = I.pR + (wsel ? nbf : 0);
    double* __restrict__ wD = I.pK + (wsel ? nbf : 0);
    block_partial2_1<kStepNW>(gs, wG, ds, wD, lb);
}

template <typename T, int K, int R>
__global__ __launch_bounds__(kStepNT) void k_cg_step(const Inst<T>* __restrict__ insts, const int* __restrict__ blk, int only,
                                                 const CgState* __restrict__ sin, CgState* __restrict__ sout) {
    const int ii = only >= 0 ? only : blk[blockIdx.x];
    const Inst<T>& I = insts[ii];
    const int lb = (int)blockIdx.x - I.basef;
    if ((unsigned)lb >= (unsigned)I.nbf) return;
    CgState st = sin[ii];
    const bool writer = lb == 0 && threadIdx.x == 0;
    if (st.done) {
        if (writer) put_state(&sout[ii], st);
        return;
    }
    cg_step_body<T, K, R, false>(I, lb, st, &sout[ii], writer);
}

}  // namespace maid
