// devctx.h -- data shared by the host control code and the kernels of
// libmaid: the per-instance table every pass reads, the solver states, and
// the LDS sizing rules.
//
// A context holds one or more problem instances (a batch of ragged images).
// Each pass launch covers the tiles of a group of instances with the same
// kernel size K and tile height: a block looks up its instance in a
// block -> instance map, reads that instance's entry of the table (pointers,
// sizes, parameters; read-only in kernels, so scalar loads) and its solver
// state.  Solver states are kept in separate arrays (two copies for the
// lower-level solver, three for CG, one element per instance): a pass reads
// one copy through a const __restrict__ pointer and its block 0 of each
// instance writes the next copy, so every block of a launch sees the same
// state.  A plain solve is a batch of one.
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>

namespace maid {

constexpr int kMaxC = 3;       // colour channels supported by the LDS tiles
constexpr int kMaxK = 31;      // largest odd kernel size
constexpr int kTW = 64;        // tile width: one wave64 spans a tile row
constexpr int kNT = 256;       // threads per block (4 waves)
constexpr int kStepNW = 8;     // waves per block of the one-pass forms (a tile row per wave)
constexpr int kStepNT = 64 * kStepNW;

enum Status : int32_t { ST_OK = 0, ST_MAXITER = 1, ST_NOT_SPD = -4, ST_NONFINITE = -5 };

// Lower-level (FISTA) solver state, one per instance, in two arrays: the
// gradient pass reads the first and its block 0 of each instance writes the
// second; the trial pass reads the second and writes the first.  No kernel
// writes the copy it reads, so every block of a launch sees the same state.
// (PH_STEP_*: the one-pass form -- the last pass computed G and a trial at a
// new point, or again at the same point after a rejection.)
enum ApgPhase : int32_t {
    PH_START = 0, PH_GRAD_READY = 1, PH_RETRY = 2, PH_TRIALED = 3, PH_STEP_NEW = 4, PH_STEP_RETRY = 5
};

struct ApgState {
    double L, t, t_prev, m;      // Lipschitz estimate, momentum sequence, m = (t_prev-1)/t
    double gn2;                  // ||G||^2 at the current extrapolated point
    double tol;                  // stop when ||G|| <= tol
    double delta_last;           // last h(x+) - h(v)
    int32_t max_iter, iters, bt, nb_iter;
    int32_t status, done, phase;
    int32_t cur, prev, nxt;      // rotation of the three x / Kx buffers
    int32_t trace_cap;
    int32_t resync;              // theta*x - y recomputed when iters % resync < 2 (0: never)
    int32_t resync_full;         // ... from theta*x+ - y in FP64 (taps and sums), moving the base
                                 // point there, when iters % resync_full == 0; else as
                                 // theta*(x+ - x_base) + r_base (0: never)
    int32_t pp;                  // one-pass form: half of pA / pB the last pass wrote its partials to
    int32_t fixed;               // fixed-step gradient descent (Section 4.1's baselines): no
                                 // momentum (m = 0) and every trial accepted, L = 1/step
};

// CG state, one per instance, in three arrays: the direction pass reads the
// first and writes the second, the Hessian pass second -> third, the update
// pass third -> first.
struct CgState {
    double gamma, kappa, a, tol;
    int32_t max, iters, status, done, pc, first;
};

// Control block of a team launch (the persistent solver loops for small
// instances): one team of P blocks per XCD.
constexpr int kTeamMax = 128;    // members per team
constexpr int kTeamXcd = 8;      // teams per launch (XCDs)
struct TeamCtl {
    uint64_t* arrive;     // kTeamXcd x kTeamMax arrival words, never reset
    unsigned* err;        // nonzero once a member gave up waiting
    uint64_t epoch;       // (launch number) << 32: arrival words only grow
    int32_t P;            // members per team
    int64_t wait;         // wall-clock ticks a member waits at most
};

// Problem parameters the kernels need (part of the instance table, which
// kernels only read, so they come in through scalar loads).
struct Params {
    int32_t C, H, W, reg;
    double alpha, eps_tv;
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

// The convolution tile's LDS region, in elements of the storage type (esz
// bytes).  FP32 passes with 13 <= K <= 31 and 4 or 8 rows per thread may
// correlate on the matrix cores, which write the tile's FP16 halves (two
// tiles of pitch mf_p16 halfs) and then the waves' partial sums (two planes
// of tile_h x 68 floats) over the staged tile, so their region is the
// largest of the three.
__host__ __device__ constexpr int mf_p16(int K) { return 48 + ((K + 15) + 7) / 8 * 8 + 8; }
__host__ __device__ constexpr bool mf_tile(int K, int R, int esz) {
    return esz == 4 && K >= 13 && K <= 31 && (R == 4 || R == 8);
}
__host__ __device__ constexpr int lds_conv(int K, int R, int esz) {
    return mf_tile(K, R, esz) ? cmax(cmax(cv_rows(K, R) * cv_pitch(K), cv_rows(K, R) * mf_p16(K)), 2 * tile_h(R) * 68)
                              : cv_rows(K, R) * cv_pitch(K);
}
// Kernels of 5 taps and more: the passes stage the TV tiles and the
// convolution tile one after the other in one LDS region, which leaves room
// for more blocks per CU and for tiles of 8 rows per thread (at 2048x2048x3
// and 4096x4096, K = 5..11, a FISTA + CG iteration takes 1.2-1.8x less time
// than with every tile staged at once, with bitwise the same results).
// K <= 3: all tiles are staged at once, side by side.
__host__ __device__ constexpr bool seq_lds(int K) { return K >= 5; }
__host__ __device__ constexpr int lds_side(bool seq, int a, int b) { return seq ? cmax(a, b) : a + b; }
__host__ __device__ constexpr int lds_apg_grad(int K, int R, int C, int nw, int esz) {
    // sequential staging parks the TV gradient of each output past the tile region
    return lds_side(seq_lds(K), C * tv_rows(R) * tv_pitch() + nw * fx_rows(R) * fx_pitch(), lds_conv(K, R, esz)) +
           (seq_lds(K) ? R * 256 : 0);
}
__host__ __device__ constexpr int lds_apg_trial(int K, int R, int C, int esz) {
    // small kernels also stage v and the step of every channel for the TV decrease
    return seq_lds(K) ? lds_conv(K, R, esz) : lds_conv(K, R, esz) + 2 * C * tv_rows(R) * tv_pitch();
}
__host__ __device__ constexpr int lds_cg_hvp(int K, int R, int C, int nw, int esz) {
    // small kernels: the Kp tile, x and p of every channel, two weight planes;
    // large kernels: x, p of one channel and the weight planes, then the Kp
    // tile in the same region, plus a park for the TV term and p of each
    // output (2 R values per thread)
    return seq_lds(K) ? cmax(2 * tv_rows(R) * tv_pitch() + 2 * fx_rows(R) * fx_pitch(), lds_conv(K, R, esz)) +
                            2 * R * 256
                      : lds_conv(K, R, esz) + 2 * C * tv_rows(R) * tv_pitch() + 2 * fx_rows(R) * fx_pitch();
}
__host__ __device__ constexpr int lds_cg_dir(int K, int R, int esz) {
    return seq_lds(K) ? lds_conv(K, R, esz) : 2 * lds_conv(K, R, esz);
}

// ------------------------------------------------------------------ instance table
// Every table pointer is a global-memory pointer: in the device pass it
// carries the global address space, so loads and stores through it (and
// through pointers derived from it) compile to global (not flat) memory
// instructions, and uniform loads of read-only data to scalar loads.  The
// host pass sees plain pointers of the same size.
#if defined(__HIP_DEVICE_COMPILE__)
#define MAID_GLOBAL __attribute__((address_space(1)))
#else
#define MAID_GLOBAL
#endif
template <typename T> using gp = T MAID_GLOBAL*;

template <typename T> struct Inst {
    Params pr;                   // C, H, W, reg, alpha, eps_tv
    int32_t K;                   // kernel size
    int32_t kc;                  // kernel planes: 1 (one kernel for every channel) or C (one per channel)
    int32_t nb, base;            // stencil blocks (tiles x channels) and first block within its group launch
    int32_t nbe, base_e;         // elementwise blocks and first block within the elementwise launch
    int32_t nbf, basef;          // blocks of the one-pass FISTA launch (0: not on that path)
    int32_t cg1;                 // the CG solve runs the one-pass form (on the same blocks)
    int32_t cv_prev_slot;        // red slot for cv_prev_part's total
    int64_t N;                   // C*H*W
    // lower level (FISTA)
    gp<T> X[3];                     // iterates (rotating: cur, prev, next)
    gp<T> KX[3];                    // residuals theta * x - y, kept by linearity
    gp<T> xb;                       // base point of the residual recomputation
    gp<T> rb;                       // its residual theta * xb - y (FP64 sums, rounded once)
    gp<T> G;                        // gradient at the extrapolated point
    gp<const T> y;
    gp<T> th;                       // theta in the compute type, correlation form, column-major (kc planes)
    gp<T> thf;                      // the flipped kernel (convolution form), column-major (kc planes)
    // matrix-core operand layouts of th and thf (FP32 storage, K >= 13;
    // nullable: the correlations then run on the vector ALUs) and the
    // power-of-two exponent they were scaled by (one int per plane, written with them)
    gp<uint4> mf_th;
    gp<uint4> mf_thf;
    gp<int> mf_sh;
    gp<double> pA;                  // per-block partials, gradient pass (nb entries)
    gp<double> pB;                  // per-block partials, trial pass (nb entries)
    gp<int> trace;                  // rejected trials per iteration
    gp<T> xout;                     // where the returned point is written
    gp<T> hist;                     // nullable (two-pass form): iterate k+1 written to hist + k*N
    // conjugate gradients
    gp<T> q;
    gp<T> r;
    gp<T> P[2];                     // search direction (ping-pong)
    gp<T> Kp;                       // theta * p
    gp<T> Hp;
    gp<const T> xt;                 // point the Hessian is taken at
    gp<const T> b;                  // right-hand side
    gp<const T> q0;                 // the caller's starting point (read by the set-up passes)
    gp<double> pR;                  // per-block partials of ||r||^2 (nbe entries)
    gp<double> pK;                  // per-block partials of <p, Hp> (nb entries)
    gp<T> V[2];                     // one-pass CG: the second w buffer, and p
    gp<double> S64[2];              // one-pass CG: s = Hp, carried in FP64 (two buffers)
    // one convolution job: cv_out = cv_ker (x) cv_in [- cv_sub], partials of its square
    gp<const T> cv_ker;
    gp<const uint4> cv_mf;          // nullable: matrix-core layout of cv_ker
    gp<const int> cv_mfsh;          // its scale exponent
    gp<const double> cv_ker64;      // nullable (FP32 storage): the kernel as kc KxK planes of doubles, row-major;
                                    // the job then runs with FP64 taps and FP64 sums
    gp<double> cv_out64;            // nullable (with cv_ker64): cv_out kept in FP64 here instead
    int32_t cv_flip64;              // cv_ker64 is applied flipped (true convolution)
    gp<const T> cv_in;
    gp<const T> cv_sub;
    gp<T> cv_out;
    gp<T> cv_out2;                  // nullable: a second copy of cv_out
    gp<T> cv_out3;                  // nullable: a third copy of cv_out
    gp<T> cv_cp[3];                 // nullable: copies of cv_in
    gp<double> cv_part;             // nullable
    gp<const double> cv_prev_part;  // nullable: partials of an earlier pass, summed by block 0 into red[cv_prev_slot]
    // kernel preparation: theta64 (kc*K*K doubles) -> th / thf
    gp<const double> theta64;       // nullable: nothing to prepare
    gp<double> red;                 // per-instance reduction results (8 doubles)
    // Sobolev term r(theta) of Eq. (2.5) for the finishing pass (sob_th nullable)
    gp<const double> sob_th;
    gp<const double> sob_a;
    double beta, h1_w0;
    // batched hypergradient (Eq. 3.2): the correlation of (hg_rho, hg_q) and
    // (hg_w, cv_in) on hg_nblk blocks from block hg_base of its launch
    // (hg_nblk == 0: not in the launch), then z = -that + with_r grad r(theta64)
    // against hg_a, and ||z||^2 into *hg_zn2
    gp<const double> hg_rho;        // rho and theta*q in FP64 (FP32 storage: formed with FP64 taps
    gp<const double> hg_w;          // and sums, never rounded; FP64 storage: the images themselves)
    gp<const T> hg_q;
    gp<double> hg_part;
    gp<const double> hg_a;
    gp<double> hg_z;
    gp<double> hg_zn2;
    int32_t hg_nblk, hg_base, hg_with_r;
    // initial solver states, copied into the state arrays by the preparation
    // pass at the start of a solve (one upload per solve carries both)
    ApgState st0;
    CgState cg0;
};

}  // namespace maid
