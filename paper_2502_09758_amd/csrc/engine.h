// engine.h -- the host side of libmaid: a context over one or more problem
// instances (a ragged batch), its device workspace, solver states and
// instance tables, and the drivers of the solver passes.
//
// The host only enqueues kernels and polls: every arithmetic step runs on
// the GPU, and every solver decision (stop tests, backtracking, CG
// coefficients) is taken on the GPU by the pass that consumes the
// reduction, per instance, in the device-resident state arrays.  Solver
// passes are replayed in chunks from captured HIP graphs; the host copies
// the small state arrays back once per chunk to learn whether every solve
// has finished.  MAID's outer loop (Algorithm 2) runs on the host over
// scalars the kernels computed in FP64, in lockstep over the instances.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "devctx.h"
#include "maid.h"
#include "ops.h"

namespace maid {

constexpr int kRedSlots = 8;   // per-instance reduction results
constexpr int kRedG = 0, kRedGrad = 1, kRedZ = 2, kRedSob = 3, kRedAbs = 4;
constexpr int kTraceCap = 1 << 16;
constexpr int kHgMaxBlocks = 512;
constexpr int kEwMaxBlocks = 2048;

// kernel planes of a problem: 1 for a kernel shared by the channels, C for
// one kernel per channel (theta, a and z hold kplanes * K * K doubles)
inline int kplanes(const maid_desc& d) { return d.kc > 1 ? d.kc : 1; }

// Each pass family reads its own device copy of the instance table, so a
// captured graph (which embeds the table address) always sees the entries
// written for its family, and a later call can rewrite another family's
// entries while an earlier one is still queued.
enum Role { ROLE_APG = 0, ROLE_CG = 1, ROLE_CV0 = 2, ROLE_CV1 = 3, ROLE_CV2 = 4, ROLE_CV3 = 5, kRoles = 6 };

struct Member {
    maid_desc d;
    Shape shape;
    int64_t N;
    int R_auto;                 // rows per thread from the size rule
    int R_tuned;                // rows per thread chosen by the autotuner (0: none)
    int fuse_tuned;             // one-pass FISTA chosen by the autotuner (-1: not tuned, 0 no, 1 yes)
    int nbe;                    // elementwise blocks
    // current layout (depends on the tile rows)
    int R, nb, base, base_e;
    int nbf, basef;             // one-pass FISTA blocks and first block in the group's launch (0: two-pass)
    // device workspace, carved from the context's allocation
    void* X[3];
    void* KX[3];
    void* xb;                   // base point of the lower-level residual recomputation
    void* rb;                   // its residual theta*xb - y
    void* G;
    void* cq;
    void* cr;
    void* cP[2];
    void* cKp;
    void* cHp;
    void* cV[2];                // one-pass CG: second w buffer and p
    double* cS64[2];            // one-pass CG: s = Hp in FP64 (one-channel instances with 3 <= K <= 11)
    void* tmp0;
    void* tmp1;
    double* hg64[2];   // FP32 storage: rho and theta*q of the hypergradient, kept in FP64
    void* xtrial;
    void* gradg;
    void* th_c;
    void* thf_c;
    void* a_c;
    void* af_c;
    // matrix-core operand layouts of theta (FP32 storage, K >= 13; else
    // null): [0] theta, [1] flipped theta, and their scale exponent
    void* mf[2];
    int* mf_sh;
    bool on_team;               // its group runs the team loops (no matrix-core path there)
    double* th_trial;
    double* zbuf;
    double* pA;
    double* pB;
    double* pR;
    double* pK;
    double* pC;
    double* hg_part;
    int* trace;
};

struct LaunchGroup {
    Group g;
    std::vector<int> members;
    int team = 0;               // members per team of the persistent loops (0: multi-kernel passes)
    const int* list = nullptr;  // device copy of `members` (the team launches' instance list)
};

}  // namespace maid

struct maid_ctx {
    int n = 0;
    int dtype = 0;
    size_t esz = 0;
    std::vector<maid::Member> m;
    int R_override = 0;
    // layout: stencil groups and the elementwise map (device maps in `maps`)
    std::vector<maid::LaunchGroup> groups;
    int grid_e = 0;
    const int* blk_e = nullptr;
    int only_e = -1;                  // 0 for a single instance (no map lookup), else -1
    int* maps = nullptr;
    size_t maps_cap = 0;
    int layout_gen = 0;
    // maps of the active sub-layouts (device) and their pinned staging copy
    int* sub_maps = nullptr;
    int* sub_host = nullptr;
    bool compact = true;              // solves over part of a batch launch only its blocks
    // device-resident solver states (+ pinned host mirror of the same layout)
    char* st_dev = nullptr;
    char* st_host = nullptr;
    // host-visible, GPU-writable copy of the state block and its ready flag:
    // the solver loops learn the state without a stream synchronisation
    char* pub = nullptr;
    unsigned* pub_flag = nullptr;
    size_t st_bytes = 0;
    maid::ApgState* apg[2] = {};      // device arrays of n
    maid::CgState* cg[3] = {};
    // error words of the team loops, just before apg[0] and cg[0] in the
    // state block so that one publication brings back word and states
    unsigned* team_err_apg = nullptr;
    unsigned* team_err_cg = nullptr;
    double* red = nullptr;            // n x kRedSlots
    maid::ApgState* apg_h = nullptr;  // host mirror of apg[0]
    maid::CgState* cg_h = nullptr;    // host mirror of cg[0]
    double* red_h = nullptr;
    // instance tables: kRoles x n entries, device and pinned host
    char* tab_dev = nullptr;
    char* tab_host = nullptr;
    // workspace
    char* ws = nullptr;
    size_t ws_bytes = 0;
    // persistent team loops for small instances (one team per XCD)
    bool fuse = true;                 // one-pass FISTA where the group allows it
    bool cg_fuse = false;             // one-pass (Chronopoulos-Gear) CG on the one-pass instances (opt-in)
    bool mfma = true;                 // large-kernel correlations on the matrix cores (FP32 storage)
    int fuse_force = -1;              // autotuner's candidate: -1 none, 0 two-pass, 1 one-pass
    int fuse_pin = -1;                // the caller's choice (maid_set_one_pass): -1 none, 0, 1
    int team_req = -1;                // members per team: -1 size rule, 0 never, > 0 that many (capped)
    bool team_ok = false;             // blocks reach the XCDs round-robin and XCC_ID reads them
    int cus_per_xcd = 0;
    uint64_t* team_arrive = nullptr;  // kTeamXcd x kTeamMax arrival words
    uint64_t team_epoch = 0;
    int64_t team_wait = 0;            // wall-clock ticks of the longest wait at a team barrier
    hipStream_t cap = nullptr;        // private stream for graph capture
    bool use_graphs = true;
    bool in_step = false;             // inside a MAID step: solves need not drain the stream at their end
    bool upload_kernel = true;        // tables go up by a copy kernel reading mapped host memory
    int pred_first = 100;             // first chunk of a solve: this percentage of the predicted slots
    int pred_first_cg = 100;          // the same for the CG solves
    int kx_resync = 16;               // residual recomputed every kx_resync iterations (twice in a row)
    int kx_resync_full = 0;           // ... from scratch in FP64 every kx_resync_full (0: never)
    // fixed-step descent for the next lower-level solves (Section 4.1's
    // baselines; set by their entry points for one call): no momentum,
    // every step accepted; hist (single instance, two-pass form) receives
    // the iterates
    bool lower_fixed = false;
    void* lower_hist = nullptr;
    // the ADP baselines' workspace (unrolled iterates, adjoint vectors),
    // allocated at their first call and grown on demand
    char* adp_ws = nullptr;
    size_t adp_ws_bytes = 0;
    // FP64 companion of an FP32 context: the precision form's refinement
    // evaluates its gradients there (created at the first refinement)
    maid_ctx* ref64 = nullptr;
    // slots the last solve of each kind needed (sizes the first chunk of the
    // next): lower level for callers, for Algorithm 2's InexactGradient and
    // for its psi trials (their counts differ: the first starts from the
    // accepted trial's solution, the second from a new theta); CG
    long pred_slots[4] = {0, 0, 0, 0};
    struct Graph { int kind; int chunk; int gen; hipGraphExec_t exec; };
    std::vector<Graph> graphs;
    // decision trace of Algorithm 2 for one instance (maid_set_step_trace)
    struct StepTrace {
        int inst = -1;
        int32_t* w = nullptr;
        double* v = nullptr;
        int32_t cap_w = 0, cap_v = 0, n_w = 0, n_v = 0;
        bool full = false;
    } strace;
    std::string err;
    std::string cfg;
    // per-launch timing with HIP events on the launch stream
    bool prof_on = false;
    struct Rec { int kind; hipEvent_t a, b; };
    std::vector<Rec> prof_pending;
    std::vector<hipEvent_t> prof_pool;
    int64_t prof_launches[MAID_PROF_KINDS] = {};
    int64_t prof_work[MAID_PROF_KINDS] = {};
    double prof_ms[MAID_PROF_KINDS] = {};
};

namespace maid {

int fail(maid_ctx* c, int code, const std::string& msg);
int validate_desc(const maid_desc* d, std::string& why);
// Newton refinement of the single instance's lower-level solution x (see
// maid_lower_solve_refined)
template <typename T>
int refine_one(maid_ctx* c, const double* theta, const T* y, T* x, double rel_tol, int max_newton, int max_cg,
               double cg_rel, maid_refine_info* out, hipStream_t s);

// what is wrong with a description (a static string), or nullptr
const char* desc_problem(const maid_desc* d);

// maid_upper_value_grad_noalloc: the two instance-table entries (as words,
// to travel as kernel arguments), the launch group and the addresses inside
// the caller's fixed workspace ws (ws_bytes) of one upper-level evaluation
// laid out as on a new context.  MAID_EINVAL (with *why) when the instance
// does not fit.
template <int NW> struct Words { unsigned w[NW]; };
template <typename T> constexpr int kInstWords = (int)(sizeof(Inst<T>) / 4);
template <typename T> struct NoallocUpper {
    Words<kInstWords<T>> words[2];
    Group g;
    char* tab_dev;     // where the two entries go
    double* red_dev;   // the reduction slots
};
template <typename T>
int noalloc_upper_setup(const maid_desc* d, const double* a, const T* y, const T* x, T* grad_out, char* ws,
                        size_t ws_bytes, NoallocUpper<T>* job, const char** why);
int create_ctx(const maid_desc* descs, int n, maid_ctx** out, std::string& why);
void destroy_ctx(maid_ctx* c);
int relayout(maid_ctx* c);
void prof_harvest(maid_ctx* c);

// Per-instance results go to codes[i] (MAID_OK for inactive instances); the
// return value is MAID_OK or a negative error of the call as a whole.
template <typename T>
int lower_batch(maid_ctx* c, const std::vector<char>& act, const std::vector<const double*>& theta,
                const std::vector<const T*>& y, const std::vector<T*>& x, const std::vector<double>& tol, int max_iter,
                double* L_inout, maid_solve_info* info, int* codes, int32_t* trace_bt, hipStream_t s,
                int pred_role = 0, const std::vector<const T*>* xin = nullptr);
template <typename T>
int adjoint_batch(maid_ctx* c, const std::vector<char>& act, const std::vector<const double*>& theta,
                  const std::vector<const T*>& xt, const std::vector<const T*>& rhs, const std::vector<T*>& q,
                  const std::vector<double>& tol, int max_iter, maid_solve_info* info, int* codes, hipStream_t s);
template <typename T>
int upper_batch(maid_ctx* c, const std::vector<char>& act, const std::vector<const double*>& a,
                const std::vector<const T*>& y, const std::vector<const T*>& x, const std::vector<T*>& grad,
                double* g_out, double* gn_out, hipStream_t s);
template <typename T>
int hypergrad_batch(maid_ctx* c, const std::vector<char>& act, const std::vector<const double*>& theta,
                    const std::vector<const double*>& a, const std::vector<const T*>& y, const std::vector<const T*>& xt,
                    const std::vector<const T*>& q, int with_r, const std::vector<double*>& z, double* znorm_out,
                    hipStream_t s);
int sobolev_batch(maid_ctx* c, const std::vector<char>& act, const std::vector<const double*>& theta,
                  const std::vector<const double*>& a, double* r_out, hipStream_t s);
template <typename T>
int apply_operator_one(maid_ctx* c, const double* theta, const T* in, T* out, int adjoint, hipStream_t s);
// Time short lower-level and CG probes with each rows-per-thread candidate
// per group of instances sharing K, keep the fastest (rows_out: nullable,
// the choice per instance).
template <typename T>
int autotune_batch(maid_ctx* c, const std::vector<const double*>& theta, const std::vector<const T*>& y, int probe_iters,
                   int32_t* rows_out, hipStream_t s);
template <typename T>
// active (nullable): the instances that take the step (the others are left
// as they are, their info zeroed and code MAID_OK)
int step_batch(maid_ctx* c, const std::vector<const double*>& a, const std::vector<const T*>& y, maid_state* st,
               const maid_hparams* hp, maid_step_info* out, int* codes, hipStream_t s,
               const std::vector<char>* active = nullptr);

// Proposition 1's Hessian at x applied to w (single instance), by the
// adjoint solve's set-up passes.
template <typename T>
int hessian_one(maid_ctx* c, const double* theta, const T* x, const T* w, T* out, hipStream_t s);

// Section 4.1's baselines (adp.cpp), single instance: fixed-step descent
// (hist nullable), one ADP-IFT and one ADP-LISTA upper-level iteration.
template <typename T>
int gd_one(maid_ctx* c, const double* theta, const T* y, T* x, double step, int n_iter, double tol, T* hist,
           maid_solve_info* info, hipStream_t s);
template <typename T>
int ift_step_one(maid_ctx* c, const double* a, const T* y, maid_state* st, int n_lower, double lambda_x,
                 double cg_tol, int max_cg, maid_step_info* info, hipStream_t s);
template <typename T>
int lista_step_one(maid_ctx* c, const double* a, const T* y, maid_state* st, int n_unroll, double lambda_x,
                   maid_step_info* info, hipStream_t s);

// MAID_OK if every code is MAID_OK, else the first code that is not.
int combine_codes(const int* codes, int n);

}  // namespace maid
