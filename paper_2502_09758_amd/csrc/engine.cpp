// engine.cpp -- context set-up, launch layout, instance tables, graph
// capture, timing, and the batched solver drivers (Algorithm 1's lower-level
// solve and Hessian system, the upper-level value and gradient, the
// hypergradient of Eq. 3.2, and Algorithm 2 in lockstep over the instances).
#include "engine.h"
#include "mfconv.cuh"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>

namespace maid {

static_assert(sizeof(Inst<float>) == sizeof(Inst<double>), "instance tables share one layout");

int fail(maid_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                                        \
    do {                                                                                                     \
        hipError_t e_ = (expr);                                                                              \
        if (e_ != hipSuccess)                                                                                \
            return fail(c, MAID_EHIP, std::string("HIP error in ") + #expr + ": " + hipGetErrorString(e_)); \
    } while (0)

#define TRY(expr)               \
    do {                        \
        int rc_ = (expr);       \
        if (rc_) return rc_;    \
    } while (0)

namespace {

// Instances whose large-kernel correlations can run on the matrix cores
// (FP32 storage, K >= 13): they carry the operand layouts of theta.
bool mf_member(int dtype, int K) { return dtype == MAID_F32 && K >= 13 && K <= kMaxK; }

bool finite(double v) { return std::isfinite(v); }

int auto_rows(const Shape& d) {
    // the largest tile height that still gives every CU (256) four blocks
    if (stencil_blocks(d, 4) >= 1024) return 4;
    if (stencil_blocks(d, 2) >= 1024) return 2;
    return 1;
}

int round8(int v) { return (v + 7) & ~7; }

int status_code(int st) {
    switch (st) {
        case ST_OK: return MAID_OK;
        case ST_MAXITER: return MAID_MAXITER;
        case ST_NOT_SPD: return MAID_NOT_SPD;
        default: return MAID_NONFINITE;
    }
}

bool any(const std::vector<char>& v) {
    for (char b : v)
        if (b) return true;
    return false;
}

template <typename T> Inst<T>* tab_host(maid_ctx* c, int role) {
    return reinterpret_cast<Inst<T>*>(c->tab_host) + (size_t)role * c->n;
}
template <typename T> const Inst<T>* tab_dev(maid_ctx* c, int role) {
    return reinterpret_cast<const Inst<T>*>(c->tab_dev) + (size_t)role * c->n;
}

// copy a byte range of the state block between device and the pinned mirror
int pull(maid_ctx* c, hipStream_t s, const void* dev_ptr, size_t n) {
    const size_t off = (const char*)dev_ptr - c->st_dev;
    HIP_TRY(hipMemcpyAsync(c->st_host + off, c->st_dev + off, n, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return MAID_OK;
}
int push(maid_ctx* c, hipStream_t s, const void* dev_ptr, size_t n) {
    const size_t off = (const char*)dev_ptr - c->st_dev;
    HIP_TRY(hipMemcpyAsync(c->st_dev + off, c->st_host + off, n, hipMemcpyHostToDevice, s));
    return MAID_OK;
}
// copy `roles` adjacent role tables, starting at `role`, in one transfer
template <typename T> int upload(maid_ctx* c, int role, hipStream_t s, int roles = 1) {
    const size_t bytes = sizeof(Inst<T>) * c->n;
    if (c->upload_kernel)
        HIP_TRY(launch_upload(c->tab_host + role * bytes, roles * bytes, c->tab_dev + role * bytes, s));
    else
        HIP_TRY(hipMemcpyAsync(c->tab_dev + role * bytes, c->tab_host + role * bytes, roles * bytes,
                               hipMemcpyHostToDevice, s));
    return MAID_OK;
}
// upload `roles` adjacent role tables starting at `role` and run the
// preparation pass over the first of them (one launch with the upload kernel)
template <typename T>
int upload_prep(maid_ctx* c, int role, int roles, ApgState* Lst, CgState* Cst, int slot_abs, hipStream_t s) {
    const size_t bytes = sizeof(Inst<T>) * c->n;
    if (!c->upload_kernel) {
        TRY(upload<T>(c, role, s, roles));
        HIP_TRY(Ops<T>::prep_kernel(tab_dev<T>(c, role), c->n, Lst, Cst, slot_abs, s));
        return MAID_OK;
    }
    HIP_TRY(Ops<T>::prep_upload(c->tab_host + role * bytes, c->tab_dev + role * bytes, roles, c->n, Lst, Cst,
                                slot_abs, s));
    return MAID_OK;
}
int publish(maid_ctx* c, hipStream_t s, const void* dev_ptr, size_t n);
int pull_red(maid_ctx* c, hipStream_t s) { return publish(c, s, c->red, sizeof(double) * kRedSlots * c->n); }

// Like pull, without synchronising the stream: a one-block kernel copies
// the range into host-visible memory and raises a flag, which the host
// waits for (with the stream synchronisation as the fallback after a long
// wait).  The state lands in the same mirror as with pull.
int publish(maid_ctx* c, hipStream_t s, const void* dev_ptr, size_t n) {
    const size_t off = (const char*)dev_ptr - c->st_dev;
    volatile unsigned* flag = c->pub_flag;
    *flag = 0u;
    HIP_TRY(launch_publish(c->st_dev + off, n, c->pub + off, c->pub_flag, s));
    const auto t0 = std::chrono::steady_clock::now();
    long spins = 0;
    while (*flag == 0u) {
        if ((++spins & 1023) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(200)) {
            HIP_TRY(hipStreamSynchronize(s));
            if (*flag == 0u) return fail(c, MAID_EHIP, "state publication did not arrive");
            break;
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    std::memcpy(c->st_host + off, c->pub + off, n);
    return MAID_OK;
}

// Table entry of instance i with every workspace pointer set; the caller
// adds the per-call pointers.
template <typename T> void fill_base(maid_ctx* c, int i, Inst<T>& I) {
    std::memset(&I, 0, sizeof(I));
    const Member& M = c->m[i];
    I.pr = Params{M.d.C, M.d.H, M.d.W, M.d.reg, M.d.alpha, M.d.eps_tv};
    I.K = M.d.K;
    I.kc = kplanes(M.d);
    I.nb = M.nb;
    I.base = M.base;
    I.nbe = M.nbe;
    I.base_e = M.base_e;
    I.nbf = M.nbf;
    I.basef = M.basef;
    I.cg1 = M.nbf > 0 && c->cg_fuse ? 1 : 0;
    I.N = M.N;
    for (int k = 0; k < 3; ++k) {
        I.X[k] = (T*)M.X[k];
        I.KX[k] = (T*)M.KX[k];
    }
    I.xb = (T*)M.xb;
    I.rb = (T*)M.rb;
    I.G = (T*)M.G;
    I.th = (T*)M.th_c;
    I.thf = (T*)M.thf_c;
    if (c->mfma && M.mf[0] && !M.on_team) {
        I.mf_th = (uint4*)M.mf[0];
        I.mf_thf = (uint4*)M.mf[1];
        I.mf_sh = M.mf_sh;
    }
    I.pA = M.pA;
    I.pB = M.pB;
    I.trace = M.trace;
    I.q = (T*)M.cq;
    I.r = (T*)M.cr;
    I.P[0] = (T*)M.cP[0];
    I.P[1] = (T*)M.cP[1];
    I.Kp = (T*)M.cKp;
    I.Hp = (T*)M.cHp;
    I.pR = M.pR;
    I.pK = M.pK;
    I.V[0] = (T*)M.cV[0];
    I.V[1] = (T*)M.cV[1];
    I.S64[0] = M.cS64[0];
    I.S64[1] = M.cS64[1];
    I.red = c->red + (size_t)i * kRedSlots;
}

}  // namespace

int combine_codes(const int* codes, int n) {
    for (int i = 0; i < n; ++i)
        if (codes[i] != MAID_OK) return codes[i];
    return MAID_OK;
}

// ------------------------------------------------------------------ profiling
namespace {

hipEvent_t prof_event(maid_ctx* c) {
    if (!c->prof_pool.empty()) {
        hipEvent_t e = c->prof_pool.back();
        c->prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct ProfScope {
    maid_ctx* c;
    int kind;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    // the events ride on the one launch made inside the scope and carry that
    // kernel's start and end timestamps
    ProfScope(maid_ctx* c_, int k, hipStream_t s_) : c(c_), kind(k), s(s_) {
        if (!c->prof_on) return;
        a = prof_event(c);
        b = prof_event(c);
        if (a && b) launch_timing() = LaunchTiming{a, b};
    }
    ~ProfScope() {
        if (!c->prof_on || !a || !b) return;
        launch_timing() = LaunchTiming{};
        c->prof_pending.push_back({kind, a, b});
        if (c->prof_pending.size() >= 4096) prof_harvest(c);
    }
};

}  // namespace

// Accumulate the durations of recorded launches (waits for the last one).
void prof_harvest(maid_ctx* c) {
    if (c->prof_pending.empty()) return;
    (void)hipEventSynchronize(c->prof_pending.back().b);
    for (auto& r : c->prof_pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            c->prof_launches[r.kind] += 1;
            c->prof_ms[r.kind] += ms;
            // kinds without early exits: every launch works
            if (r.kind != MAID_PROF_APG_GRAD && r.kind != MAID_PROF_APG_TRIAL && r.kind != MAID_PROF_CG_DIR &&
                r.kind != MAID_PROF_CG_HVP && r.kind != MAID_PROF_CG_UPDATE && r.kind != MAID_PROF_APG_TEAM &&
                r.kind != MAID_PROF_CG_TEAM && r.kind != MAID_PROF_APG_STEP && r.kind != MAID_PROF_CG_STEP)
                c->prof_work[r.kind] += 1;
        }
        c->prof_pool.push_back(r.a);
        c->prof_pool.push_back(r.b);
    }
    c->prof_pending.clear();
}

// Launch expression `expr` (returning hipError_t) timed as `kind`.
#define LAUNCH(kind, expr)                       \
    do {                                         \
        ProfScope ps_(c, (kind), s);             \
        HIP_TRY(expr);                           \
    } while (0)

// ------------------------------------------------------------------ graph-captured chunks
// A chunk of solver passes is captured once into a HIP graph (per pass
// family, chunk length and launch layout) and replayed; the passes read
// everything that changes between replays from the instance table and the
// state arrays, whose addresses are fixed.  With timing on, passes launch
// directly so that each one is bracketed by its own events.
namespace {

enum { G_APG = 1, G_CG = 2 };

template <typename F>
int run_chunk(maid_ctx* c, int kind, int chunk, hipStream_t s, F enqueue, bool graphs) {
    if (c->prof_on || !c->use_graphs || !graphs) return enqueue(s);
    for (auto& g : c->graphs)
        if (g.kind == kind && g.chunk == chunk && g.gen == c->layout_gen) {
            HIP_TRY(hipGraphLaunch(g.exec, s));
            return MAID_OK;
        }
    HIP_TRY(hipStreamBeginCapture(c->cap, hipStreamCaptureModeRelaxed));
    int rc = enqueue(c->cap);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(c->cap, &graph);
    if (rc != MAID_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return fail(c, MAID_EHIP, std::string("graph capture failed: ") + hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(c, MAID_EHIP, std::string("graph instantiation failed: ") + hipGetErrorString(e));
    if (c->graphs.size() >= 48) {
        (void)hipGraphExecDestroy(c->graphs.front().exec);
        c->graphs.erase(c->graphs.begin());
    }
    c->graphs.push_back({kind, chunk, c->layout_gen, exec});
    HIP_TRY(hipGraphLaunch(exec, s));
    return MAID_OK;
}

// Launch `want` slots as power-of-two graph chunks back to back (no host
// round trip between them).
template <typename F>
int run_slots(maid_ctx* c, int kind, long want, hipStream_t s, F enqueue, bool graphs = true) {
    for (int p = 32; p >= 1; p >>= 1)
        while (want >= p) {
            int rc = run_chunk(c, kind, p, s, [&](hipStream_t st) { return enqueue(st, p); }, graphs);
            if (rc) return rc;
            want -= p;
        }
    return MAID_OK;
}

// Slots to launch before the next look at the state: first first_pct % of
// the count the previous solve of this kind needed (warm-started solves in
// Algorithm 2 need similar counts; a slot past the end costs two early-exit
// launches, a few microseconds, while a look costs a host round trip with
// the GPU drained; measured at 256 x 256, K = 9: 100 % beats 75 % by ~5 %
// per MAID step and 50 % by ~12 %; for the CG solves alone 100 % beats 75 %
// by ~7 % and 125 % by ~5 %), then steps of an eighth of it; with no
// history 1, 2, 4, ...
long next_slots(long pred, long done_so_far, long last, int first_pct) {
    if (done_so_far == 0) return pred > 0 ? std::max(1L, pred * first_pct / 100) : 1;
    if (pred > 0 && done_so_far == last) return std::max(1L, pred / 8);
    return std::min(last * 2, 64L);
}

// The launch layout of a solve over the instances of `act`.  A solve over
// part of a batch (Algorithm 2's trial solves and retries, where instances
// step in lockstep but need different numbers of solves) would otherwise
// launch every block of every group in every pass, the inactive instances'
// blocks exiting at once: per pass a dispatch of the whole batch for the
// work of a few instances.  The sub-layout gives each group's active
// instances consecutive block ranges, each starting at a multiple of 8 as in
// the full layout (the same local block indices and tiles, so bitwise the
// same results), and a group without an active instance launches nothing.
// Its chunks run without graphs (a graph embeds its grid); team groups keep
// their layout.
struct SubLayout {
    bool full = true;
    std::vector<LaunchGroup> groups;
    int grid_e = 0;
    const int* blk_e = nullptr;
    int only_e = -1;
    std::vector<int> base, basef, base_e;   // per instance (active, compacted groups)
    template <typename T> void apply(Inst<T>* tab, const std::vector<char>& act) const {
        if (full) return;
        for (size_t i = 0; i < base.size(); ++i)
            if (act[i]) {
                tab[i].base = base[i];
                tab[i].basef = basef[i];
                tab[i].base_e = base_e[i];
            }
    }
};

// Blocks of one pass over the multi-kernel groups for the instances of act
// (the sub-layout's grids, without building it).
int64_t pass_blocks(maid_ctx* c, const std::vector<char>& act) {
    int64_t b = 0;
    for (auto& lg : c->groups) {
        if (lg.team > 0) continue;
        for (int i : lg.members)
            if (act[i]) b += round8(lg.g.grid_f > 0 ? c->m[i].nbf : c->m[i].nb);
    }
    return b;
}

int sub_layout(maid_ctx* c, const std::vector<char>& act, SubLayout& L, hipStream_t s);

// Between chunks of a solve: once the instances still iterating hold less
// than 60 % of the blocks the passes launch, launch theirs alone (the
// finished ones' final states stay where the last slot left them, in the
// arrays the solve reads them from; their table entries keep their ranges).
template <typename T>
int shrink_layout(maid_ctx* c, SubLayout& L, std::vector<char>& cur, const std::vector<char>& still, Inst<T>* tab,
                  const Inst<T>* tabd, hipStream_t s) {
    if (!c->compact || !c->sub_maps) return MAID_OK;
    const int64_t now = pass_blocks(c, cur), left = pass_blocks(c, still);
    if (left == 0 || left * 10 >= now * 6) return MAID_OK;
    TRY(sub_layout(c, still, L, s));
    L.apply(tab, still);
    HIP_TRY(hipMemcpyAsync(const_cast<Inst<T>*>(tabd), tab, (size_t)c->n * sizeof(Inst<T>), hipMemcpyHostToDevice,
                           s));
    cur = still;
    return MAID_OK;
}

int sub_layout(maid_ctx* c, const std::vector<char>& act, SubLayout& L, hipStream_t s) {
    const int n = c->n;
    L = SubLayout();
    L.groups = c->groups;
    L.grid_e = c->grid_e;
    L.blk_e = c->blk_e;
    L.only_e = c->only_e;
    bool all = true;
    for (char a : act) all = all && a;
    if (all || !c->compact || !c->sub_maps) return MAID_OK;
    L.full = false;
    L.base.assign(n, 0);
    L.basef.assign(n, 0);
    L.base_e.assign(n, 0);
    for (int i = 0; i < n; ++i) {   // team groups keep the full layout's ranges
        L.base[i] = c->m[i].base;
        L.basef[i] = c->m[i].basef;
    }
    int* h = c->sub_host;
    size_t used = 0;
    auto fill = [&](const std::vector<int>& ids, const std::vector<int>& b, int grid) {
        for (size_t t = 0; t < ids.size(); ++t) {
            const int end = t + 1 < ids.size() ? b[ids[t + 1]] : grid;
            for (int k = b[ids[t]]; k < end; ++k) h[used + k] = ids[t];
        }
    };
    std::vector<size_t> off(L.groups.size(), 0), offf(L.groups.size(), 0);
    for (size_t g = 0; g < L.groups.size(); ++g) {
        LaunchGroup& lg = L.groups[g];
        if (lg.team > 0) continue;
        std::vector<int> ids;
        for (int i : lg.members)
            if (act[i]) ids.push_back(i);
        int base = 0, grid = 0;
        for (int i : ids) {
            L.base[i] = base;
            grid = base + c->m[i].nb;
            base = round8(grid);
        }
        lg.g.grid = grid;
        lg.g.only = ids.size() == 1 ? ids[0] : -1;
        off[g] = used;
        fill(ids, L.base, grid);
        used += grid;
        int basef = 0, gridf = 0;
        if (lg.g.grid_f > 0) {
            for (int i : ids) {
                L.basef[i] = basef;
                gridf = basef + c->m[i].nbf;
                basef = round8(gridf);
            }
            lg.g.grid_f = gridf;
            offf[g] = used;
            fill(ids, L.basef, gridf);
            used += gridf;
        }
    }
    std::vector<int> ids_e;
    int base_e = 0;
    for (int i = 0; i < n; ++i) {
        if (!act[i]) continue;
        ids_e.push_back(i);
        L.base_e[i] = base_e;
        L.grid_e = base_e + c->m[i].nbe;
        base_e = round8(L.grid_e);
    }
    if (ids_e.empty()) L.grid_e = 0;
    const size_t off_e = used;
    fill(ids_e, L.base_e, L.grid_e);
    used += L.grid_e;
    L.only_e = -1;
    if (used > c->maps_cap) return fail(c, MAID_EHIP, "sub_layout: block maps exceed their allocation");
    // the previous sub-layout's copy and the passes that read it are behind
    // the previous solve's last state publication, which waited for them
    HIP_TRY(hipMemcpyAsync(c->sub_maps, h, used * sizeof(int), hipMemcpyHostToDevice, s));
    for (size_t g = 0; g < L.groups.size(); ++g) {
        LaunchGroup& lg = L.groups[g];
        if (lg.team > 0) continue;
        lg.g.blk = c->sub_maps + off[g];
        lg.g.blk_f = lg.g.grid_f > 0 ? c->sub_maps + offf[g] : nullptr;
    }
    L.blk_e = c->sub_maps + off_e;
    return MAID_OK;
}

}  // namespace

// ------------------------------------------------------------------ set-up
const char* desc_problem(const maid_desc* d) {
    if (!d) return "desc is NULL";
    if (d->H < 1 || d->W < 1) return "H and W must be >= 1";
    if (d->C < 1 || d->C > kMaxC) return "C must be 1, 2 or 3";
    if (d->K < 1 || d->K > kMaxK || (d->K % 2) == 0) return "K must be odd, 1 <= K <= 31";
    if (d->K > d->H || d->K > d->W) return "K must not exceed H or W";
    if (d->dtype != MAID_F32 && d->dtype != MAID_F64) return "dtype must be MAID_F32 or MAID_F64";
    if (d->boundary == MAID_BOUNDARY_PERIODIC) return "boundary: periodic convolution is not implemented (zero boundary only)";
    if (d->boundary != MAID_BOUNDARY_ZERO) return "boundary must be MAID_BOUNDARY_ZERO";
    if (d->reg < 0 || d->reg > 2) return "reg must be 0, 1 or 2";
    if (d->kc < 0 || (d->kc > 1 && d->kc != d->C)) return "kc must be 0 or 1 (one kernel) or C (one kernel per channel)";
    if (!finite(d->alpha) || d->alpha < 0) return "alpha must be finite and >= 0";
    if (d->reg != MAID_REG_QUADRATIC && !(d->eps_tv > 0 && finite(d->eps_tv))) return "eps_tv must be > 0";
    if (!finite(d->beta) || d->beta < 0) return "beta must be finite and >= 0";
    if (!finite(d->h1_w0) || d->h1_w0 < 0) return "h1_w0 must be finite and >= 0";
    // one channel plane is indexed with 32-bit offsets in the kernels
    if ((double)d->H * d->W >= 2147483648.0) return "H*W must be below 2^31";
    return nullptr;
}

template <typename T>
int noalloc_upper_setup(const maid_desc* d, const double* a, const T* y, const T* x, T* grad_out, char* ws,
                        size_t ws_bytes, NoallocUpper<T>* job, const char** why) {
    static_assert(sizeof(Inst<T>) % 4 == 0 && 2 * sizeof(Inst<T>) <= 3072, "entries travel as kernel arguments");
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const Shape sh{d->C, d->H, d->W, d->K, d->reg};
    const int R = auto_rows(sh);
    const int nb = stencil_blocks(sh, R);
    const size_t N = (size_t)d->C * d->H * d->W;
    // tables, kernel copies, reduction slots, two partial arrays, the
    // residual image and (without grad_out) the gradient
    const size_t o_kc = al(2 * sizeof(Inst<T>));
    const size_t o_kf = o_kc + al((size_t)kplanes(*d) * d->K * d->K * sizeof(T));
    const size_t o_red = o_kf + al((size_t)kplanes(*d) * d->K * d->K * sizeof(T));
    const size_t o_pc = o_red + al(kRedSlots * sizeof(double));
    const size_t o_pa = o_pc + al((size_t)nb * sizeof(double));
    const size_t o_rho = o_pa + al((size_t)nb * sizeof(double));
    const size_t o_grad = o_rho + al(N * sizeof(T));
    const size_t end = o_grad + (grad_out ? 0 : al(N * sizeof(T)));
    if (end > ws_bytes) {
        if (why)
            *why = "upper_value_grad_noalloc: the instance needs more than the fixed 64 MiB workspace "
                   "(C*H*W*element size must stay below about 64 MiB, 32 MiB with grad_out NULL)";
        return MAID_EINVAL;
    }
    Inst<T> t[2];
    std::memset(static_cast<void*>(t), 0, sizeof(t));
    for (auto& I : t) {
        I.pr = Params{d->C, d->H, d->W, d->reg, d->alpha, d->eps_tv};
        I.K = d->K;
        I.kc = kplanes(*d);
        I.nb = nb;
        I.base = 0;
        I.N = (int64_t)N;
        I.red = reinterpret_cast<double*>(ws + o_red);
    }
    // the entries of upper_impl: rho = a*x - y (flipped a), grad = a.rho
    t[0].th = reinterpret_cast<T*>(ws + o_kc);
    t[0].thf = reinterpret_cast<T*>(ws + o_kf);
    t[0].theta64 = a;
    t[0].cv_ker = reinterpret_cast<T*>(ws + o_kf);
    t[0].cv_ker64 = a;
    t[0].cv_flip64 = 1;
    t[0].cv_in = x;
    t[0].cv_sub = y;
    t[0].cv_out = reinterpret_cast<T*>(ws + o_rho);
    t[0].cv_part = reinterpret_cast<double*>(ws + o_pc);
    t[1].cv_ker = reinterpret_cast<T*>(ws + o_kc);
    t[1].cv_ker64 = a;
    t[1].cv_flip64 = 0;
    t[1].cv_in = reinterpret_cast<T*>(ws + o_rho);
    t[1].cv_out = grad_out ? grad_out : reinterpret_cast<T*>(ws + o_grad);
    t[1].cv_part = reinterpret_cast<double*>(ws + o_pa);
    t[1].cv_prev_part = reinterpret_cast<double*>(ws + o_pc);
    t[1].cv_prev_slot = kRedG;
    std::memcpy(&job->words[0], &t[0], sizeof(Inst<T>));
    std::memcpy(&job->words[1], &t[1], sizeof(Inst<T>));
    job->g = Group{};
    job->g.K = d->K;
    job->g.R = R;
    job->g.C = d->C;
    job->g.nw = d->reg == 1 ? d->C : 1;
    job->g.grid = nb;
    job->g.blk = nullptr;
    job->g.only = 0;
    job->tab_dev = ws;
    job->red_dev = reinterpret_cast<double*>(ws + o_red);
    return MAID_OK;
}
template int noalloc_upper_setup<float>(const maid_desc*, const double*, const float*, const float*, float*, char*,
                                        size_t, NoallocUpper<float>*, const char**);
template int noalloc_upper_setup<double>(const maid_desc*, const double*, const double*, const double*, double*, char*,
                                         size_t, NoallocUpper<double>*, const char**);

int validate_desc(const maid_desc* d, std::string& why) {
    const char* p = desc_problem(d);
    if (!p) return MAID_OK;
    why = p;
    return MAID_EINVAL;
}

// Members per team of a group's persistent loops, 0 for the multi-kernel
// passes.  Every member must hold at least one tile and one elementwise
// block of each instance (each member takes the solver decisions itself), and
// a team must fit on its XCD at once.  Size rule: the team path for groups
// whose instances have at most kTeamTiles x 256 pixels (kTeamTiles tiles of
// one row per thread), one tile per member.  A pass
// on one XCD is bound by that XCD's vector ALUs once each member holds more
// than one tile (measured: 128x128 at one row per thread, 64 tiles, runs
// lower + CG iterations ~17% faster on teams than as kernels; 256x256, 256
// tiles, 2.4x slower), so larger instances stay on the multi-kernel passes.
constexpr int kTeamTiles = 64;
int team_members(maid_ctx* c, const LaunchGroup& lg) {
    if (!c->team_ok || c->team_req == 0 || lg.g.R > 4) return 0;
    int most_tiles = 0, cap = kTeamMax;
    for (int i : lg.members) {
        const int tiles = lg.g.grid_f > 0 ? c->m[i].nbf : c->m[i].nb;
        most_tiles = std::max(most_tiles, tiles);
        cap = std::min(cap, std::min(tiles, c->m[i].nbe));
    }
    // the size rule counts pixels (tiles of one row per thread), whatever the tile height
    int64_t most_px = 0;
    for (int i : lg.members) most_px = std::max<int64_t>(most_px, c->m[i].N);
    if (c->team_req < 0 && most_px > (int64_t)kTeamTiles * kTW * tile_h(1)) return 0;
    int bpc = 0;
    const hipError_t e = c->dtype == MAID_F64 ? Ops<double>::team_occupancy(lg.g, &bpc)
                                              : Ops<float>::team_occupancy(lg.g, &bpc);
    if (e != hipSuccess || bpc < 1) return 0;
    cap = std::min(cap, bpc * c->cus_per_xcd);
    const int want = c->team_req > 0 ? c->team_req : most_tiles;
    return std::max(0, std::min(want, cap));
}

// Group the instances by (K, tile rows), give each instance a block range
// starting at a multiple of 8 (so that the XCD-major tile order holds within
// every instance), build the block -> instance maps and upload them.
int relayout(maid_ctx* c) {
    c->groups.clear();
    std::vector<int> host;
    for (int i = 0; i < c->n; ++i) {
        Member& M = c->m[i];
        M.R = c->R_override ? std::min(c->R_override, max_rows(M.d.K)) : (M.R_tuned ? M.R_tuned : M.R_auto);
        M.nb = stencil_blocks(M.shape, M.R);
        // the one-pass FISTA form (one channel, 3 <= K <= 11) is opt-in
        // (maid_set_one_pass(ctx, 1)): GPUs were lost while its tests ran and
        // no cause has been found, so the default path keeps the two-pass form
        bool fuse = c->fuse && step_ok(M.d.C, M.d.K, M.R);
        if (c->fuse_force >= 0) fuse = fuse && c->fuse_force == 1;
        else fuse = fuse && c->fuse_pin == 1;
        M.nbf = fuse ? step_blocks(M.d.H, M.d.W, M.d.K, M.R) : 0;
    }
    std::vector<char> placed(c->n, 0);
    for (int i = 0; i < c->n; ++i) {
        if (placed[i]) continue;
        LaunchGroup lg;
        lg.g = Group{c->m[i].d.K, c->m[i].R, 1, 1, 0, nullptr, -1, 0, nullptr, 0};
        for (int k = i; k < c->n; ++k)
            if (!placed[k] && c->m[k].d.K == lg.g.K && c->m[k].R == lg.g.R &&
                (c->m[k].nbf > 0) == (c->m[i].nbf > 0)) {
                placed[k] = 1;
                lg.members.push_back(k);
            }
        int base = 0;
        for (size_t t = 0; t < lg.members.size(); ++t) {
            Member& M = c->m[lg.members[t]];
            M.base = base;
            lg.g.C = std::max(lg.g.C, M.d.C);
            lg.g.nw = std::max(lg.g.nw, M.d.reg == MAID_REG_TV_CHANNELWISE ? M.d.C : 1);
            lg.g.grid = base + M.nb;
            base = round8(base + M.nb);
        }
        c->groups.push_back(lg);
    }
    // one-pass block ranges, then team loops for groups of tiny instances
    for (auto& lg : c->groups) {
        int basef = 0;
        for (int i : lg.members) {
            Member& M = c->m[i];
            M.basef = M.nbf > 0 ? basef : 0;
            if (M.nbf > 0) {
                lg.g.grid_f = basef + M.nbf;
                basef = round8(basef + M.nbf);
            }
        }
        lg.g.cg1 = lg.g.grid_f > 0 && c->cg_fuse ? 1 : 0;
        lg.team = team_members(c, lg);
        for (int i : lg.members) c->m[i].on_team = lg.team > 0;
    }
    int base_e = 0;
    for (int i = 0; i < c->n; ++i) {
        c->m[i].base_e = base_e;
        c->grid_e = base_e + c->m[i].nbe;
        base_e = round8(base_e + c->m[i].nbe);
    }
    // maps: every group's stencil map, then the elementwise map
    std::vector<size_t> offs;
    for (auto& lg : c->groups) {
        offs.push_back(host.size());
        host.resize(host.size() + lg.g.grid);
        int* mp = host.data() + offs.back();
        for (size_t t = 0; t < lg.members.size(); ++t) {
            const Member& M = c->m[lg.members[t]];
            const int end = t + 1 < lg.members.size() ? c->m[lg.members[t + 1]].base : lg.g.grid;
            for (int b = M.base; b < end; ++b) mp[b] = lg.members[t];
        }
    }
    const size_t off_e = host.size();
    host.resize(host.size() + c->grid_e);
    for (int i = 0; i < c->n; ++i) {
        const int end = i + 1 < c->n ? c->m[i + 1].base_e : c->grid_e;
        for (int b = c->m[i].base_e; b < end; ++b) host[off_e + b] = i;
    }
    std::vector<size_t> offs_l, offs_f;
    for (auto& lg : c->groups) {
        offs_l.push_back(host.size());
        host.insert(host.end(), lg.members.begin(), lg.members.end());
    }
    for (auto& lg : c->groups) {
        offs_f.push_back(host.size());
        host.resize(host.size() + lg.g.grid_f);
        int* mp = host.data() + offs_f.back();
        for (size_t t = 0; t < lg.members.size() && lg.g.grid_f > 0; ++t) {
            const Member& M = c->m[lg.members[t]];
            const int end = t + 1 < lg.members.size() ? c->m[lg.members[t + 1]].basef : lg.g.grid_f;
            for (int b = M.basef; b < end; ++b) mp[b] = lg.members[t];
        }
    }
    if (host.size() > c->maps_cap) return fail(c, MAID_EHIP, "relayout: block maps exceed their allocation");
    HIP_TRY(hipMemcpy(c->maps, host.data(), host.size() * sizeof(int), hipMemcpyHostToDevice));
    for (size_t g = 0; g < c->groups.size(); ++g) {
        c->groups[g].g.blk = c->maps + offs[g];
        c->groups[g].g.only = c->groups[g].members.size() == 1 ? c->groups[g].members[0] : -1;
    }
    c->blk_e = c->maps + off_e;
    c->only_e = c->n == 1 ? 0 : -1;
    for (size_t g = 0; g < c->groups.size(); ++g) {
        LaunchGroup& lg = c->groups[g];
        lg.list = c->maps + offs_l[g];
        lg.g.blk_f = lg.g.grid_f > 0 ? c->maps + offs_f[g] : nullptr;
    }
    c->layout_gen += 1;
    for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
    c->graphs.clear();
    char buf[96];
    c->cfg.clear();
    for (auto& lg : c->groups) {
        std::snprintf(buf, sizeof(buf), "%sK=%d rows_per_thread=%d tile=64x%d instances=%zu", c->cfg.empty() ? "" : "; ",
                      lg.g.K, lg.g.R, tile_h(lg.g.R), lg.members.size());
        c->cfg += buf;
        if (lg.team > 0) {
            std::snprintf(buf, sizeof(buf), " team=%d", lg.team);
            c->cfg += buf;
        }
        if (lg.g.grid_f > 0) {
            // the one-pass passes run on blocks of kStepNW waves
            std::snprintf(buf, sizeof(buf), " one-pass(tile=%dx%d)", kTW, kStepNW * lg.g.R);
            c->cfg += buf;
        }
        if (lg.g.cg1) c->cfg += " cg-one-pass";
        if (c->mfma && mf_member(c->dtype, lg.g.K) && (lg.g.R == 4 || lg.g.R == 8)) c->cfg += " mfma";
    }
    return MAID_OK;
}

// The team loops need every XCD's blocks to be the ones the XCC_ID register
// names and the hardware to deal blocks to the XCDs round-robin (block b to
// XCD (b + b0) mod 8); a map of one grid checks both.  Without it (another
// partitioning of the device, another dispatch order) the team path stays
// off.
hipError_t team_setup(maid_ctx* c) {
    int dev = 0, cus = 0, khz = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    if (e != hipSuccess) return e;
    c->cus_per_xcd = cus / kTeamXcd;
    // a member waits at most ~200 ms at a barrier
    c->team_wait = (int64_t)(khz > 0 ? khz : 100000) * 200;
    c->team_ok = false;
    if (cus % kTeamXcd != 0 || c->cus_per_xcd < 1) return hipSuccess;
    const int nblk = kTeamXcd * kTeamMax;
    int* d = nullptr;
    e = hipMalloc((void**)&d, nblk * sizeof(int));
    if (e != hipSuccess) return e;
    std::vector<int> h(nblk, -1);
    e = launch_team_map(d, c->cap);
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), d, nblk * sizeof(int), hipMemcpyDeviceToHost, c->cap);
    if (e == hipSuccess) e = hipStreamSynchronize(c->cap);
    (void)hipFree(d);
    if (e != hipSuccess) return e;
    bool ok = h[0] >= 0 && h[0] < kTeamXcd;
    for (int b = 0; b < nblk && ok; ++b) ok = h[b] == (b + h[0]) % kTeamXcd;
    c->team_ok = ok;
    return hipSuccess;
}

void destroy_ctx(maid_ctx* c) {
    if (!c) return;
    prof_harvest(c);
    for (hipEvent_t e : c->prof_pool) (void)hipEventDestroy(e);
    for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    if (c->ws) (void)hipFree(c->ws);
    if (c->st_dev) (void)hipFree(c->st_dev);
    if (c->st_host) (void)hipHostFree(c->st_host);
    if (c->pub) (void)hipHostFree(c->pub);
    if (c->tab_dev) (void)hipFree(c->tab_dev);
    if (c->tab_host) (void)hipHostFree(c->tab_host);
    if (c->maps) (void)hipFree(c->maps);
    if (c->sub_maps) (void)hipFree(c->sub_maps);
    if (c->sub_host) (void)hipHostFree(c->sub_host);
    if (c->team_arrive) (void)hipFree(c->team_arrive);
    if (c->adp_ws) (void)hipFree(c->adp_ws);
    if (c->ref64) destroy_ctx(c->ref64);
    delete c;
}

int create_ctx(const maid_desc* descs, int n, maid_ctx** out, std::string& why) {
    *out = nullptr;
    for (int i = 0; i < n; ++i) {
        int rc = validate_desc(&descs[i], why);
        if (rc) {
            if (n > 1) why = "instance " + std::to_string(i) + ": " + why;
            return rc;
        }
        if (descs[i].dtype != descs[0].dtype) {
            why = "all instances of a batch must share the storage type";
            return MAID_EINVAL;
        }
    }
    maid_ctx* c = new maid_ctx();
    c->n = n;
    c->dtype = descs[0].dtype;
    c->esz = c->dtype == MAID_F64 ? 8 : 4;
    c->m.resize(n);
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    size_t total = 0, maps = 0;
    // one buffer of taps: kc planes of up to 32 x 32 doubles
    auto kern_bytes = [&](const maid_desc& d) { return al((size_t)kplanes(d) * 1024 * 8); };
    for (int i = 0; i < n; ++i) {
        Member& M = c->m[i];
        std::memset(&M, 0, sizeof(M));
        M.d = descs[i];
        M.shape = Shape{M.d.C, M.d.H, M.d.W, M.d.K, M.d.reg};
        M.N = (int64_t)M.d.C * M.d.H * M.d.W;
        M.R_auto = auto_rows(M.shape);
        M.fuse_tuned = -1;
        M.nbe = (int)std::min<int64_t>((M.N + kNT - 1) / kNT, kEwMaxBlocks);
        const size_t img = al((size_t)M.N * c->esz);
        const size_t nblk = std::max<size_t>(std::max<size_t>(stencil_blocks(M.shape, 1), (size_t)M.nbe),
                                             (size_t)step_blocks(M.d.H, M.d.W, M.d.K, 1));
        const size_t part = al(nblk * sizeof(double));
        // FP64 s buffers of the one-pass CG, for instances that can take it
        const size_t s64 = step_ok(M.d.C, M.d.K, 1) ? 2 * al((size_t)M.N * sizeof(double)) : 0;
        total += s64;
        total += 21 * img + 6 * kern_bytes(M.d) + 9 * part + al((size_t)kHgMaxBlocks * 1024 * sizeof(double)) +
                 al(kTraceCap * sizeof(int));
        if (mf_member(c->dtype, M.d.K))
            total += 2 * al((size_t)kplanes(M.d) * mf_frag_bytes(M.d.K)) + al(kplanes(M.d) * sizeof(int));
        if (c->dtype == MAID_F32) total += 2 * al((size_t)M.N * sizeof(double));
        maps += round8(stencil_blocks(M.shape, 1)) + round8(M.nbe) + round8(step_blocks(M.d.H, M.d.W, M.d.K, 1));
    }
    c->ws_bytes = total;
    maps += n;   // the groups' instance lists
    c->maps_cap = maps;
    c->st_bytes = 256 + al(2 * n * sizeof(ApgState)) + 256 + al(3 * n * sizeof(CgState)) +
                  al(n * kRedSlots * sizeof(double));
    const size_t tab_bytes = (size_t)kRoles * n * sizeof(Inst<double>);
    hipError_t e = hipMalloc((void**)&c->ws, c->ws_bytes);
    if (e == hipSuccess) e = hipMalloc((void**)&c->st_dev, c->st_bytes);
    if (e == hipSuccess) e = hipHostMalloc((void**)&c->st_host, c->st_bytes, hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&c->pub, c->st_bytes + 256, hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) c->pub_flag = (unsigned*)(c->pub + c->st_bytes);
    if (e == hipSuccess) e = hipMalloc((void**)&c->tab_dev, tab_bytes);
    // mapped and coherent: the upload kernel reads it (the host rewrites it
    // only after the solve that read it has been waited for)
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&c->tab_host, tab_bytes, hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) e = hipMalloc((void**)&c->maps, maps * sizeof(int));
    if (e == hipSuccess && n > 1) e = hipMalloc((void**)&c->sub_maps, maps * sizeof(int));
    if (e == hipSuccess && n > 1) e = hipHostMalloc((void**)&c->sub_host, maps * sizeof(int), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMemset(c->ws, 0, c->ws_bytes);
    if (e == hipSuccess) e = hipMemset(c->st_dev, 0, c->st_bytes);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc((void**)&c->team_arrive, kTeamXcd * kTeamMax * sizeof(uint64_t));
    if (e == hipSuccess) e = hipMemset(c->team_arrive, 0, kTeamXcd * kTeamMax * sizeof(uint64_t));
    if (e == hipSuccess) e = team_setup(c);
    if (e != hipSuccess) {
        why = std::string("allocation failed: ") + hipGetErrorString(e);
        const int code = e == hipErrorOutOfMemory ? MAID_ENOMEM : MAID_EHIP;
        destroy_ctx(c);
        return code;
    }
    if (const char* g = std::getenv("MAID_GRAPHS")) c->use_graphs = std::strcmp(g, "0") != 0;
    if (const char* g = std::getenv("MAID_COMPACT")) c->compact = std::strcmp(g, "0") != 0;
    if (const char* t = std::getenv("MAID_TEAM")) c->team_req = std::max(-1, std::atoi(t));
    if (const char* f = std::getenv("MAID_FUSE")) c->fuse = std::strcmp(f, "0") != 0;
    if (const char* f = std::getenv("MAID_CG_ONE_PASS")) c->cg_fuse = std::strcmp(f, "0") != 0;
    if (const char* f = std::getenv("MAID_MFMA")) c->mfma = std::strcmp(f, "0") != 0;
    if (const char* u = std::getenv("MAID_UPLOAD_KERNEL")) c->upload_kernel = std::strcmp(u, "0") != 0;
    if (const char* u = std::getenv("MAID_PRED_FIRST")) c->pred_first = std::max(1, std::min(400, std::atoi(u)));
    if (const char* u = std::getenv("MAID_PRED_FIRST_CG")) c->pred_first_cg = std::max(1, std::min(400, std::atoi(u)));
    // longest wait at a team barrier, in wall-clock ticks (0 forces the
    // multi-kernel fallback, for tests)
    if (const char* w = std::getenv("MAID_TEAM_WAIT")) c->team_wait = std::max(0LL, std::atoll(w));
    // period of the exact recomputation of theta*x in the lower-level solve
    c->kx_resync = c->dtype == MAID_F64 ? 32 : 8;
    if (const char* r = std::getenv("MAID_KX_RESYNC")) c->kx_resync = std::max(0, std::atoi(r));
    // FP32 storage: a residual recomputed relative to the base point stays
    // accurate while x stays near it; the base moves (FP64 recomputation)
    // every 64 iterations.  FP64 storage needs no base moves.
    c->kx_resync_full = c->dtype == MAID_F64 ? 0 : 64;
    if (const char* r = std::getenv("MAID_KX_RESYNC_FULL")) c->kx_resync_full = std::max(0, std::atoi(r));
    if (c->kx_resync_full > 0 && c->kx_resync > 0 && c->kx_resync_full % c->kx_resync != 0)
        c->kx_resync_full = (c->kx_resync_full / c->kx_resync + 1) * c->kx_resync;
    std::memset(c->st_host, 0, c->st_bytes);
    std::memset(c->tab_host, 0, tab_bytes);
    {
        char* p = c->st_dev;
        c->team_err_apg = (unsigned*)p;
        p += 256;
        c->apg[0] = (ApgState*)p;
        c->apg[1] = c->apg[0] + n;
        p += al(2 * n * sizeof(ApgState));
        c->team_err_cg = (unsigned*)p;
        p += 256;
        c->cg[0] = (CgState*)p;
        c->cg[1] = c->cg[0] + n;
        c->cg[2] = c->cg[1] + n;
        p += al(3 * n * sizeof(CgState));
        c->red = (double*)p;
        c->apg_h = (ApgState*)(c->st_host + ((char*)c->apg[0] - c->st_dev));
        c->cg_h = (CgState*)(c->st_host + ((char*)c->cg[0] - c->st_dev));
        c->red_h = (double*)(c->st_host + ((char*)c->red - c->st_dev));
    }
    char* p = c->ws;
    auto take = [&](size_t b) { char* r = p; p += b; return (void*)r; };
    for (int i = 0; i < n; ++i) {
        Member& M = c->m[i];
        const size_t img = al((size_t)M.N * c->esz);
        const size_t nblk = std::max<size_t>(std::max<size_t>(stencil_blocks(M.shape, 1), (size_t)M.nbe),
                                             (size_t)step_blocks(M.d.H, M.d.W, M.d.K, 1));
        const size_t part = al(nblk * sizeof(double));
        for (int k = 0; k < 3; ++k) M.X[k] = take(img);
        for (int k = 0; k < 3; ++k) M.KX[k] = take(img);
        M.xb = take(img);
        M.rb = take(img);
        M.G = take(img);
        M.cq = take(img);
        M.cr = take(img);
        M.cP[0] = take(img);
        M.cP[1] = take(img);
        M.cKp = take(img);
        M.cHp = take(img);
        M.cV[0] = take(img);
        M.cV[1] = take(img);
        const bool s64 = step_ok(M.d.C, M.d.K, 1);
        M.cS64[0] = s64 ? (double*)take(al((size_t)M.N * sizeof(double))) : nullptr;
        M.cS64[1] = s64 ? (double*)take(al((size_t)M.N * sizeof(double))) : nullptr;
        M.tmp0 = take(img);
        M.tmp1 = take(img);
        for (int k = 0; k < 2; ++k)
            M.hg64[k] = c->dtype == MAID_F32 ? (double*)take(al((size_t)M.N * sizeof(double))) : (double*)(k ? M.tmp1 : M.tmp0);
        M.xtrial = take(img);
        M.gradg = take(img);
        const size_t kern = kern_bytes(M.d);
        M.th_c = take(kern);
        M.thf_c = take(kern);
        M.a_c = take(kern);
        M.af_c = take(kern);
        M.th_trial = (double*)take(kern);
        M.zbuf = (double*)take(kern);
        // pA, pB: two halves each for the one-pass form
        M.pA = (double*)take(2 * part);
        M.pB = (double*)take(2 * part);
        // pR, pK: two halves each for the one-pass CG form
        M.pR = (double*)take(2 * part);
        M.pK = (double*)take(2 * part);
        M.pC = (double*)take(part);
        M.hg_part = (double*)take(al((size_t)kHgMaxBlocks * 1024 * sizeof(double)));
        M.trace = (int*)take(al(kTraceCap * sizeof(int)));
        if (mf_member(c->dtype, M.d.K)) {
            for (int k = 0; k < 2; ++k) M.mf[k] = take(al((size_t)kplanes(M.d) * mf_frag_bytes(M.d.K)));
            M.mf_sh = (int*)take(al(kplanes(M.d) * sizeof(int)));
        }
    }
    int rc = relayout(c);
    if (rc) {
        why = c->err;
        destroy_ctx(c);
        return rc;
    }
    *out = c;
    return MAID_OK;
}

// ------------------------------------------------------------------ lower level (Algorithm 1, FISTA)
template <typename T>
int lower_batch(maid_ctx* c, const std::vector<char>& act, const std::vector<const double*>& theta,
                const std::vector<const T*>& y, const std::vector<T*>& x, const std::vector<double>& tol, int max_iter,
                double* L_inout, maid_solve_info* info, int* codes, int32_t* trace_bt, hipStream_t s,
                int pred_role, const std::vector<const T*>* xin) {
    const int n = c->n;
    Inst<T>* tab = tab_host<T>(c, ROLE_APG);
    const Inst<T>* tabd = tab_dev<T>(c, ROLE_APG);
    for (int i = 0; i < n; ++i) {
        ApgState& h = c->apg_h[i];
        std::memset(&h, 0, sizeof(h));
        h.status = ST_OK;
        fill_base(c, i, tab[i]);
        if (!act[i]) {
            h.done = 1;
            continue;
        }
        h.L = L_inout[i];
        h.t = 1.0;
        h.t_prev = 1.0;
        h.tol = tol[i];
        h.max_iter = max_iter;
        h.phase = PH_START;
        h.cur = 0;
        h.prev = 1;
        h.nxt = 2;
        h.trace_cap = kTraceCap;
        h.resync = c->kx_resync;
        h.resync_full = c->kx_resync > 0 ? c->kx_resync_full : 0;
        h.fixed = c->lower_fixed ? 1 : 0;
        Inst<T>& I = tab[i];
        if (n == 1) I.hist = (T*)c->lower_hist;
        I.y = y[i];
        I.xout = x[i];
        I.theta64 = theta[i];
        // set-up in one pass: X0 = X1 = x_start, KX0 = KX1 = theta*x_start - y
        // (FP64 taps and sums for FP32 storage), and the residual's base
        // point xb = x_start with rb = that residual
        I.cv_ker = I.thf;
        I.cv_mf = I.mf_thf;
        I.cv_mfsh = I.mf_sh;
        I.cv_ker64 = theta[i];
        I.cv_flip64 = 1;
        I.cv_in = xin ? (*xin)[i] : x[i];
        I.cv_sub = y[i];
        I.cv_out = I.KX[0];
        I.cv_out2 = I.KX[1];
        I.cv_out3 = I.rb;
        I.cv_cp[0] = I.X[0];
        I.cv_cp[1] = I.X[1];
        I.cv_cp[2] = I.xb;
    }
    // the initial states travel in the table; the preparation pass copies them
    for (int i = 0; i < n; ++i) tab[i].st0 = c->apg_h[i];
    SubLayout SL;
    TRY(sub_layout(c, act, SL, s));
    SL.apply(tab, act);
    std::vector<char> cur_act = act;
    {
        ProfScope ps_(c, MAID_PROF_OTHER, s);
        TRY(upload_prep<T>(c, ROLE_APG, 1, c->apg[0], nullptr, -1, s));
    }
    for (auto& lg : SL.groups)
        if (lg.g.grid > 0) LAUNCH(MAID_PROF_CONV, Ops<T>::conv(lg.g, tabd, s));
    // each slot is one gradient pass and one trial pass; a slot advances every
    // unfinished solve by one iteration or by one backtracking step
    const long slot_cap = (long)max_iter + 256 + 1;
    // groups of small instances: the whole loop in one launch per group
    std::vector<char> in_team(n, 0);
    bool graph_any = false;
    for (auto& lg : c->groups) {
        if (lg.team == 0) {
            graph_any = true;
            continue;
        }
        for (int i : lg.members) in_team[i] = 1;
        const TeamCtl ctl{c->team_arrive, c->team_err_apg, (++c->team_epoch) << 32, lg.team, c->team_wait};
        LAUNCH(MAID_PROF_APG_TEAM,
               Ops<T>::apg_team(lg.g, tabd, lg.list, (int)lg.members.size(), c->apg[0], ctl, slot_cap, s));
    }
    const size_t pub_bytes = 256 + n * sizeof(ApgState);
    if (graph_any) {
        const long pred = std::min(c->pred_slots[pred_role], (long)max_iter + 1);
        long slots = 0, chunk = 0;
        for (;;) {
            chunk = next_slots(pred, slots, chunk, c->pred_first);
            int rc = run_slots(c, G_APG, chunk, s, [&](hipStream_t s, int cnt) {
                // one-pass groups take two iterations per slot (state there and back)
                for (int k = 0; k < cnt; ++k) {
                    for (auto& lg : SL.groups) {
                        if (lg.team != 0 || lg.g.grid == 0) continue;
                        if (lg.g.grid_f > 0)
                            LAUNCH(MAID_PROF_APG_STEP, Ops<T>::apg_step(lg.g, tabd, c->apg[0], c->apg[1], s));
                        else
                            LAUNCH(MAID_PROF_APG_GRAD, Ops<T>::apg_grad(lg.g, tabd, c->apg[0], c->apg[1], s));
                    }
                    for (auto& lg : SL.groups) {
                        if (lg.team != 0 || lg.g.grid == 0) continue;
                        if (lg.g.grid_f > 0)
                            LAUNCH(MAID_PROF_APG_STEP, Ops<T>::apg_step(lg.g, tabd, c->apg[1], c->apg[0], s));
                        else
                            LAUNCH(MAID_PROF_APG_TRIAL, Ops<T>::apg_trial(lg.g, tabd, c->apg[1], c->apg[0], s));
                    }
                }
                return (int)MAID_OK;
            }, SL.full);
            if (rc) return rc;
            slots += chunk;
            TRY(publish(c, s, c->team_err_apg, pub_bytes));
            bool done = true;
            for (int i = 0; i < n; ++i) done = done && (c->apg_h[i].done || in_team[i]);
            if (done) break;
            if (slots > slot_cap) return fail(c, MAID_NONFINITE, "lower_solve: backtracking did not terminate");
            std::vector<char> still(n);
            for (int i = 0; i < n; ++i) still[i] = cur_act[i] && !c->apg_h[i].done && !in_team[i];
            TRY(shrink_layout<T>(c, SL, cur_act, still, tab, tabd, s));
        }
    } else {
        TRY(publish(c, s, c->team_err_apg, pub_bytes));
    }
    if (*(const unsigned*)(c->st_host + ((const char*)c->team_err_apg - c->st_dev)) != 0u) {
        // a team did not assemble (its blocks were not resident together):
        // repeat the solve on the multi-kernel passes, which the context
        // keeps using from now on
        HIP_TRY(hipMemsetAsync(c->team_err_apg, 0, sizeof(unsigned), s));
        c->team_ok = false;
        TRY(relayout(c));
        return lower_batch<T>(c, act, theta, y, x, tol, max_iter, L_inout, info, codes, trace_bt, s, pred_role, xin);
    }
    for (int i = 0; i < n; ++i)
        if (act[i] && !c->apg_h[i].done) return fail(c, MAID_NONFINITE, "lower_solve: backtracking did not terminate");
    {
        // one-pass instances: a pass per iteration or backtracking step, one
        // more at the start, two passes per slot
        long need = 1;
        for (int i = 0; i < n; ++i) {
            if (!act[i]) continue;
            const long steps = (long)c->apg_h[i].iters + c->apg_h[i].bt;
            need = std::max<long>(need, c->m[i].nbf > 0 ? (steps + 3) / 2 : steps + 1);
        }
        c->pred_slots[pred_role] = need;
    }
    if (c->prof_on) {
        // passes that did work: a gradient at the start and after every
        // accepted step, a trial for every accepted or rejected step (the
        // busiest instance of the batch); team loops: the slots of every
        // instance (each slot one trial pass and one gradient pass)
        // one-pass form: every pass but the one that finds the stop computes
        int64_t wg = 0, wt = 0, wteam = 0, wstep = 0;
        for (int i = 0; i < n; ++i)
            if (act[i] && in_team[i]) {
                wteam += c->apg_h[i].iters + c->apg_h[i].bt;
            } else if (act[i] && c->m[i].nbf > 0) {
                wstep = std::max<int64_t>(wstep, c->apg_h[i].iters + c->apg_h[i].bt + 1);
            } else if (act[i]) {
                wg = std::max<int64_t>(wg, c->apg_h[i].iters + 1);
                wt = std::max<int64_t>(wt, c->apg_h[i].iters + c->apg_h[i].bt);
            }
        c->prof_work[MAID_PROF_APG_GRAD] += wg;
        c->prof_work[MAID_PROF_APG_TRIAL] += wt;
        c->prof_work[MAID_PROF_APG_TEAM] += wteam;
        c->prof_work[MAID_PROF_APG_STEP] += wstep;
    }
    if (cur_act != act) {
        // the layout shrank during the solve: the returned points of every
        // instance of the solve are written over the full elementwise layout
        // (its inactive entries have no output and return at once)
        for (int i = 0; i < n; ++i) {
            tab[i].base = c->m[i].base;
            tab[i].basef = c->m[i].basef;
            tab[i].base_e = c->m[i].base_e;
        }
        HIP_TRY(hipMemcpyAsync(const_cast<Inst<T>*>(tabd), tab, (size_t)n * sizeof(Inst<T>), hipMemcpyHostToDevice, s));
        LAUNCH(MAID_PROF_OTHER, Ops<T>::apg_final(c->grid_e, c->blk_e, c->only_e, tabd, c->apg[0], s));
    } else if (SL.grid_e > 0) {
        LAUNCH(MAID_PROF_OTHER, Ops<T>::apg_final(SL.grid_e, SL.blk_e, SL.only_e, tabd, c->apg[0], s));
    }
    // (inside a MAID step the next work is stream-ordered after this pass,
    // and no host buffer it reads is still being copied: the last state
    // publication drained everything before it)
    if (!c->in_step) HIP_TRY(hipStreamSynchronize(s));
    for (int i = 0; i < n; ++i) {
        codes[i] = MAID_OK;
        if (!act[i]) continue;
        const ApgState& h = c->apg_h[i];
        codes[i] = status_code(h.status);
        if (codes[i] >= 0) L_inout[i] = h.L;
        if (info) {
            info[i].iters = h.iters;
            info[i].backtracks = h.bt;
            info[i].status = codes[i];
            info[i].res_norm = std::sqrt(h.gn2);
            info[i].obj = 0.0;
            info[i].L = h.L;
        }
    }
    if (trace_bt && n == 1 && c->apg_h[0].iters > 0) {
        const int cnt = std::min(c->apg_h[0].iters, kTraceCap);
        HIP_TRY(hipMemcpy(trace_bt, c->m[0].trace, cnt * sizeof(int), hipMemcpyDeviceToHost));
    }
    return MAID_OK;
}

// ------------------------------------------------------------------ adjoint (Algorithm 1, CG)
template <typename T>
int adjoint_batch(maid_ctx* c, const std::vector<char>& act, const std::vector<const double*>& theta,
                  const std::vector<const T*>& xt, const std::vector<const T*>& rhs, const std::vector<T*>& q,
                  const std::vector<double>& tol, int max_iter, maid_solve_info* info, int* codes, hipStream_t s) {
    const int n = c->n;
    Inst<T>* tab = tab_host<T>(c, ROLE_CG);
    const Inst<T>* tabd = tab_dev<T>(c, ROLE_CG);
    for (int i = 0; i < n; ++i) {
        CgState& h = c->cg_h[i];
        std::memset(&h, 0, sizeof(h));
        h.status = ST_OK;
        fill_base(c, i, tab[i]);
        if (!act[i]) {
            h.done = 1;
            continue;
        }
        h.tol = tol[i];
        h.max = max_iter;
        // one-pass form: its priming pass first (w_0 = H r_0 and the sums)
        h.first = c->m[i].nbf > 0 && c->cg_fuse ? 2 : 1;
        tab[i].xt = xt[i];
        tab[i].b = rhs[i];
        tab[i].q0 = q[i];
        tab[i].theta64 = theta[i];
    }
    for (int i = 0; i < n; ++i) tab[i].cg0 = c->cg_h[i];
    SubLayout SL;
    TRY(sub_layout(c, act, SL, s));
    SL.apply(tab, act);
    std::vector<char> cur_act = act;
    {
        ProfScope ps_(c, MAID_PROF_OTHER, s);
        TRY(upload_prep<T>(c, ROLE_CG, 1, nullptr, c->cg[0], -1, s));
    }
    // r = rhs - H q0 (the direction pass in set-up mode copies q0 into q and p)
    CgState** S = c->cg;
    for (auto& lg : SL.groups)
        if (lg.g.grid > 0) LAUNCH(MAID_PROF_CG_DIR, Ops<T>::cg_dir(lg.g, tabd, S[0], S[1], 1, s));
    for (auto& lg : SL.groups)
        if (lg.g.grid > 0) LAUNCH(MAID_PROF_CG_HVP, Ops<T>::cg_hvp(lg.g, tabd, S[0], S[2], 1, s));
    if (SL.grid_e > 0) LAUNCH(MAID_PROF_OTHER, Ops<T>::cg_init(SL.grid_e, SL.blk_e, SL.only_e, tabd, S[0], s));
    // groups of small instances: the whole loop in one launch per group
    std::vector<char> in_team(n, 0);
    bool graph_any = false;
    for (auto& lg : c->groups) {
        if (lg.team == 0) {
            graph_any = true;
            continue;
        }
        for (int i : lg.members) in_team[i] = 1;
        const TeamCtl ctl{c->team_arrive, c->team_err_cg, (++c->team_epoch) << 32, lg.team, c->team_wait};
        LAUNCH(MAID_PROF_CG_TEAM,
               Ops<T>::cg_team(lg.g, tabd, lg.list, (int)lg.members.size(), S[0], n, ctl, (long)max_iter + 2, s));
    }
    const size_t pub_bytes = 256 + n * sizeof(CgState);
    // the elementwise update pass serves the three-pass groups only
    bool hs_any = false;
    for (auto& lg : SL.groups) hs_any = hs_any || (lg.team == 0 && lg.g.grid > 0 && !lg.g.cg1);
    if (graph_any) {
        // one-pass groups: the priming pass and the first iteration
        for (auto& lg : SL.groups)
            if (lg.team == 0 && lg.g.grid > 0 && lg.g.cg1) {
                LAUNCH(MAID_PROF_CG_STEP, Ops<T>::cg_step(lg.g, tabd, S[0], S[1], s));
                LAUNCH(MAID_PROF_CG_STEP, Ops<T>::cg_step(lg.g, tabd, S[1], S[0], s));
            }
        const long pred = std::min(c->pred_slots[3], (long)max_iter + 1);
        long slots = 0, chunk = 0;
        for (;;) {
            chunk = next_slots(pred, slots, chunk, c->pred_first_cg);
            // one-pass groups take two iterations per slot (state there and back)
            int rc = run_slots(c, G_CG, chunk, s, [&](hipStream_t s, int cnt) {
                for (int k = 0; k < cnt; ++k) {
                    for (auto& lg : SL.groups) {
                        if (lg.team != 0 || lg.g.grid == 0) continue;
                        if (lg.g.cg1) LAUNCH(MAID_PROF_CG_STEP, Ops<T>::cg_step(lg.g, tabd, S[0], S[1], s));
                        else LAUNCH(MAID_PROF_CG_DIR, Ops<T>::cg_dir(lg.g, tabd, S[0], S[1], 0, s));
                    }
                    for (auto& lg : SL.groups) {
                        if (lg.team != 0 || lg.g.grid == 0) continue;
                        if (lg.g.cg1) LAUNCH(MAID_PROF_CG_STEP, Ops<T>::cg_step(lg.g, tabd, S[1], S[0], s));
                        else LAUNCH(MAID_PROF_CG_HVP, Ops<T>::cg_hvp(lg.g, tabd, S[1], S[2], 0, s));
                    }
                    if (hs_any)
                        LAUNCH(MAID_PROF_CG_UPDATE,
                               Ops<T>::cg_update(SL.grid_e, SL.blk_e, SL.only_e, tabd, S[2], S[0], s));
                }
                return (int)MAID_OK;
            }, SL.full);
            if (rc) return rc;
            slots += chunk;
            TRY(publish(c, s, c->team_err_cg, pub_bytes));
            bool done = true;
            for (int i = 0; i < n; ++i) done = done && (c->cg_h[i].done || in_team[i]);
            if (done) break;
            if (slots > (long)max_iter + 2) return fail(c, MAID_EHIP, "adjoint_solve: iteration count lost");
            std::vector<char> still(n);
            for (int i = 0; i < n; ++i) still[i] = cur_act[i] && !c->cg_h[i].done && !in_team[i];
            TRY(shrink_layout<T>(c, SL, cur_act, still, tab, tabd, s));
        }
    } else {
        TRY(publish(c, s, c->team_err_cg, pub_bytes));
    }
    if (*(const unsigned*)(c->st_host + ((const char*)c->team_err_cg - c->st_dev)) != 0u) {
        // a team did not assemble: repeat on the multi-kernel passes
        HIP_TRY(hipMemsetAsync(c->team_err_cg, 0, sizeof(unsigned), s));
        c->team_ok = false;
        TRY(relayout(c));
        return adjoint_batch<T>(c, act, theta, xt, rhs, q, tol, max_iter, info, codes, s);
    }
    for (int i = 0; i < n; ++i)
        if (act[i] && !c->cg_h[i].done) return fail(c, MAID_EHIP, "adjoint_solve: iteration count lost");
    {
        // one-pass instances: a pass per iteration after the two set-up
        // passes, two passes per slot
        long need = 1;
        for (int i = 0; i < n; ++i) {
            if (!act[i]) continue;
            const long it = c->cg_h[i].iters;
            need = std::max<long>(need, c->m[i].nbf > 0 && c->cg_fuse ? (it + 1) / 2 : it + 1);
        }
        c->pred_slots[3] = need;
    }
    if (c->prof_on) {
        // the set-up direction and Hessian passes, then one of each per
        // iteration; team loops: the iterations of every instance; one-pass
        // form: the priming pass and one per iteration
        int64_t w = 0, wteam = 0, wstep = 0;
        for (int i = 0; i < n; ++i)
            if (act[i] && in_team[i]) wteam += c->cg_h[i].iters;
            else if (act[i] && c->m[i].nbf > 0 && c->cg_fuse) wstep = std::max<int64_t>(wstep, c->cg_h[i].iters + 1);
            else if (act[i]) w = std::max<int64_t>(w, c->cg_h[i].iters);
        c->prof_work[MAID_PROF_CG_DIR] += w + 1;
        c->prof_work[MAID_PROF_CG_HVP] += w + 1;
        c->prof_work[MAID_PROF_CG_UPDATE] += w;
        c->prof_work[MAID_PROF_CG_TEAM] += wteam;
        c->prof_work[MAID_PROF_CG_STEP] += wstep;
    }
    for (int i = 0; i < n; ++i) {
        codes[i] = MAID_OK;
        if (!act[i]) continue;
        const CgState& h = c->cg_h[i];
        codes[i] = status_code(h.status);
        if (codes[i] >= 0)
            HIP_TRY(hipMemcpyAsync(q[i], c->m[i].cq, (size_t)c->m[i].N * sizeof(T), hipMemcpyDeviceToDevice, s));
        if (info) {
            info[i].iters = h.iters;
            info[i].backtracks = 0;
            info[i].status = codes[i];
            info[i].res_norm = std::sqrt(h.gamma);
            info[i].obj = 0.0;
            info[i].L = 0.0;
        }
    }
    if (!c->in_step) HIP_TRY(hipStreamSynchronize(s));
    return MAID_OK;
}

// ------------------------------------------------------------------ upper level at x
// rho = a*x - y, g = 1/2 ||rho||^2, grad = a . rho, ||grad||.
// With sob_theta, also r(theta_i) of the Sobolev term (Eq. 2.5) into r_out,
// read back with the same host round trip.
namespace {
template <typename T>
int upper_impl(maid_ctx* c, const std::vector<char>& act, const std::vector<const double*>& a,
               const std::vector<const T*>& y, const std::vector<const T*>& x, const std::vector<T*>& grad,
               double* g_out, double* gn_out, const std::vector<const double*>* sob_theta, double* r_out,
               hipStream_t s) {
    // prep(a) [+ ||a||_1] -> rho = a*x - y (partials in pC) -> grad = a.rho
    // (partials in pA; its block 0 sums pC) -> finish: sum pA [+ r(theta)]
    const int n = c->n;
    Inst<T>* t0 = tab_host<T>(c, ROLE_CV0);
    Inst<T>* t1 = tab_host<T>(c, ROLE_CV1);
    for (int i = 0; i < n; ++i) {
        fill_base(c, i, t0[i]);
        fill_base(c, i, t1[i]);
        if (!act[i]) continue;
        const Member& M = c->m[i];
        t0[i].th = (T*)M.a_c;
        t0[i].thf = (T*)M.af_c;
        t0[i].theta64 = a[i];
        t0[i].cv_ker = (T*)M.af_c;
        // the upper level convolves in FP64 (taps and sums): its residual
        // a*x - y is small next to a*x at a lower-level solution
        t0[i].cv_ker64 = a[i];
        t0[i].cv_flip64 = 1;
        t0[i].mf_th = t0[i].mf_thf = nullptr;
        t0[i].cv_in = x[i];
        t0[i].cv_sub = y[i];
        t0[i].cv_out = (T*)M.tmp0;
        t0[i].cv_part = M.pC;
        t1[i].cv_ker = (T*)M.a_c;
        t1[i].cv_ker64 = a[i];
        t1[i].cv_flip64 = 0;
        t1[i].cv_in = (T*)M.tmp0;
        t1[i].cv_out = grad[i] ? grad[i] : (T*)M.gradg;
        t1[i].cv_part = M.pA;
        t1[i].cv_prev_part = M.pC;
        t1[i].cv_prev_slot = kRedG;
        if (sob_theta && M.d.beta != 0.0) {
            t1[i].sob_th = (*sob_theta)[i];
            t1[i].sob_a = a[i];
            t1[i].beta = M.d.beta;
            t1[i].h1_w0 = M.d.h1_w0;
        }
    }
    const Inst<T>* d0 = tab_dev<T>(c, ROLE_CV0);
    const Inst<T>* d1 = tab_dev<T>(c, ROLE_CV1);
    {
        // ROLE_CV0 and ROLE_CV1 go up; the first is prepared
        ProfScope ps_(c, MAID_PROF_OTHER, s);
        TRY(upload_prep<T>(c, ROLE_CV0, 2, nullptr, nullptr, kRedAbs, s));
    }
    for (auto& lg : c->groups) LAUNCH(MAID_PROF_CONV, Ops<T>::conv(lg.g, d0, s));
    for (auto& lg : c->groups) LAUNCH(MAID_PROF_CONV, Ops<T>::conv(lg.g, d1, s));
    LAUNCH(MAID_PROF_OTHER, Ops<T>::finish(d1, n, kRedGrad, kRedSob, s));
    TRY(pull_red(c, s));
    for (int i = 0; i < n; ++i)
        if (act[i]) {
            if (g_out) g_out[i] = 0.5 * c->red_h[i * kRedSlots + kRedG];
            if (gn_out) gn_out[i] = std::sqrt(c->red_h[i * kRedSlots + kRedGrad]);
            if (sob_theta) r_out[i] = c->m[i].d.beta != 0.0 ? c->red_h[i * kRedSlots + kRedSob] : 0.0;
        }
    return MAID_OK;
}
}  // namespace

template <typename T>
int upper_batch(maid_ctx* c, const std::vector<char>& act, const std::vector<const double*>& a,
                const std::vector<const T*>& y, const std::vector<const T*>& x, const std::vector<T*>& grad,
                double* g_out, double* gn_out, hipStream_t s) {
    return upper_impl<T>(c, act, a, y, x, grad, g_out, gn_out, nullptr, nullptr, s);
}

// ------------------------------------------------------------------ Hessian product (Proposition 1)
// out = (theta.theta* + alpha grad^2 R(x)) w for a single instance: the set-up
// passes of the adjoint solve with q0 = w leave H q0 in the Hp buffer (the
// product its first residual rhs - H q0 is formed from), so the product is
// the CG kernels' own.
template <typename T>
int hessian_one(maid_ctx* c, const double* theta, const T* x, const T* w, T* out, hipStream_t s) {
    Inst<T>* tab = tab_host<T>(c, ROLE_CG);
    const Inst<T>* tabd = tab_dev<T>(c, ROLE_CG);
    const Member& M = c->m[0];
    CgState& h = c->cg_h[0];
    std::memset(&h, 0, sizeof(h));
    h.status = ST_OK;
    h.first = 1;
    fill_base(c, 0, tab[0]);
    tab[0].xt = x;
    tab[0].b = w;
    tab[0].q0 = w;
    tab[0].theta64 = theta;
    tab[0].cg0 = h;
    {
        ProfScope ps_(c, MAID_PROF_OTHER, s);
        TRY(upload_prep<T>(c, ROLE_CG, 1, nullptr, c->cg[0], -1, s));
    }
    CgState** S = c->cg;
    for (auto& lg : c->groups) LAUNCH(MAID_PROF_CG_DIR, Ops<T>::cg_dir(lg.g, tabd, S[0], S[1], 1, s));
    for (auto& lg : c->groups) LAUNCH(MAID_PROF_CG_HVP, Ops<T>::cg_hvp(lg.g, tabd, S[0], S[2], 1, s));
    HIP_TRY(hipMemcpyAsync(out, M.cHp, (size_t)M.N * sizeof(T), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return MAID_OK;
}

// ------------------------------------------------------------------ hypergradient (Eq. 3.2)
// znorm_out == nullptr: ||z||^2 stays in the reduction slots (no host
// round trip; the next read-back of the slots brings it).
namespace {
template <typename T>
int hypergrad_impl(maid_ctx* c, const std::vector<char>& act, const std::vector<const double*>& theta,
                   const std::vector<const double*>& a, const std::vector<const T*>& y, const std::vector<const T*>& xt,
                   const std::vector<const T*>& q, int with_r, const std::vector<double*>& z, double* znorm_out,
                   hipStream_t s) {
    const int n = c->n;
    Inst<T>* t2 = tab_host<T>(c, ROLE_CV2);
    Inst<T>* t3 = tab_host<T>(c, ROLE_CV3);
    for (int i = 0; i < n; ++i) {
        fill_base(c, i, t2[i]);
        fill_base(c, i, t3[i]);
        if (!act[i]) continue;
        const Member& M = c->m[i];
        t2[i].theta64 = theta[i];
        t2[i].cv_ker = (T*)M.thf_c;
        t2[i].cv_mf = t2[i].mf_thf;
        t2[i].cv_mfsh = t2[i].mf_sh;
        t2[i].cv_in = xt[i];
        t2[i].cv_sub = y[i];
        t2[i].cv_out = (T*)M.tmp0;
        // rho = theta*x - y is a small difference of large terms, and the two
        // correlations of Eq. 3.2 nearly cancel: with FP32 storage rho and
        // theta*q are formed with FP64 taps and sums and kept in FP64
        t2[i].cv_ker64 = theta[i];
        t2[i].cv_flip64 = 1;
        if (sizeof(T) == 4) t2[i].cv_out64 = M.hg64[0];
        t3[i].cv_ker = (T*)M.thf_c;
        t3[i].cv_mf = t3[i].mf_thf;
        t3[i].cv_mfsh = t3[i].mf_sh;
        t3[i].cv_in = q[i];
        t3[i].cv_out = (T*)M.tmp1;
        if (sizeof(T) == 4) {
            t3[i].cv_ker64 = theta[i];
            t3[i].cv_flip64 = 1;
            t3[i].cv_out64 = M.hg64[1];
        }
    }
    // the correlations and their finishing, batched per tile class: each
    // instance keeps its own block count, so z is bitwise the same in any batch
    int hg_blocks[2] = {0, 0};
    for (int i = 0; i < n; ++i) {
        if (!act[i]) continue;
        const Member& M = c->m[i];
        Inst<T>& I = t2[i];
        const int cls = M.d.K <= 16 ? 0 : 1;
        I.hg_rho = M.hg64[0];
        I.hg_w = M.hg64[1];
        I.hg_q = q[i];
        I.hg_part = M.hg_part;
        // per-channel kernels: kc equal block ranges, one per channel
        const int KP = kplanes(M.d);
        I.hg_nblk = KP == 1 ? std::min(kHgMaxBlocks, hg_items(M.shape))
                            : KP * std::min(kHgMaxBlocks / KP, hg_items(Shape{1, M.d.H, M.d.W, M.d.K, M.d.reg}));
        I.hg_base = hg_blocks[cls];
        hg_blocks[cls] += I.hg_nblk;
        I.hg_with_r = with_r && M.d.beta != 0.0;
        I.hg_a = I.hg_with_r ? a[i] : nullptr;
        I.beta = M.d.beta;
        I.h1_w0 = M.d.h1_w0;
        I.hg_z = z[i];
        I.hg_zn2 = c->red + (size_t)i * kRedSlots + kRedZ;
    }
    const Inst<T>* d2 = tab_dev<T>(c, ROLE_CV2);
    const Inst<T>* d3 = tab_dev<T>(c, ROLE_CV3);
    {
        // ROLE_CV2 and ROLE_CV3 go up; the first is prepared
        ProfScope ps_(c, MAID_PROF_OTHER, s);
        TRY(upload_prep<T>(c, ROLE_CV2, 2, nullptr, nullptr, -1, s));
    }
    for (auto& lg : c->groups) LAUNCH(MAID_PROF_CONV, Ops<T>::conv(lg.g, d2, s));
    for (auto& lg : c->groups) LAUNCH(MAID_PROF_CONV, Ops<T>::conv(lg.g, d3, s));
    for (int cls = 0; cls < 2; ++cls)
        if (hg_blocks[cls]) LAUNCH(MAID_PROF_HG_CORR, Ops<T>::hg_corr_batch(cls ? 32 : 16, hg_blocks[cls], d2, n, s));
    for (int cls = 0; cls < 2; ++cls)
        if (hg_blocks[cls]) LAUNCH(MAID_PROF_OTHER, Ops<T>::hg_final_batch(cls ? 32 : 16, d2, n, s));
    if (!znorm_out) return MAID_OK;
    TRY(pull_red(c, s));
    for (int i = 0; i < n; ++i)
        if (act[i]) znorm_out[i] = std::sqrt(c->red_h[i * kRedSlots + kRedZ]);
    return MAID_OK;
}
}  // namespace

template <typename T>
int hypergrad_batch(maid_ctx* c, const std::vector<char>& act, const std::vector<const double*>& theta,
                    const std::vector<const double*>& a, const std::vector<const T*>& y, const std::vector<const T*>& xt,
                    const std::vector<const T*>& q, int with_r, const std::vector<double*>& z, double* znorm_out,
                    hipStream_t s) {
    std::vector<double> zn(c->n, 0.0);
    TRY(hypergrad_impl<T>(c, act, theta, a, y, xt, q, with_r, z, zn.data(), s));
    if (znorm_out)
        for (int i = 0; i < c->n; ++i)
            if (act[i]) znorm_out[i] = zn[i];
    return MAID_OK;
}

int sobolev_batch(maid_ctx* c, const std::vector<char>& act, const std::vector<const double*>& theta,
                  const std::vector<const double*>& a, double* r_out, hipStream_t s) {
    bool any_work = false;
    for (int i = 0; i < c->n; ++i) {
        if (!act[i]) continue;
        const Member& M = c->m[i];
        if (M.d.beta == 0.0) {
            r_out[i] = 0.0;
            continue;
        }
        LAUNCH(MAID_PROF_OTHER, launch_sobolev(M.d.beta, M.d.h1_w0, theta[i], a[i], M.d.K, kplanes(M.d),
                                               c->red + (size_t)i * kRedSlots + kRedSob, s));
        any_work = true;
    }
    if (!any_work) return MAID_OK;
    TRY(pull_red(c, s));
    for (int i = 0; i < c->n; ++i)
        if (act[i] && c->m[i].d.beta != 0.0) r_out[i] = c->red_h[i * kRedSlots + kRedSob];
    return MAID_OK;
}

template <typename T>
int apply_operator_one(maid_ctx* c, const double* theta, const T* in, T* out, int adjoint, hipStream_t s) {
    Inst<T>* t = tab_host<T>(c, ROLE_CV0);
    fill_base(c, 0, t[0]);
    t[0].theta64 = theta;
    t[0].cv_ker = adjoint ? t[0].th : t[0].thf;
    t[0].cv_mf = adjoint ? t[0].mf_th : t[0].mf_thf;
    t[0].cv_mfsh = t[0].mf_sh;
    t[0].cv_in = in;
    t[0].cv_out = out;
    TRY(upload<T>(c, ROLE_CV0, s));
    const Inst<T>* d = tab_dev<T>(c, ROLE_CV0);
    LAUNCH(MAID_PROF_OTHER, Ops<T>::prep_kernel(d, 1, nullptr, nullptr, -1, s));
    for (auto& lg : c->groups) LAUNCH(MAID_PROF_CONV, Ops<T>::conv(lg.g, d, s));
    HIP_TRY(hipStreamSynchronize(s));
    return MAID_OK;
}

// ------------------------------------------------------------------ autotuner
// For every candidate tile height (rows per thread 1, 2, 4, and 8 for
// K >= 5), and with each of the two forms of the lower-level iteration
// where the one-pass form applies (one channel, 3 <= K <= 11, rows <= 4),
// all instances take that candidate; a short lower-level solve and a short
// CG solve (fixed iteration counts, tolerance 0, on the caller's data,
// writing only workspace) run with per-launch timing, and the GPU time of
// the solver passes is summed per kernel size K.  Each K group keeps its
// fastest candidate.  The caller's own timing state is restored.
template <typename T>
int autotune_batch(maid_ctx* c, const std::vector<const double*>& theta, const std::vector<const T*>& y, int probe_iters,
                   int32_t* rows_out, hipStream_t s) {
    const int n = c->n;
    const int cands[4] = {1, 2, 4, 8};
    std::vector<int> Ks;
    for (int i = 0; i < n; ++i)
        if (std::find(Ks.begin(), Ks.end(), c->m[i].d.K) == Ks.end()) Ks.push_back(c->m[i].d.K);
    std::vector<double> best(Ks.size(), 1e300);
    std::vector<int> best_R(Ks.size(), 0), best_F(Ks.size(), 0);
    // keep the caller's timing state
    prof_harvest(c);
    const bool prof_was = c->prof_on;
    int64_t sv_l[MAID_PROF_KINDS], sv_w[MAID_PROF_KINDS];
    double sv_ms[MAID_PROF_KINDS];
    std::memcpy(sv_l, c->prof_launches, sizeof(sv_l));
    std::memcpy(sv_w, c->prof_work, sizeof(sv_w));
    std::memcpy(sv_ms, c->prof_ms, sizeof(sv_ms));
    const int R_over = c->R_override;
    int rc = MAID_OK;
    std::vector<T*> xs(n);
    std::vector<const T*> xsc(n), rhs(n);
    std::vector<T*> qs(n);
    for (int i = 0; i < n; ++i) {
        xs[i] = (T*)c->m[i].xtrial;
        xsc[i] = xs[i];
        rhs[i] = y[i];
        qs[i] = (T*)c->m[i].tmp1;
    }
    std::vector<double> tol(n, 0.0), L(n, 0.0);
    std::vector<int> codes(n);
    for (int k = 0; k < (int)Ks.size() && rc == MAID_OK; ++k) {
        std::vector<char> act(n, 0);
        for (int i = 0; i < n; ++i) act[i] = c->m[i].d.K == Ks[k];
        // the one-pass FISTA form is a candidate where every instance of this K allows it
        bool fuse_ok = c->fuse && c->fuse_pin == 1;   // the one-pass form only where opted in
        for (int i = 0; i < n; ++i)
            if (act[i]) fuse_ok = fuse_ok && step_ok(c->m[i].d.C, c->m[i].d.K, 1);
        for (int cj = 0; cj < 8 && rc == MAID_OK; ++cj) {
            const int ci = cj >> 1, f = cj & 1;
            if (cands[ci] > max_rows(Ks[k])) continue;
            // the form the layout will take: one-pass where pinned and possible
            const bool one = fuse_ok && step_ok(1, Ks[k], cands[ci]);
            if (f != (one ? 1 : 0)) continue;
            c->R_override = cands[ci];
            c->fuse_force = f;
            if ((rc = relayout(c))) break;
            // twice: the first run sets the slot predictors of this layout
            // (so that neither form pays for launches past the end), the
            // second is timed
            for (int rep = 0; rep < 2 && rc == MAID_OK; ++rep) {
                for (int i = 0; i < n; ++i)
                    if (act[i]) {
                        const size_t bytes = (size_t)c->m[i].N * sizeof(T);
                        hipError_t e = hipMemcpyAsync(xs[i], y[i], bytes, hipMemcpyDeviceToDevice, s);
                        if (e == hipSuccess) e = hipMemsetAsync(qs[i], 0, bytes, s);
                        if (e != hipSuccess) {
                            rc = fail(c, MAID_EHIP, std::string("autotune: ") + hipGetErrorString(e));
                            break;
                        }
                        L[i] = 0.0;
                    }
                if (rc) break;
                c->prof_on = true;
                for (int t = 0; t < MAID_PROF_KINDS; ++t) c->prof_ms[t] = 0.0;
                rc = lower_batch<T>(c, act, theta, y, xs, tol, probe_iters, L.data(), nullptr, codes.data(), nullptr,
                                    s);
                if (rc == MAID_OK)
                    rc = adjoint_batch<T>(c, act, theta, xsc, rhs, qs, tol, probe_iters, nullptr, codes.data(), s);
                prof_harvest(c);
                c->prof_on = false;
            }
            if (rc) break;
            const double t = c->prof_ms[MAID_PROF_APG_GRAD] + c->prof_ms[MAID_PROF_APG_TRIAL] +
                             c->prof_ms[MAID_PROF_APG_STEP] + c->prof_ms[MAID_PROF_CG_DIR] +
                             c->prof_ms[MAID_PROF_CG_HVP] + c->prof_ms[MAID_PROF_APG_TEAM] +
                             c->prof_ms[MAID_PROF_CG_TEAM] + c->prof_ms[MAID_PROF_CG_STEP] +
                             c->prof_ms[MAID_PROF_CG_UPDATE];
            if (t < best[k]) {
                best[k] = t;
                best_R[k] = cands[ci];
                best_F[k] = f;
            }
        }
    }
    std::memcpy(c->prof_launches, sv_l, sizeof(sv_l));
    std::memcpy(c->prof_work, sv_w, sizeof(sv_w));
    std::memcpy(c->prof_ms, sv_ms, sizeof(sv_ms));
    c->prof_on = prof_was;
    c->R_override = R_over;
    c->fuse_force = -1;
    if (rc == MAID_OK)
        for (int i = 0; i < n; ++i)
            for (size_t k = 0; k < Ks.size(); ++k)
                if (c->m[i].d.K == Ks[k]) {
                    c->m[i].R_tuned = best_R[k];
                    c->m[i].fuse_tuned = best_F[k];
                }
    const int rc2 = relayout(c);
    if (rc) return rc;
    if (rc2) return rc2;
    if (rows_out)
        for (int i = 0; i < n; ++i) rows_out[i] = c->m[i].R;
    return MAID_OK;
}

// ------------------------------------------------------------------ MAID (Algorithm 2)
// One outer iteration per instance, in lockstep: every round computes
// InexactGradient for the instances that need one (one batched lower solve,
// upper-level pass, CG solve and hypergradient), then runs the psi trials of
// Eq. (3.4) as batched lower solves over the instances still testing step
// sizes; an instance whose j trials all fail shrinks its accuracies and
// joins the next round.  Each instance takes exactly the decisions, and
// performs exactly the solves, it would take on its own.
namespace {
// Decision-trace records (layout declared with maid_set_step_trace).
void tr_w(maid_ctx* c, int32_t w) {
    auto& t = c->strace;
    if (t.n_w >= t.cap_w) { t.full = true; return; }
    t.w[t.n_w++] = w;
}
void tr_v(maid_ctx* c, double v) {
    auto& t = c->strace;
    if (t.n_v >= t.cap_v) { t.full = true; return; }
    t.v[t.n_v++] = v;
}
// a lower-level solve of instance i that just finished on stream s
int tr_lower(maid_ctx* c, int i, int role, const maid_solve_info& li, hipStream_t s) {
    tr_w(c, 1);
    tr_w(c, role);
    tr_w(c, li.iters);
    tr_w(c, li.status);
    if (li.iters > 0) {
        std::vector<int32_t> bt(std::min(li.iters, kTraceCap));
        HIP_TRY(hipMemcpyAsync(bt.data(), c->m[i].trace, bt.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        for (int k = 0; k < li.iters; ++k) tr_w(c, k < (int)bt.size() ? bt[k] : -1);
    }
    tr_v(c, li.res_norm);
    tr_v(c, li.L);
    return MAID_OK;
}
}  // namespace

template <typename T>
int step_batch(maid_ctx* c, const std::vector<const double*>& a, const std::vector<const T*>& y, maid_state* st,
               const maid_hparams* hp, maid_step_info* out, int* codes, hipStream_t s, const std::vector<char>* active) {
    struct InStep {
        maid_ctx* c;
        InStep(maid_ctx* cc) : c(cc) { c->in_step = true; }
        ~InStep() { c->in_step = false; }
    } in_step_guard(c);
    const int n = c->n;
    std::vector<maid_step_info> I(n);
    std::memset(I.data(), 0, n * sizeof(maid_step_info));
    // the decision trace (one instance): every call writes it from the start
    const int ti = (c->strace.w && c->strace.v && c->strace.inst >= 0 && c->strace.inst < n) ? c->strace.inst : -1;
    c->strace.n_w = c->strace.n_v = 0;
    c->strace.full = false;
    // L_g <= 0: ||a||_1^2, from the first upper-level read-back (its prep of a
    // leaves ||a||_1 in the reduction slots)
    std::vector<double> Lg(n, hp->L_g);
    bool have_Lg = hp->L_g > 0;
    std::vector<const double*> theta(n), th2c(n);
    std::vector<double*> th2(n), z(n);
    std::vector<T*> x(n), q(n), xs(n), grad(n), none(n, nullptr);
    std::vector<const T*> xc(n), qc(n), xsc(n), gradc(n);
    for (int i = 0; i < n; ++i) {
        theta[i] = (const double*)st[i].theta;
        x[i] = (T*)st[i].x;
        q[i] = (T*)st[i].q;
        xc[i] = x[i];
        qc[i] = q[i];
        xs[i] = (T*)c->m[i].xtrial;
        xsc[i] = xs[i];
        grad[i] = (T*)c->m[i].gradg;
        gradc[i] = grad[i];
        th2[i] = c->m[i].th_trial;
        th2c[i] = th2[i];
        z[i] = c->m[i].zbuf;
        codes[i] = MAID_OK;
    }
    std::vector<int> j(n, hp->max_bt), rc(n);
    std::vector<char> need = active ? *active : std::vector<char>(n, 1);
    std::vector<double> tol(n), dtol(n), L(n), g_k(n), n_k(n), r_k(n), ell_k(n), znorm(n), g_n(n), n_n(n), r_n(n);
    std::vector<maid_solve_info> li(n), ci(n);
    while (any(need)) {
        // InexactGradient(theta_k, eps_k, delta_k)
        for (int i = 0; i < n; ++i) {
            tol[i] = st[i].eps * hp->mu;
            dtol[i] = st[i].delta;
            L[i] = st[i].L;
        }
        TRY(lower_batch<T>(c, need, theta, y, x, tol, hp->max_lower_iter, L.data(), li.data(), rc.data(), nullptr, s, 1));
        for (int i = 0; i < n; ++i) {
            if (!need[i]) continue;
            if (rc[i] < 0) {
                codes[i] = rc[i];
                need[i] = 0;
                continue;
            }
            st[i].L = L[i];
            I[i].lower_iters += li[i].iters;
            if (rc[i] == MAID_MAXITER) I[i].lower_status = MAID_MAXITER;
            if (i == ti) TRY(tr_lower(c, i, 0, li[i], s));
        }
        TRY(upper_impl<T>(c, need, a, y, xc, grad, g_k.data(), n_k.data(), &theta, r_k.data(), s));
        if (ti >= 0 && need[ti]) {
            tr_w(c, 2);
            tr_w(c, 0);
            tr_v(c, g_k[ti]);
            tr_v(c, n_k[ti]);
            tr_v(c, r_k[ti]);
        }
        if (!have_Lg) {
            for (int i = 0; i < n; ++i)
                if (need[i]) Lg[i] = c->red_h[i * kRedSlots + kRedAbs] * c->red_h[i * kRedSlots + kRedAbs];
            have_Lg = true;
        }
        TRY(adjoint_batch<T>(c, need, theta, xc, gradc, q, dtol, hp->max_cg_iter, ci.data(), rc.data(), s));
        for (int i = 0; i < n; ++i) {
            if (!need[i]) continue;
            I[i].cg_iters += ci[i].iters;
            if (i == ti) {
                tr_w(c, 3);
                tr_w(c, ci[i].iters);
                tr_w(c, rc[i]);
                tr_v(c, ci[i].res_norm);
            }
            if (rc[i] < 0) {
                codes[i] = rc[i];
                need[i] = 0;
            }
            if (rc[i] == MAID_MAXITER) I[i].cg_status = MAID_MAXITER;
        }
        // ||z|| comes back with the first trial's read-back (a traced step
        // reads it back at once, for its record)
        bool have_znorm = false;
        if (ti >= 0 && need[ti]) {
            std::vector<double> zn(n, 0.0);
            TRY(hypergrad_impl<T>(c, need, theta, a, y, xc, qc, 1, z, zn.data(), s));
            for (int i = 0; i < n; ++i)
                if (need[i]) {
                    znorm[i] = zn[i];
                    I[i].znorm = zn[i];
                }
            have_znorm = true;
            tr_w(c, 4);
            tr_v(c, znorm[ti]);
        } else {
            TRY(hypergrad_impl<T>(c, need, theta, a, y, xc, qc, 1, z, nullptr, s));
        }
        for (int i = 0; i < n; ++i)
            if (need[i]) {
                ell_k[i] = g_k[i] + r_k[i];
                I[i].ell_k = ell_k[i];
            }
        // the psi trials
        std::vector<char> tr = need;
        std::vector<int> cnt(n, 0);
        while (any(tr)) {
            for (int i = 0; i < n; ++i) {
                if (!tr[i]) continue;
                const int KK = kplanes(c->m[i].d) * c->m[i].d.K * c->m[i].d.K;
                LAUNCH(MAID_PROF_OTHER, launch_theta_step(theta[i], z[i], st[i].step, th2[i], KK, s));
                L[i] = st[i].L;
            }
            // the trial solve starts from x and returns in xs
            TRY(lower_batch<T>(c, tr, th2c, y, xs, tol, hp->max_lower_iter, L.data(), li.data(), rc.data(), nullptr, s,
                               2, &xc));
            for (int i = 0; i < n; ++i) {
                if (!tr[i]) continue;
                if (rc[i] < 0) {
                    codes[i] = rc[i];
                    tr[i] = 0;
                    need[i] = 0;
                    continue;
                }
                st[i].L = L[i];
                I[i].lower_iters += li[i].iters;
                if (rc[i] == MAID_MAXITER) I[i].lower_status = MAID_MAXITER;
                if (i == ti) TRY(tr_lower(c, i, 1, li[i], s));
            }
            TRY(upper_impl<T>(c, tr, a, y, xsc, none, g_n.data(), n_n.data(), &th2c, r_n.data(), s));
            if (ti >= 0 && tr[ti]) {
                tr_w(c, 2);
                tr_w(c, 1);
                tr_v(c, g_n[ti]);
                tr_v(c, n_n[ti]);
                tr_v(c, r_n[ti]);
            }
            if (!have_znorm) {
                for (int i = 0; i < n; ++i)
                    if (need[i]) {
                        znorm[i] = std::sqrt(c->red_h[i * kRedSlots + kRedZ]);
                        I[i].znorm = znorm[i];
                    }
                have_znorm = true;
            }
            for (int i = 0; i < n; ++i) {
                if (!tr[i]) continue;
                const double ell_n = g_n[i] + r_n[i];
                const double e = st[i].eps;
                const double psi = ell_n + n_n[i] * e + 0.5 * Lg[i] * e * e - ell_k[i] + n_k[i] * e +
                                   hp->lambda * st[i].step * znorm[i] * znorm[i];
                I[i].trials += 1;
                I[i].psi = psi;
                I[i].ell_next = ell_n;
                if (i == ti) {
                    tr_w(c, 5);
                    tr_w(c, psi <= 0.0 ? 1 : 0);
                    tr_v(c, psi);
                }
                if (psi <= 0.0) {
                    const int KK = kplanes(c->m[i].d) * c->m[i].d.K * c->m[i].d.K;
                    HIP_TRY(hipMemcpyAsync(st[i].theta, th2[i], KK * sizeof(double), hipMemcpyDeviceToDevice, s));
                    HIP_TRY(hipMemcpyAsync(x[i], xs[i], (size_t)c->m[i].N * sizeof(T), hipMemcpyDeviceToDevice, s));
                    st[i].eps *= hp->nu_hi;
                    st[i].delta *= hp->nu_hi;
                    st[i].step *= hp->rho_hi;
                    st[i].k += 1;
                    I[i].accepted = 1;
                    tr[i] = 0;
                    need[i] = 0;
                    continue;
                }
                st[i].step *= hp->rho_lo;
                if (++cnt[i] >= j[i]) tr[i] = 0;
            }
        }
        for (int i = 0; i < n; ++i) {
            if (!need[i]) continue;
            st[i].eps *= hp->nu_lo;
            st[i].delta *= hp->nu_lo;
            j[i] += 1;
            I[i].retries += 1;
            if (st[i].eps < hp->eps_min) {
                codes[i] = MAID_ACCURACY_FLOOR;
                need[i] = 0;
            }
        }
    }
    for (int i = 0; i < n; ++i) {
        // a solve that stopped at its iteration cap was carried on with; the
        // step says so (a warning) unless it ended in another state
        if (codes[i] == MAID_OK && (I[i].lower_status == MAID_MAXITER || I[i].cg_status == MAID_MAXITER))
            codes[i] = MAID_MAXITER;
        I[i].status = codes[i];
        if (out) out[i] = I[i];
    }
    if (c->strace.full) return fail(c, MAID_EINVAL, "maid_step: the decision trace buffers are too small");
    // the step's array outputs (theta, x, q) are complete when it returns
    HIP_TRY(hipStreamSynchronize(s));
    return MAID_OK;
}

// The precision form's refinement of a lower-level solution: Newton steps
// x <- x - d with H(x) d = grad h(x) (Proposition 1's Hessian and gradient),
// d from CG in the storage type to cg_rel relative residual.  With FP64
// storage the gradient comes from a zero-iteration lower-level solve.  With
// FP32 storage this is mixed-precision iterative refinement: the iterate is
// accumulated in FP64 (x64), its gradient evaluated by the FP64 passes of a
// companion FP64 context of the same shape (FP64 storage and arithmetic:
// the gradient's cancellations stay in FP64), rounded to FP32 as CG's
// right-hand side, and the FP32 CG correction added to x64; x is x64 rounded
// once at each step.  d is small next to x, so its FP32 rounding is too.
// Stops when ||d|| <= rel_tol ||x||, when the steps stop shrinking (the last
// one is undone), or after max_newton steps.
namespace {
// the FP64 companion of an FP32 context (created at the first refinement,
// on the two-pass form so that the gradient lands in its G)
int companion64(maid_ctx* c, maid_ctx** out) {
    if (!c->ref64) {
        maid_desc d = c->m[0].d;
        d.dtype = MAID_F64;
        std::string why;
        maid_ctx* r = nullptr;
        const int rc = create_ctx(&d, 1, &r, why);
        if (rc) return fail(c, rc, "refinement: FP64 companion context: " + why);
        r->fuse = false;
        r->team_req = 0;
        const int rr = relayout(r);
        if (rr) {
            destroy_ctx(r);
            return fail(c, rr, "refinement: FP64 companion layout failed");
        }
        c->ref64 = r;
    }
    *out = c->ref64;
    return MAID_OK;
}
}  // namespace

template <typename T>
int refine_one(maid_ctx* c, const double* theta, const T* y, T* x, double rel_tol, int max_newton, int max_cg,
               double cg_rel, maid_refine_info* out, hipStream_t s) {
    constexpr bool kMixed = sizeof(T) == 4;
    Member& M = c->m[0];
    // FP32: the FP64 companion, x64 and y64 in its workspace
    maid_ctx* c64 = nullptr;
    double* x64 = nullptr;
    double* y64 = nullptr;
    if constexpr (kMixed) {
        TRY(companion64(c, &c64));
        y64 = (double*)c64->m[0].tmp0;
        x64 = (double*)c64->m[0].tmp1;
        HIP_TRY((launch_cast<float, double>((const float*)y, y64, M.N, s)));
        HIP_TRY((launch_cast<float, double>((const float*)x, x64, M.N, s)));
    }
    // FP64 storage: the gradient must land in the workspace's G (two-pass form)
    const bool fuse = c->fuse;
    if (!kMixed && fuse) {
        c->fuse = false;
        TRY(relayout(c));
    }
    auto restore = [&]() -> int {
        if (kMixed || !fuse) return MAID_OK;
        c->fuse = true;
        return relayout(c);
    };
    maid_refine_info r{};
    T* G = (T*)M.G;
    T* d = (T*)M.xtrial;
    double* part = M.hg_part;
    constexpr int kBlocks = 512;
    std::vector<double> hp(2 * kBlocks);
    double prev_step = HUGE_VAL;
    int rc = MAID_OK;
    for (int k = 0; k <= max_newton; ++k) {
        // gradient at x (a zero-iteration solve rewrites x with the same values)
        double L = 0.0;
        maid_solve_info gi{};
        int code = MAID_OK;
        if constexpr (kMixed) {
            rc = lower_batch<double>(c64, std::vector<char>(1, 1), std::vector<const double*>(1, theta),
                                     std::vector<const double*>(1, y64), std::vector<double*>(1, x64),
                                     std::vector<double>(1, 0.0), 0, &L, &gi, &code, nullptr, s);
            if (rc) rc = fail(c, rc, "refinement: FP64 gradient: " + c64->err);
        } else {
            rc = lower_batch<T>(c, std::vector<char>(1, 1), std::vector<const double*>(1, theta),
                                std::vector<const T*>(1, y), std::vector<T*>(1, x), std::vector<double>(1, 0.0), 0, &L,
                                &gi, &code, nullptr, s);
        }
        if (rc == MAID_OK && code < 0) rc = code;
        if (rc) break;
        r.grad_norm = gi.res_norm;
        if (k == max_newton || r.grad_norm == 0.0) break;
        if constexpr (kMixed) HIP_TRY((launch_cast<double, float>((const double*)c64->m[0].G, (float*)G, M.N, s)));
        // Newton direction: CG from zero on H(x) d = G
        HIP_TRY(hipMemsetAsync(d, 0, (size_t)M.N * sizeof(T), s));
        maid_solve_info ci{};
        code = MAID_OK;
        rc = adjoint_batch<T>(c, std::vector<char>(1, 1), std::vector<const double*>(1, theta), std::vector<const T*>(1, x),
                              std::vector<const T*>(1, G), std::vector<T*>(1, d),
                              std::vector<double>(1, cg_rel * r.grad_norm), max_cg, &ci, &code, s);
        if (rc == MAID_OK && code < 0) rc = code;
        if (rc) break;
        r.cg_iters += ci.iters;
        if constexpr (kMixed)
            HIP_TRY(launch_axpy_mixed(x64, (const float*)d, -1.0, M.N, (float*)x, part, kBlocks, s));
        else
            HIP_TRY(launch_axpy_norms<T>(x, d, T(-1), M.N, part, kBlocks, s));
        HIP_TRY(hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        double dd = 0.0, xx = 0.0;
        for (int b = 0; b < kBlocks; ++b) {
            dd += hp[2 * b];
            xx += hp[2 * b + 1];
        }
        const double step = xx > 0.0 ? std::sqrt(dd / xx) : 0.0;
        r.newton_steps += 1;
        if (step > prev_step) {
            // the steps grew: undo this one and stop
            if constexpr (kMixed)
                HIP_TRY(launch_axpy_mixed(x64, (const float*)d, 1.0, M.N, (float*)x, part, kBlocks, s));
            else
                HIP_TRY(launch_axpy_norms<T>(x, d, T(1), M.N, part, kBlocks, s));
            r.newton_steps -= 1;
            r.status = MAID_MAXITER;
            prev_step = step;
            max_newton = k + 1;   // one more gradient, at the restored point
            continue;
        }
        r.rel_step = step;
        prev_step = step;
        if (step <= rel_tol) max_newton = k + 1;   // converged: report the gradient there
    }
    if (rc == MAID_OK && r.status == MAID_OK && r.rel_step > rel_tol) r.status = MAID_MAXITER;
    if (kMixed && rc == MAID_OK) HIP_TRY(hipStreamSynchronize(s));
    const int rr = restore();
    if (out) *out = r;
    if (rc) return rc;
    return rr;
}


#define MAID_ENGINE_INSTANTIATE(T)                                                                                       \
    template int lower_batch<T>(maid_ctx*, const std::vector<char>&, const std::vector<const double*>&,                 \
                                const std::vector<const T*>&, const std::vector<T*>&, const std::vector<double>&, int,  \
                                double*, maid_solve_info*, int*, int32_t*, hipStream_t, int,                            \
                                const std::vector<const T*>*);                                                           \
    template int adjoint_batch<T>(maid_ctx*, const std::vector<char>&, const std::vector<const double*>&,               \
                                  const std::vector<const T*>&, const std::vector<const T*>&, const std::vector<T*>&,   \
                                  const std::vector<double>&, int, maid_solve_info*, int*, hipStream_t);                 \
    template int upper_batch<T>(maid_ctx*, const std::vector<char>&, const std::vector<const double*>&,                 \
                                const std::vector<const T*>&, const std::vector<const T*>&, const std::vector<T*>&,     \
                                double*, double*, hipStream_t);                                                          \
    template int hypergrad_batch<T>(maid_ctx*, const std::vector<char>&, const std::vector<const double*>&,             \
                                    const std::vector<const double*>&, const std::vector<const T*>&,                    \
                                    const std::vector<const T*>&, const std::vector<const T*>&, int,                    \
                                    const std::vector<double*>&, double*, hipStream_t);                                  \
    template int apply_operator_one<T>(maid_ctx*, const double*, const T*, T*, int, hipStream_t);                       \
    template int autotune_batch<T>(maid_ctx*, const std::vector<const double*>&, const std::vector<const T*>&, int,   \
                                   int32_t*, hipStream_t);                                                               \
    template int step_batch<T>(maid_ctx*, const std::vector<const double*>&, const std::vector<const T*>&, maid_state*, \
                               const maid_hparams*, maid_step_info*, int*, hipStream_t, const std::vector<char>*);  \
    template int refine_one<T>(maid_ctx*, const double*, const T*, T*, double, int, int, double, maid_refine_info*,   \
                               hipStream_t);                                                                            \
    template int hessian_one<T>(maid_ctx*, const double*, const T*, const T*, T*, hipStream_t);

MAID_ENGINE_INSTANTIATE(float)
MAID_ENGINE_INSTANTIATE(double)

}  // namespace maid
