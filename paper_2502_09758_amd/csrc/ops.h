// ops.h -- host-side launchers of the libmaid kernels, one set per storage
// type.  Stencil passes are launched per group (instances sharing the kernel
// size K and the rows-per-thread tile parameter R, dispatched to the
// matching template instantiation); elementwise passes cover every instance
// of the table in one launch.  All launches are asynchronous on `s`.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "devctx.h"

namespace maid {

struct Shape {
    int C, H, W, K, reg;
};

// blocks of one stencil pass: one per tile and channel
inline int stencil_blocks(const Shape& d, int R) {
    return ((d.W + kTW - 1) / kTW) * ((d.H + tile_h(R) - 1) / tile_h(R)) * d.C;
}

// Rows per thread: 1, 2, 4, and 8 for the kernels staged one tile after the
// other (K >= 5), whose convolution reuses each staged column value over
// more outputs.
inline bool valid_rows(int R) { return R == 1 || R == 2 || R == 4 || R == 8; }
inline int max_rows(int K) { return seq_lds(K) ? 8 : 4; }

// Kernel timing: while a pair of events is set (per host thread), every
// launch hands them to the dispatch, which stamps them with the kernel's own
// start and end times (no host-side gaps), as a profiler's kernel trace does.
struct LaunchTiming {
    hipEvent_t start = nullptr, stop = nullptr;
};
LaunchTiming& launch_timing();

template <typename F, typename... Args>
inline hipError_t launch(F kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s, Args... args) {
    const LaunchTiming& t = launch_timing();
    if (t.start)
        hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)lds, s, t.start, t.stop, 0u, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
    return hipGetLastError();
}

// One stencil launch: the instances of a group, their block -> instance map.
struct Group {
    int K, R;          // kernel size and rows per thread shared by the group
    int C, nw;         // LDS sizing: most channels and TV-weight planes in the group
    int grid;          // blocks of one pass over the group
    const int* blk;    // device map, grid entries
    int only;          // the instance index if the group has one instance, else -1
    int grid_f;        // blocks of a one-pass FISTA launch over the group (0: two-pass form)
    const int* blk_f;  // its device map
    int cg1;           // the group's CG runs the one-pass form (needs grid_f > 0)
};

// Whether a group can take the one-pass FISTA form: one channel and
// 3 <= K <= 11 (tile rows 1, 2, 4).
inline bool step_ok(int C, int K, int R) { return C == 1 && K >= 3 && K <= 11 && R <= 4; }
// Tiles of the one-pass forms: 64 - (K - 1) columns by kStepNW R rows.
inline int step_blocks(int H, int W, int K, int R) {
    const int tw = kTW - (K - 1), th = kStepNW * R;
    return ((W + tw - 1) / tw) * ((H + th - 1) / th);
}

template <typename T> struct Ops {
    static hipError_t prep_kernel(const Inst<T>* insts, int n, ApgState* Lst, CgState* Cst, int slot_abs,
                                  hipStream_t s);
    // the same, with the upload of `roles` adjacent role tables (n entries
    // each) from mapped host memory src_host to dst folded in; the pass
    // prepares the instances of the first of them
    static hipError_t prep_upload(const void* src_host, void* dst, int roles, int n, ApgState* Lst, CgState* Cst,
                                  int slot_abs, hipStream_t s);
    static hipError_t finish(const Inst<T>* insts, int n, int slot, int sob_slot, hipStream_t s);
    static hipError_t conv(const Group& g, const Inst<T>* insts, hipStream_t s);
    static hipError_t apg_grad(const Group& g, const Inst<T>* insts, const ApgState* sin, ApgState* sout, hipStream_t s);
    static hipError_t apg_trial(const Group& g, const Inst<T>* insts, const ApgState* sin, ApgState* sout, hipStream_t s);
    static hipError_t apg_step(const Group& g, const Inst<T>* insts, const ApgState* sin, ApgState* sout, hipStream_t s);
    static hipError_t cg_step(const Group& g, const Inst<T>* insts, const CgState* sin, CgState* sout, hipStream_t s);
    static hipError_t apg_final(int grid_e, const int* blk_e, int only, const Inst<T>* insts, const ApgState* sin,
                                hipStream_t s);
    static hipError_t cg_dir(const Group& g, const Inst<T>* insts, const CgState* sin, CgState* sout, int init, hipStream_t s);
    static hipError_t cg_hvp(const Group& g, const Inst<T>* insts, const CgState* sin, CgState* sout, int init, hipStream_t s);
    static hipError_t cg_update(int grid_e, const int* blk_e, int only, const Inst<T>* insts, const CgState* sin,
                                CgState* sout, hipStream_t s);
    static hipError_t cg_init(int grid_e, const int* blk_e, int only, const Inst<T>* insts, const CgState* sin,
                              hipStream_t s);
    // Persistent loops of a group on one team per XCD (ctl.P members each);
    // list: device array of the nlist instance indices of the group.
    static hipError_t apg_team(const Group& g, const Inst<T>* insts, const int* list, int nlist, ApgState* st,
                               const TeamCtl& ctl, long max_slots, hipStream_t s);
    static hipError_t cg_team(const Group& g, const Inst<T>* insts, const int* list, int nlist, CgState* st, int n,
                              const TeamCtl& ctl, long max_slots, hipStream_t s);
    static hipError_t team_occupancy(const Group& g, int* blocks_per_cu);
    // batched forms: all instances of tile class kt (16: K <= 16, else 32),
    // `blocks` = the class's total hg_nblk; the finishing launch has n blocks
    static hipError_t hg_corr_batch(int kt, int blocks, const Inst<T>* insts, int n, hipStream_t s);
    static hipError_t hg_final_batch(int kt, const Inst<T>* insts, int n, hipStream_t s);
};

// Copy bytes (a multiple of 4) from device-mapped host memory to the device.
hipError_t launch_upload(const void* src_host, size_t bytes, void* dst, hipStream_t s);
// XCD of each block of a kTeamXcd x kTeamMax grid (out: that many ints).
hipError_t launch_team_map(int* out, hipStream_t s);
hipError_t launch_publish(const void* src, size_t bytes, void* dst_host, unsigned* flag_host, hipStream_t s);
hipError_t launch_theta_step(const double* th, const double* z, double step, double* out, int KK, hipStream_t s);
// x += alpha d (n elements), per-block FP64 partials of d^2 and the new x^2
// into part[2b], part[2b+1] (blocks of them)
template <typename T>
hipError_t launch_axpy_norms(T* x, const T* d, T alpha, int64_t n, double* part, int blocks, hipStream_t s);
// dst = (D) src
template <typename S, typename D>
hipError_t launch_cast(const S* src, D* dst, int64_t n, hipStream_t s);
// x64 += alpha d, x32 = (float) x64, partials of d^2 and x64^2 (2 per block)
hipError_t launch_axpy_mixed(double* x64, const float* d, double alpha, int64_t n, float* x32, double* part, int blocks,
                             hipStream_t s);
// r(theta) over kp kernel planes of KxK taps into *out (one block)
hipError_t launch_sobolev(double beta, double h1_w0, const double* th, const double* a, int K, int kp, double* out,
                          hipStream_t s);
int hg_items(const Shape& d);

extern template struct Ops<float>;
extern template struct Ops<double>;

}  // namespace maid
