// team.cuh -- persistent solver loops for small instances.
//
// A solve of a small image is bound by the latency of its passes, not by
// bandwidth or arithmetic: each pass is a kernel of a few microseconds, and
// the boundary between two kernels (drain, cache write-back, next dispatch)
// costs as much again.  Here the blocks that run on one XCD form a team that
// carries a whole solve (FISTA or CG iterations until the stop test) inside
// one kernel, with a team barrier where the multi-kernel path has a kernel
// boundary.  Every pass body is the one the multi-kernel path runs (same
// tiles, same partial sums in the same order, same decisions), so the two
// paths give bitwise-identical results.
//
// Coherence within a team: the blocks of an XCD share its L2, and vector
// stores write through the CU's L1 into it.  A member therefore publishes
// its pass by waiting for its stores to complete and then raising its
// arrival word; readers load everything the pass wrote with device-scope
// atomic loads (ld<true>), which bypass their own L1.  No L2 write-back or
// invalidation is needed because no data leaves the XCD during the loop.
//
// Team formation: the hardware hands block b to XCD b mod 8 (checked once
// per context by k_team_map before the team path is enabled), and each
// block reads the XCD it runs on from the XCC_ID hardware register: the
// blocks with the same XCC_ID form a team, member index blockIdx / 8.  The
// launch has 8 P blocks (P members per team) and every team's members must
// be resident together, which the host guarantees by capping P at the
// kernel's occupancy on the XCD's 32 CUs.  Every wait is bounded in time: a
// member that waits too long raises the error word and leaves, and the
// others then leave too, so the kernel always ends; the host then repeats
// the solve on the multi-kernel path.
//
// Team t serves the instances list[t], list[t + 8], ... of the launch, one
// after the other.
#pragma once
#include "kernels.cuh"
#include "step.cuh"

namespace maid {

// The XCD this wave runs on (hardware register XCC_ID, bits 0..3).
__device__ __forceinline__ int xcc_id() { return (int)(__builtin_amdgcn_s_getreg(20 | (0 << 6) | (3 << 11)) & 7u); }

struct Team {
    uint64_t* arrive;
    unsigned* err;
    uint64_t gen;
    int64_t wait;
    int P, me, x;

    __device__ __forceinline__ Team(const TeamCtl& c)
        : arrive(c.arrive + xcc_id() * kTeamMax), err(c.err), gen(c.epoch), wait(c.wait), P(c.P),
          me((int)(blockIdx.x >> 3)), x(xcc_id()) {}

    // Team barrier: returns false (every thread of the block) if the wait
    // timed out or another member reported a failure.
    __device__ __forceinline__ bool sync() {
        __shared__ int s_ok;
        gen += 1;
        // this wave's stores have reached L2 before the block arrives
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0) __hip_atomic_store(arrive + me, gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (threadIdx.x < 64) {
            const int64_t t0 = (int64_t)wall_clock64();
            bool ok = true;
            for (;;) {
                bool in = true;
                for (int i = threadIdx.x; i < P; i += 64)
                    in = in && __hip_atomic_load(arrive + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= gen;
                if (__all(in)) break;
                const bool bad = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
                if (__any(bad) || (int64_t)wall_clock64() - t0 > wait) {
                    ok = false;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            if (threadIdx.x == 0) {
                if (!ok) __hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s_ok = ok ? 1 : 0;
            }
        }
        __syncthreads();
        return s_ok != 0;
    }
};

// FISTA loop (Algorithm 1, lower level) for the instances of a group: per
// slot one gradient pass and one trial pass, as the multi-kernel path runs
// them (STEP: one pass of the one-pass form), until every solve has stopped
// or max_slots slots have run (the final point is formed by the elementwise
// pass that follows, as on the multi-kernel path).  st: the state array
// (read at the start, written at the end).
template <typename T, int K, int R, bool STEP>
__global__ __launch_bounds__(STEP ? kStepNT : kNT) __attribute__((amdgpu_waves_per_eu(min_waves<T>(K, R)))) void k_apg_team(
    const Inst<T>* __restrict__ insts, const int* __restrict__ list, int nlist, ApgState* __restrict__ st_arr,
    TeamCtl ctl, long max_slots) {
    Team tm(ctl);
    for (int j = tm.x; j < nlist; j += kTeamXcd) {
        const int ii = list[j];
        const Inst<T>& I = insts[ii];
        ApgState st = st_arr[ii];
        if constexpr (STEP) {
            // one-pass form (blocks of kStepNT threads): one pass (and one
            // barrier) per iteration
            for (long slot = 0; !st.done; ++slot) {
                ApgState nx = st;
                for (int lb = tm.me; lb < I.nbf; lb += tm.P) {
                    nx = st;
                    __syncthreads();
                    apg_step_body<T, K, R, true>(I, lb, nx, nullptr, lb == 0 && threadIdx.x == 0);
                }
                st = nx;
                if (st.done) break;
                if (!tm.sync()) return;
                if (slot + 1 >= max_slots) break;
            }
        } else if (!st.done) {
            for (long slot = 0;; ++slot) {
                ApgState nx = st;
                for (int lb = tm.me; lb < I.nb; lb += tm.P) {
                    nx = st;
                    __syncthreads();
                    apg_grad_body<T, K, R, true>(I, lb, nx, nullptr, lb == 0 && threadIdx.x == 0);
                }
                st = nx;
                if (st.done) break;
                if (!tm.sync()) return;
                for (int lb = tm.me; lb < I.nb; lb += tm.P) {
                    nx = st;
                    __syncthreads();
                    apg_trial_body<T, K, R, true>(I, lb, nx, nullptr, lb == 0 && threadIdx.x == 0);
                }
                st = nx;
                if (st.done) break;
                if (!tm.sync()) return;
                if (slot + 1 >= max_slots) break;
            }
        }
        if (tm.me == 0 && threadIdx.x == 0) put_state(&st_arr[ii], st);
    }
}

// CG loop (the adjoint solve of Algorithm 1) after its set-up passes: per
// slot a direction, a Hessian and an update pass, as the multi-kernel path
// runs them (STEP: one pass of the one-pass form).  st: the first of the three state arrays (n entries each; read
// at the start from the first).  The final state goes into all three: an
// elementwise update pass of the multi-kernel path that covers the whole
// batch then finds the instance finished and leaves it as it is.
template <typename T, int K, int R, bool STEP>
__global__ __launch_bounds__(STEP ? kStepNT : kNT) __attribute__((amdgpu_waves_per_eu(min_waves<T>(K, R)))) void k_cg_team(
    const Inst<T>* __restrict__ insts, const int* __restrict__ list, int nlist, CgState* __restrict__ st_arr,
    int n, TeamCtl ctl, long max_slots) {
    Team tm(ctl);
    for (int j = tm.x; j < nlist; j += kTeamXcd) {
        const int ii = list[j];
        const Inst<T>& I = insts[ii];
        CgState st = st_arr[ii];
        if constexpr (STEP) {
            // one-pass form (its priming pass first; blocks of kStepNT
            // threads): one pass per iteration
            for (long slot = 0; !st.done; ++slot) {
                CgState nx = st;
                for (int lb = tm.me; lb < I.nbf; lb += tm.P) {
                    nx = st;
                    __syncthreads();
                    cg_step_body<T, K, R, true>(I, lb, nx, nullptr, false);
                }
                st = nx;
                if (st.done) break;
                if (!tm.sync()) return;
                if (slot + 1 >= max_slots) break;
            }
        } else if (!st.done) {
            for (long slot = 0;; ++slot) {
                CgState nx = st;
                for (int lb = tm.me; lb < I.nb; lb += tm.P) {
                    nx = st;
                    __syncthreads();
                    cg_dir_body<T, K, R, true>(I, lb, nx, nullptr, false, 0);
                }
                st = nx;
                if (st.done) break;
                if (!tm.sync()) return;
                for (int lb = tm.me; lb < I.nb; lb += tm.P) {
                    __syncthreads();
                    cg_hvp_body<T, K, R, true>(I, lb, st, 0);
                }
                if (!tm.sync()) return;
                for (int lb = tm.me; lb < I.nbe; lb += tm.P) {
                    nx = st;
                    cg_update_body<T, true>(I, lb, nx, nullptr, false);
                }
                st = nx;
                if (st.done) break;
                if (!tm.sync()) return;
                if (slot + 1 >= max_slots) break;
            }
        }
        if (tm.me == 0 && threadIdx.x == 0) {
            put_state(&st_arr[ii], st);
            put_state(&st_arr[ii + n], st);
            put_state(&st_arr[ii + 2 * n], st);
        }
    }
}

}  // namespace maid
