// launch.cuh -- the per-K stencil launchers: R dispatch to the kernel
// templates of kernels.cuh, with the dynamic LDS sized for the group's
// largest instance.  Included by the per-K instantiation units.
#pragma once
#include "kernels.cuh"
#include "team.cuh"
#include "step.cuh"
#include "stencil_decl.h"

namespace maid {

// Raise the dynamic-LDS limit of a kernel if it needs more than 64 KiB
// together with its static LDS (the matrix-core correlation's tiles).
template <typename Kern>
static inline hipError_t ensure_lds(Kern kern, size_t bytes, size_t static_bytes = 0) {
    if (bytes + static_bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}
// static LDS of the correlation selector in the instantiations that have
// the matrix-core path (its block maximum; the tiles live in the dynamic
// region)
template <typename T, int K, int R> constexpr size_t mf_static() {
    if constexpr (mf_ok<T, K, R>()) return 64;
    else return 0;
}

template <typename T, int K, int R>
static hipError_t conv_kr(const Group& g, const Inst<T>* insts, hipStream_t s) {
    const size_t lds = sizeof(T) * lds_conv(K, R, sizeof(T));
    auto kern = k_conv<T, K, R>;
    hipError_t e = ensure_lds(kern, lds, mf_static<T, K, R>());
    if (e != hipSuccess) return e;
    return launch(kern, dim3(g.grid), dim3(kNT), lds, s, insts, g.blk, g.only);
}

template <typename T, int K, int R>
static hipError_t apg_grad_kr(const Group& g, const Inst<T>* insts, const ApgState* sin, ApgState* sout, hipStream_t s) {
    const size_t lds = sizeof(T) * lds_apg_grad(K, R, g.C, g.nw, sizeof(T));
    auto kern = k_apg_grad<T, K, R>;
    hipError_t e = ensure_lds(kern, lds, mf_static<T, K, R>());
    if (e != hipSuccess) return e;
    return launch(kern, dim3(g.grid), dim3(kNT), lds, s, insts, g.blk, g.only, sin, sout);
}

template <typename T, int K, int R>
static hipError_t apg_trial_kr(const Group& g, const Inst<T>* insts, const ApgState* sin, ApgState* sout, hipStream_t s) {
    const size_t lds = sizeof(T) * lds_apg_trial(K, R, g.C, sizeof(T));
    auto kern = k_apg_trial<T, K, R>;
    hipError_t e = ensure_lds(kern, lds, mf_static<T, K, R>());
    if (e != hipSuccess) return e;
    return launch(kern, dim3(g.grid), dim3(kNT), lds, s, insts, g.blk, g.only, sin, sout);
}

template <typename T, int K, int R>
static hipError_t cg_dir_kr(const Group& g, const Inst<T>* insts, const CgState* sin, CgState* sout, int init,
                            hipStream_t s) {
    const size_t lds = sizeof(T) * lds_cg_dir(K, R, sizeof(T));
    auto kern = k_cg_dir<T, K, R>;
    hipError_t e = ensure_lds(kern, lds, mf_static<T, K, R>());
    if (e != hipSuccess) return e;
    return launch(kern, dim3(g.grid), dim3(kNT), lds, s, insts, g.blk, g.only, sin, sout, init);
}

template <typename T, int K, int R>
static hipError_t cg_hvp_kr(const Group& g, const Inst<T>* insts, const CgState* sin, CgState* sout, int init,
                            hipStream_t s) {
    const size_t lds = sizeof(T) * lds_cg_hvp(K, R, g.C, g.nw, sizeof(T));
    auto kern = k_cg_hvp<T, K, R>;
    hipError_t e = ensure_lds(kern, lds, mf_static<T, K, R>());
    if (e != hipSuccess) return e;
    return launch(kern, dim3(g.grid), dim3(kNT), lds, s, insts, g.blk, g.only, sin, sout, init);
}

// Team launches (persistent loops for small instances): 8 P blocks; their
// LDS is the larger of the two passes each loop alternates.
template <typename T, int K, int R, bool STEP>
static size_t apg_team_lds(const Group& g) {
    if constexpr (STEP) return sizeof(T) * lds_apg_step<K, R>();
    else return sizeof(T) * cmax(lds_apg_grad(K, R, g.C, g.nw, sizeof(T)), lds_apg_trial(K, R, g.C, sizeof(T)));
}
// one-pass team loops exist where the one-pass form does
template <int K, int R> constexpr bool step_team() { return K >= 3 && K <= 11 && R <= 4; }
template <typename T, int K, int R, bool STEP>
static size_t cg_team_lds(const Group& g) {
    if constexpr (STEP) return sizeof(T) * lds_cg_step<K, R>();
    else return sizeof(T) * cmax(lds_cg_dir(K, R, sizeof(T)), lds_cg_hvp(K, R, g.C, g.nw, sizeof(T)));
}

template <typename T, int K, int R, bool STEP>
static hipError_t apg_team_krs(const Group& g, const Inst<T>* insts, const int* list, int nlist, ApgState* st,
                               const TeamCtl& ctl, long max_slots, hipStream_t s) {
    const size_t lds = apg_team_lds<T, K, R, STEP>(g);
    auto kern = k_apg_team<T, K, R, STEP>;
    hipError_t e = ensure_lds(kern, lds, mf_static<T, K, R>());
    if (e != hipSuccess) return e;
    return launch(kern, dim3(kTeamXcd * ctl.P), dim3(STEP ? kStepNT : kNT), lds, s, insts, list, nlist, st, ctl,
                  max_slots);
}
template <typename T, int K, int R>
static hipError_t apg_team_kr(const Group& g, const Inst<T>* insts, const int* list, int nlist, ApgState* st,
                              const TeamCtl& ctl, long max_slots, hipStream_t s) {
    if constexpr (step_team<K, R>())
        if (g.grid_f > 0) return apg_team_krs<T, K, R, true>(g, insts, list, nlist, st, ctl, max_slots, s);
    return apg_team_krs<T, K, R, false>(g, insts, list, nlist, st, ctl, max_slots, s);
}

template <typename T, int K, int R, bool STEP>
static hipError_t cg_team_krs(const Group& g, const Inst<T>* insts, const int* list, int nlist, CgState* st, int n,
                              const TeamCtl& ctl, long max_slots, hipStream_t s) {
    const size_t lds = cg_team_lds<T, K, R, STEP>(g);
    auto kern = k_cg_team<T, K, R, STEP>;
    hipError_t e = ensure_lds(kern, lds, mf_static<T, K, R>());
    if (e != hipSuccess) return e;
    return launch(kern, dim3(kTeamXcd * ctl.P), dim3(STEP ? kStepNT : kNT), lds, s, insts, list, nlist, st, n, ctl,
                  max_slots);
}
template <typename T, int K, int R>
static hipError_t cg_team_kr(const Group& g, const Inst<T>* insts, const int* list, int nlist, CgState* st, int n,
                             const TeamCtl& ctl, long max_slots, hipStream_t s) {
    if constexpr (step_team<K, R>())
        if (g.cg1) return cg_team_krs<T, K, R, true>(g, insts, list, nlist, st, n, ctl, max_slots, s);
    return cg_team_krs<T, K, R, false>(g, insts, list, nlist, st, n, ctl, max_slots, s);
}

// Blocks of the group's two team kernels that fit on one CU at once (the
// smaller of the two).
template <typename T, int K, int R, bool STEP, bool STEP_CG>
static hipError_t team_occupancy_krs(const Group& g, int* blocks_per_cu) {
    int a = 0, b = 0;
    hipError_t e = ensure_lds(k_apg_team<T, K, R, STEP>, apg_team_lds<T, K, R, STEP>(g), mf_static<T, K, R>());
    if (e == hipSuccess)
        e = ensure_lds(k_cg_team<T, K, R, STEP_CG>, cg_team_lds<T, K, R, STEP_CG>(g), mf_static<T, K, R>());
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_apg_team<T, K, R, STEP>, STEP ? kStepNT : kNT,
                                                         apg_team_lds<T, K, R, STEP>(g));
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_cg_team<T, K, R, STEP_CG>, STEP_CG ? kStepNT : kNT,
                                                         cg_team_lds<T, K, R, STEP_CG>(g));
    *blocks_per_cu = e == hipSuccess ? (a < b ? a : b) : 0;
    return e;
}
template <typename T, int K, int R>
static hipError_t team_occupancy_kr(const Group& g, int* blocks_per_cu) {
    if constexpr (step_team<K, R>()) {
        if (g.grid_f > 0 && g.cg1) return team_occupancy_krs<T, K, R, true, true>(g, blocks_per_cu);
        if (g.grid_f > 0) return team_occupancy_krs<T, K, R, true, false>(g, blocks_per_cu);
    }
    return team_occupancy_krs<T, K, R, false, false>(g, blocks_per_cu);
}

// One-pass FISTA (single channel, 3 <= K <= 11; tile rows 1, 2, 4).
template <typename T, int K, int R>
static hipError_t apg_step_kr(const Group& g, const Inst<T>* insts, const ApgState* sin, ApgState* sout,
                              hipStream_t s) {
    if constexpr (K >= 3 && K <= 11) {
        const size_t lds = sizeof(T) * lds_apg_step<K, R>();
        auto kern = k_apg_step<T, K, R>;
        hipError_t e = ensure_lds(kern, lds, mf_static<T, K, R>());
        if (e != hipSuccess) return e;
        return launch(kern, dim3(g.grid_f), dim3(kStepNT), lds, s, insts, g.blk_f, g.only, sin, sout);
    } else {
        return hipErrorInvalidValue;
    }
}

template <typename T, int K, int R>
static hipError_t cg_step_kr(const Group& g, const Inst<T>* insts, const CgState* sin, CgState* sout, hipStream_t s) {
    if constexpr (K >= 3 && K <= 11) {
        const size_t lds = sizeof(T) * lds_cg_step<K, R>();
        auto kern = k_cg_step<T, K, R>;
        hipError_t e = ensure_lds(kern, lds, mf_static<T, K, R>());
        if (e != hipSuccess) return e;
        return launch(kern, dim3(g.grid_f), dim3(kStepNT), lds, s, insts, g.blk_f, g.only, sin, sout);
    } else {
        return hipErrorInvalidValue;
    }
}

// Team loops exist for tile rows 1, 2 and 4.
#define MAID_TEAM_R_DISPATCH(FN, ...)                              \
    switch (g.R) {                                                 \
        case 1: return FN<T, K, 1>(__VA_ARGS__);                   \
        case 2: return FN<T, K, 2>(__VA_ARGS__);                   \
        case 4: return FN<T, K, 4>(__VA_ARGS__);                   \
        default: return hipErrorInvalidValue;                      \
    }

#define MAID_R_DISPATCH(FN, ...)                                   \
    switch (g.R) {                                                 \
        case 1: return FN<T, K, 1>(__VA_ARGS__);                   \
        case 2: return FN<T, K, 2>(__VA_ARGS__);                   \
        case 4: return FN<T, K, 4>(__VA_ARGS__);                   \
        case 8:                                                    \
            if constexpr (seq_lds(K)) return FN<T, K, 8>(__VA_ARGS__); \
            else return hipErrorInvalidValue;                      \
        default: return hipErrorInvalidValue;                      \
    }

template <typename T, int K>
hipError_t conv_k(const Group& g, const Inst<T>* insts, hipStream_t s) {
    MAID_R_DISPATCH(conv_kr, g, insts, s)
}
template <typename T, int K>
hipError_t apg_grad_k(const Group& g, const Inst<T>* insts, const ApgState* sin, ApgState* sout, hipStream_t s) {
    MAID_R_DISPATCH(apg_grad_kr, g, insts, sin, sout, s)
}
template <typename T, int K>
hipError_t apg_trial_k(const Group& g, const Inst<T>* insts, const ApgState* sin, ApgState* sout, hipStream_t s) {
    MAID_R_DISPATCH(apg_trial_kr, g, insts, sin, sout, s)
}
template <typename T, int K>
hipError_t cg_dir_k(const Group& g, const Inst<T>* insts, const CgState* sin, CgState* sout, int init, hipStream_t s) {
    MAID_R_DISPATCH(cg_dir_kr, g, insts, sin, sout, init, s)
}
template <typename T, int K>
hipError_t cg_hvp_k(const Group& g, const Inst<T>* insts, const CgState* sin, CgState* sout, int init, hipStream_t s) {
    MAID_R_DISPATCH(cg_hvp_kr, g, insts, sin, sout, init, s)
}

template <typename T, int K>
hipError_t apg_team_k(const Group& g, const Inst<T>* insts, const int* list, int nlist, ApgState* st, const TeamCtl& ctl,
                      long max_slots, hipStream_t s) {
    MAID_TEAM_R_DISPATCH(apg_team_kr, g, insts, list, nlist, st, ctl, max_slots, s)
}
template <typename T, int K>
hipError_t cg_team_k(const Group& g, const Inst<T>* insts, const int* list, int nlist, CgState* st, int n,
                     const TeamCtl& ctl, long max_slots, hipStream_t s) {
    MAID_TEAM_R_DISPATCH(cg_team_kr, g, insts, list, nlist, st, n, ctl, max_slots, s)
}
template <typename T, int K>
hipError_t apg_step_k(const Group& g, const Inst<T>* insts, const ApgState* sin, ApgState* sout, hipStream_t s) {
    MAID_TEAM_R_DISPATCH(apg_step_kr, g, insts, sin, sout, s)
}
template <typename T, int K>
hipError_t cg_step_k(const Group& g, const Inst<T>* insts, const CgState* sin, CgState* sout, hipStream_t s) {
    MAID_TEAM_R_DISPATCH(cg_step_kr, g, insts, sin, sout, s)
}
template <typename T, int K>
hipError_t team_occupancy_k(const Group& g, int* blocks_per_cu) {
    MAID_TEAM_R_DISPATCH(team_occupancy_kr, g, blocks_per_cu)
}

#define MAID_INSTANTIATE_T(T, KV)                                                                                       \
    template hipError_t conv_k<T, KV>(const Group&, const Inst<T>*, hipStream_t);                                       \
    template hipError_t apg_grad_k<T, KV>(const Group&, const Inst<T>*, const ApgState*, ApgState*, hipStream_t);       \
    template hipError_t apg_trial_k<T, KV>(const Group&, const Inst<T>*, const ApgState*, ApgState*, hipStream_t);      \
    template hipError_t cg_dir_k<T, KV>(const Group&, const Inst<T>*, const CgState*, CgState*, int, hipStream_t);      \
    template hipError_t cg_hvp_k<T, KV>(const Group&, const Inst<T>*, const CgState*, CgState*, int, hipStream_t);      \
    template hipError_t apg_team_k<T, KV>(const Group&, const Inst<T>*, const int*, int, ApgState*, const TeamCtl&,      \
                                          long, hipStream_t);                                                           \
    template hipError_t cg_team_k<T, KV>(const Group&, const Inst<T>*, const int*, int, CgState*, int, const TeamCtl&,  \
                                         long, hipStream_t);                                                            \
    template hipError_t team_occupancy_k<T, KV>(const Group&, int*);                                               \
    template hipError_t apg_step_k<T, KV>(const Group&, const Inst<T>*, const ApgState*, ApgState*, hipStream_t);     \
    template hipError_t cg_step_k<T, KV>(const Group&, const Inst<T>*, const CgState*, CgState*, hipStream_t);

// Instantiate every stencil launcher of both storage types for one K.
#define MAID_INSTANTIATE_K(KV) MAID_INSTANTIATE_T(float, KV) MAID_INSTANTIATE_T(double, KV)

}  // namespace maid
