// stencil_decl.h -- per-K stencil launchers (defined in launch.cuh and
// explicitly instantiated, a few kernel sizes per translation unit, so the
// build parallelises).
#pragma once
#include "ops.h"

namespace maid {
template <typename T, int K>
hipError_t conv_k(const Group& g, const Inst<T>* insts, hipStream_t s);
template <typename T, int K>
hipError_t apg_grad_k(const Group& g, const Inst<T>* insts, const ApgState* sin, ApgState* sout, hipStream_t s);
template <typename T, int K>
hipError_t apg_trial_k(const Group& g, const Inst<T>* insts, const ApgState* sin, ApgState* sout, hipStream_t s);
template <typename T, int K>
hipError_t cg_dir_k(const Group& g, const Inst<T>* insts, const CgState* sin, CgState* sout, int init, hipStream_t s);
template <typename T, int K>
hipError_t cg_hvp_k(const Group& g, const Inst<T>* insts, const CgState* sin, CgState* sout, int init, hipStream_t s);
template <typename T, int K>
hipError_t apg_team_k(const Group& g, const Inst<T>* insts, const int* list, int nlist, ApgState* st, const TeamCtl& ctl,
                      long max_slots, hipStream_t s);
template <typename T, int K>
hipError_t cg_team_k(const Group& g, const Inst<T>* insts, const int* list, int nlist, CgState* st, int n,
                     const TeamCtl& ctl, long max_slots, hipStream_t s);
template <typename T, int K>
hipError_t team_occupancy_k(const Group& g, int* blocks_per_cu);
template <typename T, int K>
hipError_t apg_step_k(const Group& g, const Inst<T>* insts, const ApgState* sin, ApgState* sout, hipStream_t s);
template <typename T, int K>
hipError_t cg_step_k(const Group& g, const Inst<T>* insts, const CgState* sin, CgState* sout, hipStream_t s);
}  // namespace maid
