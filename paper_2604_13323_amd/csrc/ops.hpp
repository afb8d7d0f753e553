// Per-family, per-precision kernel launchers. Each translation unit instantiates the
// generic kernels for one model in one precision mode and exports one FamilyOps table;
// the C-ABI layer dispatches on (family, dtype).
#pragma once

#include "kernels.hpp"

namespace mc {

struct FamilyOps {
  int family;
  int f64;      // 1: FP64 mode tables (IO = double, S = double)
  int dof_max;  // compiled D (padded for the linear family)
  hipError_t (*project_persistent)(const ProjArgs& a, int grid, int block, hipStream_t s);
  hipError_t (*project_persistent_cyclic)(const ProjArgs& a, int grid, int block, hipStream_t s);
  // two waves per SIMD (256-thread blocks), for batches beyond the lanes of the one-wave launch;
  // null where one wave per SIMD is not the register limit
  hipError_t (*project_persistent_wide)(const ProjArgs& a, int grid, hipStream_t s);
  int (*persistent_wide_blocks_per_cu)();
  hipError_t (*project_tail_cyclic)(const ProjArgs& a, int grid, hipStream_t s);  // FP32 mode only
  hipError_t (*project_plain)(const ProjArgs& a, hipStream_t s);
  hipError_t (*project_tail)(const ProjArgs& a, int grid, hipStream_t s);  // FP32 mode only
  hipError_t (*check_tail)(const ProjArgs& a, int grid, hipStream_t s);
  hipError_t (*check)(const CheckArgs& a, int minsd, hipStream_t s);
  // check_batch's broad phase (verdicts only), whose queue check_tail finishes; null where the
  // model has no broad phase
  hipError_t (*check_broad)(const CheckArgs& a, unsigned* count, int32_t* idx, double* qbuf, int64_t cap,
                            hipStream_t s);
  hipError_t (*vjp)(const VjpArgs& a, hipStream_t s);
  hipError_t (*vjp_tail)(const VjpArgs& a, int grid, hipStream_t s);  // FP32 mode only
  hipError_t (*vjp_exact)(const VjpxArgs& a, hipStream_t s);
  hipError_t (*eval_fj)(const DevProblem* P, int64_t n, const void* q, int64_t ld, void* F, void* J, hipStream_t s);
  hipError_t (*eval_cond)(const DevProblem* P, int64_t n, const void* q, int64_t ld, double lambda, void* kappa,
                          hipStream_t s);
  int (*persistent_blocks_per_cu)(int block);
  size_t (*lds_bytes)(int block);
};

inline unsigned blocks_for(int64_t n, int block) { return unsigned((n + block - 1) / block); }

constexpr int kCheckLanes = 4;       // check_batch: lanes per configuration

// The launchers of one (model, precision) pair. Declared here; defined in ops_impl.hpp, which the
// translation units that instantiate them include (the heavy families split their launchers over
// several translation units, so their kernels compile in parallel).
template <class Model, class IO, class S>
struct OpsImpl {
  static size_t lds_bytes(int block) { return size_t(Model::D) * sizeof(double) * size_t(block); }
  static hipError_t project_persistent(const ProjArgs& a, int grid, int block, hipStream_t s);
  static int persistent_blocks_per_cu(int block);
  // cyclic mode (models with several constraint blocks): a second LDS tile holds the iterate at
  // the start of each iteration
  static hipError_t project_persistent_cyclic(const ProjArgs& a, int grid, int block, hipStream_t s);
  static hipError_t project_tail_cyclic(const ProjArgs& a, int grid, hipStream_t s);
  static hipError_t project_plain(const ProjArgs& a, hipStream_t s);
  static hipError_t project_tail(const ProjArgs& a, int grid, hipStream_t s);
  static hipError_t check_tail(const ProjArgs& a, int grid, hipStream_t s);
  static hipError_t vjp_tail(const VjpArgs& a, int grid, hipStream_t s);
  static hipError_t check(const CheckArgs& a, int minsd, hipStream_t s);
  static hipError_t check_broad(const CheckArgs& a, unsigned* count, int32_t* idx, double* qbuf, int64_t cap,
                                hipStream_t s);
  static hipError_t vjp(const VjpArgs& a, hipStream_t s);
  static hipError_t vjp_exact(const VjpxArgs& a, hipStream_t s);
  static hipError_t eval_fj(const DevProblem* P, int64_t n, const void* q, int64_t ld, void* F, void* J, hipStream_t s);
  static hipError_t eval_cond(const DevProblem* P, int64_t n, const void* q, int64_t ld, double lambda, void* kappa,
                              hipStream_t s);
  static hipError_t project_persistent_wide(const ProjArgs& a, int grid, hipStream_t s);
  static int persistent_wide_blocks_per_cu();
  static constexpr bool kF32 = std::is_same<S, float>::value;
  // the 36-DoF tree in FP32 mode needs more than 256 registers per lane: its one-wave launch
  // leaves half the wave slots empty, which the two-wave launch fills on large batches
  static constexpr bool kWide = Model::D > 16 && kF32;
  static FamilyOps make() {
    FamilyOps o;
    o.family = Model::family;
    o.f64 = kF32 ? 0 : 1;
    o.dof_max = Model::D;
    o.project_persistent = &project_persistent;
    // with a single constraint block the cyclic mode is the stacked one (only the launchers a table
    // names are instantiated, so the choices are compile-time)
    o.project_tail_cyclic = nullptr;
    if constexpr (Model::NBLK > 1) {
      o.project_persistent_cyclic = &project_persistent_cyclic;
      if constexpr (kF32) o.project_tail_cyclic = &project_tail_cyclic;
    } else {
      o.project_persistent_cyclic = &project_persistent;
      if constexpr (kF32) o.project_tail_cyclic = &project_tail;
    }
    if constexpr (kWide) {
      o.project_persistent_wide = &project_persistent_wide;
      o.persistent_wide_blocks_per_cu = &persistent_wide_blocks_per_cu;
    } else {
      o.project_persistent_wide = nullptr;
      o.persistent_wide_blocks_per_cu = nullptr;
    }
    o.project_plain = &project_plain;
    o.project_tail = nullptr;
    o.vjp_tail = nullptr;
    if constexpr (kF32) {
      o.project_tail = &project_tail;
      o.vjp_tail = &vjp_tail;
    }
    o.check_tail = nullptr;
    o.check_broad = nullptr;
    if constexpr (Model::broad_in_residual) {
      o.check_tail = &check_tail;
      o.check_broad = &check_broad;
    }
    o.check = &check;
    o.vjp = &vjp;
    o.vjp_exact = &vjp_exact;
    o.eval_fj = &eval_fj;
    o.eval_cond = &eval_cond;
    o.persistent_blocks_per_cu = &persistent_blocks_per_cu;
    o.lds_bytes = &lds_bytes;
    return o;
  }
};

#define MC_FAMILY_TABLE(name) \
  extern const FamilyOps ops_##name##_f32; \
  extern const FamilyOps ops_##name##_f64;
MC_FAMILY_TABLE(sphere3)
MC_FAMILY_TABLE(linear)
MC_FAMILY_TABLE(planar2)
MC_FAMILY_TABLE(arm7_axis)
MC_FAMILY_TABLE(dual14_rel)
MC_FAMILY_TABLE(humanoid36)
MC_FAMILY_TABLE(digit36)
MC_FAMILY_TABLE(arm7_tsr)
#undef MC_FAMILY_TABLE

}  // namespace mc
