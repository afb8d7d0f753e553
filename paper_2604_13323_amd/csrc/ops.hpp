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
  hipError_t (*vjp)(const VjpArgs& a, hipStream_t s);
  hipError_t (*vjp_tail)(const VjpArgs& a, int grid, hipStream_t s);  // FP32 mode only
  hipError_t (*eval_fj)(const DevProblem* P, int64_t n, const void* q, int64_t ld, void* F, void* J, hipStream_t s);
  int (*persistent_blocks_per_cu)(int block);
  size_t (*lds_bytes)(int block);
};

inline unsigned blocks_for(int64_t n, int block) { return unsigned((n + block - 1) / block); }

constexpr int kCheckLanes = 4;       // check_batch: lanes per configuration

template <class Model, class IO, class S>
struct OpsImpl {
  static size_t lds_bytes(int block) { return size_t(Model::D) * sizeof(double) * size_t(block); }
  static hipError_t project_persistent(const ProjArgs& a, int grid, int block, hipStream_t s) {
    hipLaunchKernelGGL((k_project_persistent<Model, IO, S>), dim3(grid), dim3(block), lds_bytes(block), s, a);
    return hipGetLastError();
  }
  // cyclic mode (models with several constraint blocks): a second LDS tile holds the iterate at
  // the start of each iteration
  static hipError_t project_persistent_cyclic(const ProjArgs& a, int grid, int block, hipStream_t s) {
    hipLaunchKernelGGL((k_project_persistent<Model, IO, S, true>), dim3(grid), dim3(block), 2 * lds_bytes(block), s, a);
    return hipGetLastError();
  }
  static hipError_t project_tail_cyclic(const ProjArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((k_project_tail<Model, IO, true>), dim3(grid), dim3(64), 2 * lds_bytes(64), s, a);
    return hipGetLastError();
  }
  static hipError_t project_plain(const ProjArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_project_plain<Model, IO, S>), dim3(blocks_for(a.n, 64)), dim3(64), lds_bytes(64), s, a);
    return hipGetLastError();
  }
  static hipError_t project_tail(const ProjArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((k_project_tail<Model, IO>), dim3(grid), dim3(64), lds_bytes(64), s, a);
    return hipGetLastError();
  }
  static hipError_t check_tail(const ProjArgs& a, int grid, hipStream_t s) {
    const size_t stage = size_t(a.n_sph + a.n_obs) * 16;
    // short queues: a wave (or part of one configuration's links) per work item, one pass of
    // `small` work items over 4 waves per workgroup; the LDS covers the long-queue path's 64
    // lane groups of 4
    const int64_t small = int64_t(grid) * 4;
    const size_t cols = size_t(256 / kTailCheckLanesLong) * Model::D * sizeof(double);
    hipLaunchKernelGGL((k_check_tail<Model, IO>), dim3(grid), dim3(256), cols + stage, s, a, small);
    return hipGetLastError();
  }
  static hipError_t vjp_tail(const VjpArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((k_vjp_tail<Model, IO>), dim3(grid), dim3(64), lds_bytes(64), s, a);
    return hipGetLastError();
  }
  static hipError_t check(const CheckArgs& a, int minsd, hipStream_t s) {
    if (minsd) {
      hipLaunchKernelGGL((k_check<Model, IO, true, 1>), dim3(blocks_for(a.n, 256)), dim3(256), 0, s, a);
    } else {
      constexpr int L = kCheckLanes;
      hipLaunchKernelGGL((k_check<Model, IO, false, L>), dim3(blocks_for(a.n * L, 256)), dim3(256), 0, s, a);
    }
    return hipGetLastError();
  }
  static hipError_t vjp(const VjpArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_vjp<Model, IO, S>), dim3(blocks_for(a.n, 64)), dim3(64), lds_bytes(64), s, a);
    return hipGetLastError();
  }
  static hipError_t eval_fj(const DevProblem* P, int64_t n, const void* q, int64_t ld, void* F, void* J, hipStream_t s) {
    hipLaunchKernelGGL((k_eval_fj<Model, IO, S>), dim3(blocks_for(n, 64)), dim3(64), 0, s, P, n, q, ld, F, J);
    return hipGetLastError();
  }
  static hipError_t project_persistent_wide(const ProjArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((k_project_persistent_wide<Model, IO, S>), dim3(grid), dim3(256), lds_bytes(256), s, a);
    return hipGetLastError();
  }
  static int persistent_wide_blocks_per_cu() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(&k_project_persistent_wide<Model, IO, S>),
                                                     256, lds_bytes(256)) != hipSuccess)
      return 1;
    return nb > 0 ? nb : 1;
  }
  static int persistent_blocks_per_cu(int block) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(&k_project_persistent<Model, IO, S>),
                                                     block, lds_bytes(block)) != hipSuccess)
      return 1;
    return nb > 0 ? nb : 1;
  }
  static FamilyOps make() {
    FamilyOps o;
    o.family = Model::family;
    o.f64 = std::is_same<S, double>::value ? 1 : 0;
    o.dof_max = Model::D;
    o.project_persistent = &project_persistent;
    // with a single constraint block the cyclic mode is the stacked one
    if constexpr (Model::NBLK > 1) {
      o.project_persistent_cyclic = &project_persistent_cyclic;
      o.project_tail_cyclic = std::is_same<S, float>::value ? &project_tail_cyclic : nullptr;
    } else {
      o.project_persistent_cyclic = &project_persistent;
      o.project_tail_cyclic = std::is_same<S, float>::value ? &project_tail : nullptr;
    }
    // the 36-DoF tree in FP32 mode needs more than 256 registers per lane: its one-wave launch
    // leaves half the wave slots empty, which the wide launch fills on large batches
    if constexpr (Model::D > 16 && std::is_same<S, float>::value) {
      o.project_persistent_wide = &project_persistent_wide;
      o.persistent_wide_blocks_per_cu = &persistent_wide_blocks_per_cu;
    } else {
      o.project_persistent_wide = nullptr;
      o.persistent_wide_blocks_per_cu = nullptr;
    }
    o.project_plain = &project_plain;
    o.project_tail = std::is_same<S, float>::value ? &project_tail : nullptr;
    o.check_tail = Model::broad_in_residual ? &check_tail : nullptr;
    o.check = &check;
    o.vjp = &vjp;
    o.vjp_tail = std::is_same<S, float>::value ? &vjp_tail : nullptr;
    o.eval_fj = &eval_fj;
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
#undef MC_FAMILY_TABLE

}  // namespace mc
