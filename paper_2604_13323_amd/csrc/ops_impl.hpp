// Definitions of the OpsImpl launchers (see ops.hpp). A translation unit that includes this file
// instantiates the launchers it needs, explicitly (MC_INSTANTIATE_* below), together with their
// kernels.
#pragma once

#include "ops.hpp"

namespace mc {

template <class Model, class IO, class S>
hipError_t OpsImpl<Model, IO, S>::project_persistent(const ProjArgs& a, int grid, int block, hipStream_t s) {
  hipLaunchKernelGGL((k_project_persistent<Model, IO, S>), dim3(grid), dim3(block), lds_bytes(block), s, a);
  return hipGetLastError();
}
template <class Model, class IO, class S>
int OpsImpl<Model, IO, S>::persistent_blocks_per_cu(int block) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(&k_project_persistent<Model, IO, S>),
                                                   block, lds_bytes(block)) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}
template <class Model, class IO, class S>
hipError_t OpsImpl<Model, IO, S>::project_persistent_cyclic(const ProjArgs& a, int grid, int block, hipStream_t s) {
  hipLaunchKernelGGL((k_project_persistent<Model, IO, S, true>), dim3(grid), dim3(block), 2 * lds_bytes(block), s, a);
  return hipGetLastError();
}
template <class Model, class IO, class S>
hipError_t OpsImpl<Model, IO, S>::project_tail_cyclic(const ProjArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_project_tail<Model, IO, true>), dim3(grid), dim3(64), 2 * lds_bytes(64), s, a);
  return hipGetLastError();
}
template <class Model, class IO, class S>
hipError_t OpsImpl<Model, IO, S>::project_plain(const ProjArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((k_project_plain<Model, IO, S>), dim3(blocks_for(a.n, 64)), dim3(64), lds_bytes(64), s, a);
  return hipGetLastError();
}
template <class Model, class IO, class S>
hipError_t OpsImpl<Model, IO, S>::project_tail(const ProjArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_project_tail<Model, IO>), dim3(grid), dim3(64), lds_bytes(64), s, a);
  return hipGetLastError();
}
template <class Model, class IO, class S>
hipError_t OpsImpl<Model, IO, S>::check_tail(const ProjArgs& a, int grid, hipStream_t s) {
  const size_t stage = size_t(a.n_sph + a.n_obs) * 16;
  // short queues: a wave (or part of one configuration's links) per work item, one pass of
  // `small` work items over 4 waves per workgroup
  const int64_t small = int64_t(grid) * 4;
  // the smallest lane group whose staged configurations fit beside the spheres in a quarter of the
  // CU's LDS; the LDS covers 256 / min_lanes groups (or the wave path's slots, if more)
  int min_lanes = 4;
  if constexpr (Model::D <= kTailCheckLowLanesMaxD) {
    for (int L = 1; L < 4; L *= 2)
      if (size_t(256 / L) * Model::D * sizeof(double) + stage <= kTailCheckLdsBudget) {
        min_lanes = L;
        break;
      }
  }
  // the wave-per-configuration path: 4 configurations and 4 x 64 candidate slots (float4)
  const size_t cols64 = size_t(4) * Model::D * sizeof(double) + size_t(4) * 64 * 16;
  const size_t cols_l = size_t(256 / min_lanes) * Model::D * sizeof(double);
  const size_t cols = cols_l > cols64 ? cols_l : cols64;
  hipLaunchKernelGGL((k_check_tail<Model, IO>), dim3(grid), dim3(256), cols + stage, s, a, small, min_lanes);
  return hipGetLastError();
}
template <class Model, class IO, class S>
hipError_t OpsImpl<Model, IO, S>::vjp_tail(const VjpArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_vjp_tail<Model, IO>), dim3(grid), dim3(64), 2 * lds_bytes(64), s, a);
  return hipGetLastError();
}
template <class Model, class IO, class S>
hipError_t OpsImpl<Model, IO, S>::check(const CheckArgs& a, int minsd, hipStream_t s) {
  if (minsd) {
    hipLaunchKernelGGL((k_check<Model, IO, true, 1>), dim3(blocks_for(a.n, 256)), dim3(256), 0, s, a);
  } else {
    constexpr int L = kCheckLanes;
    hipLaunchKernelGGL((k_check<Model, IO, false, L>), dim3(blocks_for(a.n * L, 256)), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}
template <class Model, class IO, class S>
hipError_t OpsImpl<Model, IO, S>::check_broad(const CheckArgs& a, unsigned* count, int32_t* idx, double* qbuf,
                                              int64_t cap, hipStream_t s) {
  if constexpr (Model::broad_in_residual) {
    hipLaunchKernelGGL((k_check_broad<Model, IO>), dim3(blocks_for(a.n, 256)), dim3(256), 0, s, a, count, idx, qbuf, cap);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;  // not in the launch table of such a model
  }
}
template <class Model, class IO, class S>
hipError_t OpsImpl<Model, IO, S>::vjp(const VjpArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((k_vjp<Model, IO, S>), dim3(blocks_for(a.n, 64)), dim3(64),
                     lds_bytes(64) + size_t(Model::D) * sizeof(S) * 64, s, a);
  return hipGetLastError();
}
template <class Model, class IO, class S>
hipError_t OpsImpl<Model, IO, S>::vjp_exact(const VjpxArgs& a, hipStream_t s) {
  // LDS per wave: the FP64 iterate and cotangent tiles and the FP32 direction tile
  hipLaunchKernelGGL((k_vjp_exact<Model, IO>), dim3(blocks_for(a.n, 64)), dim3(64), size_t(Model::D) * 64 * 20, s, a);
  return hipGetLastError();
}
template <class Model, class IO, class S>
hipError_t OpsImpl<Model, IO, S>::eval_fj(const DevProblem* P, int64_t n, const void* q, int64_t ld, void* F, void* J,
                                          hipStream_t s) {
  hipLaunchKernelGGL((k_eval_fj<Model, IO, S>), dim3(blocks_for(n, 64)), dim3(64), 0, s, P, n, q, ld, F, J);
  return hipGetLastError();
}
template <class Model, class IO, class S>
hipError_t OpsImpl<Model, IO, S>::eval_cond(const DevProblem* P, int64_t n, const void* q, int64_t ld, double lambda,
                                            void* kappa, hipStream_t s) {
  hipLaunchKernelGGL((k_eval_cond<Model, IO, S>), dim3(blocks_for(n, 64)), dim3(64), lds_bytes(64), s, P, n, q, ld,
                     lambda, kappa);
  return hipGetLastError();
}
template <class Model, class IO, class S>
hipError_t OpsImpl<Model, IO, S>::project_persistent_wide(const ProjArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_project_persistent_wide<Model, IO, S>), dim3(grid), dim3(256), lds_bytes(256), s, a);
  return hipGetLastError();
}
template <class Model, class IO, class S>
int OpsImpl<Model, IO, S>::persistent_wide_blocks_per_cu() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(&k_project_persistent_wide<Model, IO, S>),
                                                   256, lds_bytes(256)) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

}  // namespace mc

// Explicit instantiation of single launchers of a launcher class O = OpsImpl<M, IO, S> (named through
// an alias, since a template argument list cannot be one macro argument). Each also instantiates the
// kernel it launches.
#define MC_INST_PERSISTENT(O)                                                                        \
  template hipError_t O::project_persistent(const mc::ProjArgs&, int, int, hipStream_t);             \
  template int O::persistent_blocks_per_cu(int);
#define MC_INST_PERSISTENT_CYCLIC(O) \
  template hipError_t O::project_persistent_cyclic(const mc::ProjArgs&, int, int, hipStream_t);
#define MC_INST_TAIL_CYCLIC(O) template hipError_t O::project_tail_cyclic(const mc::ProjArgs&, int, hipStream_t);
#define MC_INST_WIDE(O)                                                                              \
  template hipError_t O::project_persistent_wide(const mc::ProjArgs&, int, hipStream_t);             \
  template int O::persistent_wide_blocks_per_cu();
#define MC_INST_PLAIN(O) template hipError_t O::project_plain(const mc::ProjArgs&, hipStream_t);
#define MC_INST_TAIL(O) template hipError_t O::project_tail(const mc::ProjArgs&, int, hipStream_t);
#define MC_INST_CHECK(O)                                                                             \
  template hipError_t O::check_tail(const mc::ProjArgs&, int, hipStream_t);                           \
  template hipError_t O::check(const mc::CheckArgs&, int, hipStream_t);                                \
  template hipError_t O::check_broad(const mc::CheckArgs&, unsigned*, int32_t*, double*, int64_t, hipStream_t);
#define MC_INST_VJP(O) template hipError_t O::vjp(const mc::VjpArgs&, hipStream_t);
#define MC_INST_VJP_TAIL(O) template hipError_t O::vjp_tail(const mc::VjpArgs&, int, hipStream_t);
#define MC_INST_VJP_EXACT(O) template hipError_t O::vjp_exact(const mc::VjpxArgs&, hipStream_t);
#define MC_INST_DIAG(O)                                                                              \
  template hipError_t O::eval_fj(const mc::DevProblem*, int64_t, const void*, int64_t, void*, void*, hipStream_t); \
  template hipError_t O::eval_cond(const mc::DevProblem*, int64_t, const void*, int64_t, double, void*, hipStream_t);
// every launcher a single-block family uses (its cyclic mode is the stacked one), in one unit
#define MC_INST_LIGHT_F32(O) MC_INST_PERSISTENT(O) MC_INST_PLAIN(O) MC_INST_TAIL(O) MC_INST_CHECK(O) \
  MC_INST_VJP(O) MC_INST_VJP_TAIL(O) MC_INST_VJP_EXACT(O) MC_INST_DIAG(O)
#define MC_INST_LIGHT_F64(O) MC_INST_PERSISTENT(O) MC_INST_PLAIN(O) MC_INST_CHECK(O) MC_INST_VJP(O) \
  MC_INST_VJP_EXACT(O) MC_INST_DIAG(O)
