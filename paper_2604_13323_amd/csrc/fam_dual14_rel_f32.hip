// Kernel instantiations: two 7-DoF arms, relative end-effector pose (Eq. 2), FP32 mode (FP64 residual and iterate, FP32 step with FP64 fallback).
#include "kin.hpp"
#include "simple_models.hpp"
#include "ops_impl.hpp"

namespace mc {
using Ops_dual14_rel_f32 = OpsImpl<Kin<TopoDual14Rel>, float, float>;
}  // namespace mc
MC_INST_LIGHT_F32(mc::Ops_dual14_rel_f32)

namespace mc {
const FamilyOps ops_dual14_rel_f32 = Ops_dual14_rel_f32::make();
}  // namespace mc
