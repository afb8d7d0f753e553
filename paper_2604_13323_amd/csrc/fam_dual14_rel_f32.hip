// Kernel instantiations: dual 7-DoF arms, relative end-effector pose (Eq. 2), FP32 mode (FP64 residual and iterate, FP32 step with FP64 fallback).
#include "kin.hpp"
#include "ops.hpp"
#include "simple_models.hpp"

namespace mc {
const FamilyOps ops_dual14_rel_f32 = OpsImpl<Kin<TopoDual14Rel>, float, float>::make();
}  // namespace mc
