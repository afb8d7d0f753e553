// Kernel instantiations: 36-DoF humanoid tree: feet poses, hands relative pose, CoM xy, FP32 mode (FP64 residual and iterate, FP32 step with FP64 fallback).
#include "kin.hpp"
#include "ops.hpp"
#include "simple_models.hpp"

namespace mc {
const FamilyOps ops_humanoid36_f32 = OpsImpl<Kin<TopoHumanoid36>, float, float>::make();
}  // namespace mc
