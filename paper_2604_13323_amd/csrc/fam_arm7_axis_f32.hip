// Kernel instantiations: 7-DoF arm, end-effector z parallel to world z, FP32 mode (FP64 residual and iterate, FP32 step with FP64 fallback).
#include "kin.hpp"
#include "ops.hpp"
#include "simple_models.hpp"

namespace mc {
const FamilyOps ops_arm7_axis_f32 = OpsImpl<Kin<TopoArm7Axis>, float, float>::make();
}  // namespace mc
