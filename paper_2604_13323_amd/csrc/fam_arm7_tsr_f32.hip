// Kernel instantiations: 7-DoF arm, TSR pose block with finite bounds on the end-effector frame, FP32 mode (FP64 residual and iterate, FP32 step with FP64 fallback).
#include "kin.hpp"
#include "simple_models.hpp"
#include "ops_impl.hpp"

namespace mc {
using Ops_arm7_tsr_f32 = OpsImpl<Kin<TopoArm7Tsr>, float, float>;
}  // namespace mc
MC_INST_LIGHT_F32(mc::Ops_arm7_tsr_f32)

namespace mc {
const FamilyOps ops_arm7_tsr_f32 = Ops_arm7_tsr_f32::make();
}  // namespace mc
