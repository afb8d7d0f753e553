// Kernel instantiations: planar 2R arm, tip position, FP32 mode (FP64 residual and iterate, FP32 step with FP64 fallback).
#include "kin.hpp"
#include "ops.hpp"
#include "simple_models.hpp"

namespace mc {
const FamilyOps ops_planar2_f32 = OpsImpl<Kin<TopoPlanar2>, float, float>::make();
}  // namespace mc
