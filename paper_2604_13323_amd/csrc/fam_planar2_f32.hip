// Kernel instantiations: planar 2R arm, tip position, FP32 mode (FP64 residual and iterate, FP32 step with FP64 fallback).
#include "kin.hpp"
#include "simple_models.hpp"
#include "ops_impl.hpp"

namespace mc {
using Ops_planar2_f32 = OpsImpl<Kin<TopoPlanar2>, float, float>;
}  // namespace mc
MC_INST_LIGHT_F32(mc::Ops_planar2_f32)

namespace mc {
const FamilyOps ops_planar2_f32 = Ops_planar2_f32::make();
}  // namespace mc
