// Kernel instantiations: unit sphere F = q.q - 1, FP32 mode (FP64 residual and iterate, FP32 step with FP64 fallback).
#include "kin.hpp"
#include "ops.hpp"
#include "simple_models.hpp"

namespace mc {
const FamilyOps ops_sphere3_f32 = OpsImpl<SphereModel, float, float>::make();
}  // namespace mc
