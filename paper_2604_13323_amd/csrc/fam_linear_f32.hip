// Kernel instantiations: linear constraints F = A q - b, FP32 mode (FP64 residual and iterate, FP32 step with FP64 fallback).
#include "kin.hpp"
#include "ops.hpp"
#include "simple_models.hpp"

namespace mc {
const FamilyOps ops_linear_f32 = OpsImpl<LinearModel, float, float>::make();
}  // namespace mc
