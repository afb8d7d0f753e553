// Kernel instantiations: linear constraints F = A q - b, FP64 mode.
#include "kin.hpp"
#include "ops.hpp"
#include "simple_models.hpp"

namespace mc {
const FamilyOps ops_linear_f64 = OpsImpl<LinearModel, double, double>::make();
}  // namespace mc
