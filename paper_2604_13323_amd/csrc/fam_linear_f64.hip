// Kernel instantiations: linear constraint F = A q - b, FP64 mode.
#include "kin.hpp"
#include "simple_models.hpp"
#include "ops_impl.hpp"

namespace mc {
using Ops_linear_f64 = OpsImpl<LinearModel, double, double>;
}  // namespace mc
MC_INST_LIGHT_F64(mc::Ops_linear_f64)

namespace mc {
const FamilyOps ops_linear_f64 = Ops_linear_f64::make();
}  // namespace mc
