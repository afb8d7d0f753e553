// Kernel instantiations: unit sphere F = q.q - 1, FP64 mode.
#include "kin.hpp"
#include "ops.hpp"
#include "simple_models.hpp"

namespace mc {
const FamilyOps ops_sphere3_f64 = OpsImpl<SphereModel, double, double>::make();
}  // namespace mc
