// Kernel instantiations: 36-DoF humanoid tree: feet poses, hands relative pose, CoM xy, FP64 mode.
#include "kin.hpp"
#include "ops.hpp"
#include "simple_models.hpp"

namespace mc {
const FamilyOps ops_humanoid36_f64 = OpsImpl<Kin<TopoHumanoid36>, double, double>::make();
}  // namespace mc
