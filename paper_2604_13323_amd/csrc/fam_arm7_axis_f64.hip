// Kernel instantiations: 7-DoF arm, end-effector z parallel to world z, FP64 mode.
#include "kin.hpp"
#include "ops.hpp"
#include "simple_models.hpp"

namespace mc {
const FamilyOps ops_arm7_axis_f64 = OpsImpl<Kin<TopoArm7Axis>, double, double>::make();
}  // namespace mc
