// Kernel instantiations: 7-DoF arm, TSR pose block with finite bounds on the end-effector frame, FP64 mode.
#include "kin.hpp"
#include "simple_models.hpp"
#include "ops_impl.hpp"

namespace mc {
using Ops_arm7_tsr_f64 = OpsImpl<Kin<TopoArm7Tsr>, double, double>;
}  // namespace mc
MC_INST_LIGHT_F64(mc::Ops_arm7_tsr_f64)

namespace mc {
const FamilyOps ops_arm7_tsr_f64 = Ops_arm7_tsr_f64::make();
}  // namespace mc
