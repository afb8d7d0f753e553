// Kernel instantiations: 36-DoF humanoid tree (feet poses, hands relative pose, CoM xy), FP64 mode:
// the exact VJP through the Newton steps (FP64 arithmetic, double inputs and outputs).
#include "kin.hpp"
#include "ops_impl.hpp"

namespace mc {
using Ops_humanoid36_f64 = OpsImpl<Kin<TopoHumanoid36>, double, double>;
}  // namespace mc
MC_INST_VJP_EXACT(mc::Ops_humanoid36_f64)
