// Kernel instantiations: 36-DoF humanoid tree (feet poses, hands relative pose, CoM xy), FP64 mode:
// the persistent kernel in cyclic mode.
#include "kin.hpp"
#include "ops_impl.hpp"

namespace mc {
using Ops_humanoid36_f64 = OpsImpl<Kin<TopoHumanoid36>, double, double>;
}  // namespace mc
MC_INST_PERSISTENT_CYCLIC(mc::Ops_humanoid36_f64)
