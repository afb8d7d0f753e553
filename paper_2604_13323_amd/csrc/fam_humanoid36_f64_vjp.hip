// Kernel instantiations: 36-DoF humanoid tree (feet poses, hands relative pose, CoM xy), FP64 mode:
// the VJP kernel and the diagnostics.
#include "kin.hpp"
#include "ops_impl.hpp"

namespace mc {
using Ops_humanoid36_f64 = OpsImpl<Kin<TopoHumanoid36>, double, double>;
}  // namespace mc
MC_INST_VJP(mc::Ops_humanoid36_f64)
MC_INST_DIAG(mc::Ops_humanoid36_f64)
