// Kernel instantiations: 36-DoF humanoid tree with the Digit constraint set (feet poses, hands relative pose, CoM in the support polygon, closed-linkage rods), FP64 mode:
// the cyclic persistent kernel.
#include "kin.hpp"
#include "ops_impl.hpp"

namespace mc {
using Ops_digit36_f64 = OpsImpl<Kin<TopoDigit36>, double, double>;
}  // namespace mc
MC_INST_PERSISTENT_CYCLIC(mc::Ops_digit36_f64)
