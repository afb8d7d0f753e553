// Kernel instantiations: 36-DoF humanoid tree with the Digit constraint set (feet poses, hands relative pose, CoM in the support polygon, closed-linkage rods), FP64 mode:
// the VJP kernels and the diagnostics.
#include "kin.hpp"
#include "ops_impl.hpp"

namespace mc {
using Ops_digit36_f64 = OpsImpl<Kin<TopoDigit36>, double, double>;
}  // namespace mc
MC_INST_VJP(mc::Ops_digit36_f64)
MC_INST_DIAG(mc::Ops_digit36_f64)
