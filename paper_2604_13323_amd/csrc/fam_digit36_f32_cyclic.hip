// Kernel instantiations: 36-DoF humanoid tree with the Digit constraint set (feet poses, hands relative pose, CoM in the support polygon, closed-linkage rods), FP32 mode (FP64 residual and iterate, FP32 step with FP64 fallback):
// the cyclic persistent kernel.
#include "kin.hpp"
#include "ops_impl.hpp"

namespace mc {
using Ops_digit36_f32 = OpsImpl<Kin<TopoDigit36>, float, float>;
}  // namespace mc
MC_INST_PERSISTENT_CYCLIC(mc::Ops_digit36_f32)
