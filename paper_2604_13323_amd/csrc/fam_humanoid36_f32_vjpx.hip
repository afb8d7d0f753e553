// Kernel instantiations: 36-DoF humanoid tree (feet poses, hands relative pose, CoM xy), FP32 mode (FP64 residual and iterate, FP32 step with FP64 fallback):
// the exact VJP through the Newton steps (FP64 arithmetic, float inputs and outputs).
#include "kin.hpp"
#include "ops_impl.hpp"

namespace mc {
using Ops_humanoid36_f32 = OpsImpl<Kin<TopoHumanoid36>, float, float>;
}  // namespace mc
MC_INST_VJP_EXACT(mc::Ops_humanoid36_f32)
