// Launch table of the 36-DoF humanoid tree with the Digit constraint set (feet poses, hands relative pose, CoM in the support polygon, closed-linkage rods), FP32 mode (FP64 residual and iterate, FP32 step with FP64 fallback).
// The launchers it names are instantiated, with their kernels, in the fam_digit36_f32_*.hip units
// (this unit sees only their declarations, so it compiles no kernel).
#include "kin.hpp"
#include "ops.hpp"

namespace mc {
const FamilyOps ops_digit36_f32 = OpsImpl<Kin<TopoDigit36>, float, float>::make();
}  // namespace mc
