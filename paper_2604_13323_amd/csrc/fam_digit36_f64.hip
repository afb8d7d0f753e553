// Launch table of the 36-DoF humanoid tree with the Digit constraint set (feet poses, hands relative pose, CoM in the support polygon, closed-linkage rods), FP64 mode.
// The launchers it names are instantiated, with their kernels, in the fam_digit36_f64_*.hip units
// (this unit sees only their declarations, so it compiles no kernel).
#include "kin.hpp"
#include "ops.hpp"

namespace mc {
const FamilyOps ops_digit36_f64 = OpsImpl<Kin<TopoDigit36>, double, double>::make();
}  // namespace mc
