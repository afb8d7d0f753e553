// Launch table of the 36-DoF humanoid tree (feet poses, hands relative pose, CoM xy), FP64 mode.
// The launchers it names are instantiated, with their kernels, in the fam_humanoid36_f64_*.hip units
// (this unit sees only their declarations, so it compiles no kernel).
#include "kin.hpp"
#include "ops.hpp"

namespace mc {
const FamilyOps ops_humanoid36_f64 = OpsImpl<Kin<TopoHumanoid36>, double, double>::make();
}  // namespace mc
