// Kernel instantiations: dual 7-DoF arms, relative end-effector pose (Eq. 2), FP64 mode.
#include "kin.hpp"
#include "ops.hpp"
#include "simple_models.hpp"

namespace mc {
const FamilyOps ops_dual14_rel_f64 = OpsImpl<Kin<TopoDual14Rel>, double, double>::make();
}  // namespace mc
