// Kernel instantiations: two 7-DoF arms, relative end-effector pose (Eq. 2), FP64 mode.
#include "kin.hpp"
#include "simple_models.hpp"
#include "ops_impl.hpp"

namespace mc {
using Ops_dual14_rel_f64 = OpsImpl<Kin<TopoDual14Rel>, double, double>;
}  // namespace mc
MC_INST_LIGHT_F64(mc::Ops_dual14_rel_f64)

namespace mc {
const FamilyOps ops_dual14_rel_f64 = Ops_dual14_rel_f64::make();
}  // namespace mc
