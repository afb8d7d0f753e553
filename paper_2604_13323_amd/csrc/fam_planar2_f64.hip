// Kernel instantiations: planar 2R arm, tip position, FP64 mode.
#include "kin.hpp"
#include "ops.hpp"
#include "simple_models.hpp"

namespace mc {
const FamilyOps ops_planar2_f64 = OpsImpl<Kin<TopoPlanar2>, double, double>::make();
}  // namespace mc
