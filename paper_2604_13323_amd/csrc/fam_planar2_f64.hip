// Kernel instantiations: planar 2R arm, tip position, FP64 mode.
#include "kin.hpp"
#include "simple_models.hpp"
#include "ops_impl.hpp"

namespace mc {
using Ops_planar2_f64 = OpsImpl<Kin<TopoPlanar2>, double, double>;
}  // namespace mc
MC_INST_LIGHT_F64(mc::Ops_planar2_f64)

namespace mc {
const FamilyOps ops_planar2_f64 = Ops_planar2_f64::make();
}  // namespace mc
