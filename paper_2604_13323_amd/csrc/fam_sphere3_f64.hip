// Kernel instantiations: unit sphere F = q.q - 1, FP64 mode.
#include "kin.hpp"
#include "simple_models.hpp"
#include "ops_impl.hpp"

namespace mc {
using Ops_sphere3_f64 = OpsImpl<SphereModel, double, double>;
}  // namespace mc
MC_INST_LIGHT_F64(mc::Ops_sphere3_f64)

namespace mc {
const FamilyOps ops_sphere3_f64 = Ops_sphere3_f64::make();
}  // namespace mc
