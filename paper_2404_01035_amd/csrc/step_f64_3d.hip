// Kernel instances of the fused step: precision double, 3d.
#include "step_dispatch.hpp"

namespace mp {
template int call_step_dim<double, true>(const StepLaunch&, const Coef<double>&, KernelCall&);
}  // namespace mp
