// Kernel instances of the fused step: precision float, 3d.
#include "step_dispatch.hpp"

namespace mp {
template int call_step_dim<float, true>(const StepLaunch&, const Coef<float>&, KernelCall&);
}  // namespace mp
