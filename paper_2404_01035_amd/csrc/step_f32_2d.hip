// Kernel instances of the fused step: precision float, 2d.
#include "step_dispatch.hpp"

namespace mp {
template int call_step_dim<float, false>(const StepLaunch&, const Coef<float>&, KernelCall&);
}  // namespace mp
