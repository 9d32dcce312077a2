// Kernel instances of the fused step: precision double, 2d.
#include "step_dispatch.hpp"

namespace mp {
template int launch_step_dim<double, false>(const StepLaunch&, const Coef<double>&, hipStream_t);
}  // namespace mp
