// Kernel instances of the fused step: precision double, 3d.
#include "step_dispatch.hpp"

namespace mp {
template int launch_step_dim<double, true>(const StepLaunch&, const Coef<double>&, hipStream_t);
}  // namespace mp
