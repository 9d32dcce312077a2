// Kernel instances of the fused step that also writes the partial
// diagnostics records of the stored state: precision float, 3d.
#include "step_dispatch.hpp"

namespace mp {
template int call_step_dim<float, true, true>(const StepLaunch&, const Coef<float>&, KernelCall&);
}  // namespace mp
