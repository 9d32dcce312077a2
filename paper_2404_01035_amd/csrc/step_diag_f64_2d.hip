// Kernel instances of the fused step that also writes the partial
// diagnostics records of the stored state: precision double, 2d.
#include "step_dispatch.hpp"

namespace mp {
template int call_step_dim<double, false, true>(const StepLaunch&, const Coef<double>&, KernelCall&);
}  // namespace mp
