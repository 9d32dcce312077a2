// Kernel instances of the extended model's general step that also writes the partial
// diagnostics records of the stored state: precision float, 3d.
#include "step_dispatch.hpp"

namespace mp {
template int call_step_gen<float, true, true>(const StepLaunch&, const Coef<float>&, const CoefX<float>&, KernelCall&);
}  // namespace mp
