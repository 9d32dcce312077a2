// Kernel instances of the extended model's general step that also writes the partial
// diagnostics records of the stored state: precision double, 2d.
#include "step_dispatch.hpp"

namespace mp {
template int call_step_gen<double, false, true>(const StepLaunch&, const Coef<double>&, const CoefX<double>&, KernelCall&);
}  // namespace mp
