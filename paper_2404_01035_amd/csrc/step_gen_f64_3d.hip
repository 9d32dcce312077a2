// Kernel instances of the extended model's general step: precision double, 3d.
#include "step_dispatch.hpp"

namespace mp {
template int call_step_gen<double, true>(const StepLaunch&, const Coef<double>&, const CoefX<double>&, KernelCall&);
}  // namespace mp
