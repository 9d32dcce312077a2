// Kernel instances of the extended model's general step: precision double, 2d.
#include "step_dispatch.hpp"

namespace mp {
template int call_step_gen<double, false>(const StepLaunch&, const Coef<double>&, const CoefX<double>&, KernelCall&);
}  // namespace mp
