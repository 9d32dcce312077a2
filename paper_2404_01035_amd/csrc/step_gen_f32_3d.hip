// Kernel instances of the extended model's general step: precision float, 3d.
#include "step_dispatch.hpp"

namespace mp {
template int call_step_gen<float, true>(const StepLaunch&, const Coef<float>&, const CoefX<float>&, KernelCall&);
}  // namespace mp
