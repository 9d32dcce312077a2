// Kernel instances of the 2D step with the anti-trapping current folded in,
// extended model (general kernels).
#include "step2d_at.hpp"

namespace mp {
template int call_step_at_gen<double>(const StepLaunch&, const Coef<double>&, const AtCoef<double>&,
                                      const CoefX<double>&, KernelCall&);
template int call_step_at_gen<float>(const StepLaunch&, const Coef<float>&, const AtCoef<float>&,
                                     const CoefX<float>&, KernelCall&);
}  // namespace mp
