// Kernel instances of the 2D step with the anti-trapping current folded in.
#include "step2d_at.hpp"

namespace mp {
template int call_step_at<double>(const StepLaunch&, const Coef<double>&, const AtCoef<double>&, KernelCall&);
template int call_step_at<float>(const StepLaunch&, const Coef<float>&, const AtCoef<float>&, KernelCall&);
}  // namespace mp
