// Batched kernel instances with the anti-trapping current folded in.
#include "batch2d_at.hpp"

namespace mp {
template int call_batch_at<double>(const BatchLaunch&, const void*, KernelCall&);
template int call_batch_at<float>(const BatchLaunch&, const void*, KernelCall&);
}  // namespace mp
