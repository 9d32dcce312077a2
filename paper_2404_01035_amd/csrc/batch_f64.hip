// Batched kernel instances, FP64.
#include "batch2d.hpp"

namespace mp {
template int call_batch<double>(const BatchLaunch&, KernelCall&);
}  // namespace mp
