// Batched kernel instances of the extended model, plain and with the
// anti-trapping current folded in.
#include "batch2d_at.hpp"
#include "batch2d_gen.hpp"

namespace mp {
template int call_batch_gen<double>(const BatchLaunch&, const void*, KernelCall&);
template int call_batch_gen<float>(const BatchLaunch&, const void*, KernelCall&);
template int call_batch_at_gen<double>(const BatchLaunch&, const void*, const void*, KernelCall&);
template int call_batch_at_gen<float>(const BatchLaunch&, const void*, const void*, KernelCall&);
}  // namespace mp
