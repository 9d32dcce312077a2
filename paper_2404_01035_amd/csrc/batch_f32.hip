// Batched kernel instances, FP32, plus the step-counter kernel.
#include "batch2d.hpp"

namespace mp {
template int call_batch<float>(const BatchLaunch&, KernelCall&);

// Advances the device time level after a run of launches (a kernel node, so
// it can sit inside a replayed graph).
__global__ void k_advance(int64_t* ctr, int64_t by) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *ctr += by;
}

void call_advance(int64_t* ctr, int64_t by, KernelCall& k) {
    k.func = (const void*)&k_advance;
    k.grid = dim3(1);
    k.block = dim3(64);
    k.arg(ctr);
    k.arg(by);
}
}  // namespace mp
