// Adjoint kernel instances, FP32, and the small helpers of the adjoint driver.
#include "adjoint2d.hpp"

namespace mp {
template int adj_launch<float>(const AdjLaunch&, const AdjCoef<float>&, hipStream_t);

__global__ void k_fill_f64(double* p, int64_t n, double v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Column sums of the per-block accumulator rows, each in a fixed order.
__global__ void k_adj_reduce(const double* __restrict__ acc, int nrows, double* __restrict__ out) {
    const int q = threadIdx.x;
    if (q < ADJ_NPAR) {
        double s = 0.0;
        for (int r = 0; r < nrows; ++r) s += acc[(size_t)r * ADJ_NPAR + q];
        out[q] = s;
    }
}

void adj_fill(double* p, int64_t n, double v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_f64, dim3(64), dim3(256), 0, s, p, n, v);
}

void adj_reduce(const double* acc, int nrows, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_reduce, dim3(1), dim3(64), 0, s, acc, nrows, out);
}
}  // namespace mp
