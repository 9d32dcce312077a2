// Moving frame (the SHIFT / Shiftj keys of Sec. 5): the solidification front's
// row and the shift of a state by whole rows along y with melt appended.
//
// k_front: every cell whose liquid fraction (the last phase) is below 1/2
// contributes its row; a grid-stride pass keeps each thread's highest row, a
// fixed LDS tree the block's, a second one-block pass the grid's (the same
// partial-record scheme as the diagnostics, so nothing is cleared first).
// k_shift: out[f][z][y][x] = in[f][z][y + s][x] while y + s < ny, melt above
// (phases 0 for the solids and 1 for the liquid, the given mu): an HBM copy.
#include "mp_internal.hpp"

namespace mp {
namespace {

constexpr int FT = 256;  // threads per block

__device__ __forceinline__ int block_max(int v) {
    __shared__ int red[FT];
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int w = FT / 2; w > 0; w >>= 1) {
        if (t < w) red[t] = max(red[t], red[t + w]);
        __syncthreads();
    }
    return red[0];
}

template <typename R>
__global__ void __launch_bounds__(FT) k_front(const R* __restrict__ st, int64_t ncells, int nx, int ny, int liq,
                                              int* __restrict__ partial) {
    int best = -1;
    const R* phl = st + (int64_t)liq * ncells;
    const int64_t stride = (int64_t)gridDim.x * FT;
    for (int64_t i = (int64_t)blockIdx.x * FT + threadIdx.x; i < ncells; i += stride)
        if (phl[i] < R(0.5)) best = max(best, (int)((i / nx) % ny));
    best = block_max(best);
    if (threadIdx.x == 0) partial[blockIdx.x] = best;
}

__global__ void __launch_bounds__(FT) k_front_final(const int* __restrict__ partial, int nblocks,
                                                    int64_t* __restrict__ result) {
    int best = -1;
    for (int i = threadIdx.x; i < nblocks; i += FT) best = max(best, partial[i]);
    best = block_max(best);
    if (threadIdx.x == 0) *result = best;
}

template <typename R>
__global__ void __launch_bounds__(FT) k_shift(const R* __restrict__ in, R* __restrict__ out, Geom g, int nfields,
                                              int nphases, int rows, R melt0, R melt1) {
    const int64_t fs = g.fstride;
    const int64_t total = fs * nfields;
    const int64_t stride = (int64_t)gridDim.x * FT;
    for (int64_t e = (int64_t)blockIdx.x * FT + threadIdx.x; e < total; e += stride) {
        const int f = (int)(e / fs);
        const int64_t r = e - (int64_t)f * fs;
        const int y = (int)((r / g.nx) % g.ny);
        R v;
        if (y + rows < g.ny) {
            v = in[e + (int64_t)rows * g.nx];
        } else if (f < nphases) {
            v = f == nphases - 1 ? R(1) : R(0);
        } else {
            v = f == nphases ? melt0 : melt1;
        }
        out[e] = v;
    }
}

int grid_for(int64_t n) {
    int64_t nb = (n + FT - 1) / FT;
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    return (int)nb;
}

}  // namespace

int front_blocks(int64_t ncells) {
    int64_t nb = (ncells + FT - 1) / FT;
    if (nb > DIAG_BLOCKS_MAX) nb = DIAG_BLOCKS_MAX;
    if (nb < 1) nb = 1;
    return (int)nb;
}

int launch_front(const void* state, int precision, const Geom& g, int nphases, int* partials,
                 int64_t* result, hipStream_t s) {
    const int nb = front_blocks(g.fstride);
    if (precision == MP_FP64)
        hipLaunchKernelGGL(k_front<double>, dim3(nb), dim3(FT), 0, s, (const double*)state, g.fstride, g.nx, g.ny,
                           nphases - 1, partials);
    else
        hipLaunchKernelGGL(k_front<float>, dim3(nb), dim3(FT), 0, s, (const float*)state, g.fstride, g.nx, g.ny,
                           nphases - 1, partials);
    hipLaunchKernelGGL(k_front_final, dim3(1), dim3(FT), 0, s, (const int*)partials, nb, result);
    return MP_OK;
}

int launch_shift(const void* in, void* out, int precision, const Geom& g, int nphases, int nmu, int rows,
                 const double* mu_melt, hipStream_t s) {
    const int nf = nphases + nmu;
    const int nb = grid_for(g.fstride * nf);
    const double m0 = nmu > 0 ? mu_melt[0] : 0.0, m1 = nmu > 1 ? mu_melt[1] : 0.0;
    if (precision == MP_FP64)
        hipLaunchKernelGGL(k_shift<double>, dim3(nb), dim3(FT), 0, s, (const double*)in, (double*)out, g, nf, nphases,
                           rows, m0, m1);
    else
        hipLaunchKernelGGL(k_shift<float>, dim3(nb), dim3(FT), 0, s, (const float*)in, (float*)out, g, nf, nphases,
                           rows, (float)m0, (float)m1);
    return MP_OK;
}

}  // namespace mp
