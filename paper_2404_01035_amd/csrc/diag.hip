// Global diagnostics of a state: solute mass sum_cells c_k dx^d with
// c_k = sum_a h_a(phi) c^a_k(mu) (the composition constraint of Sec. 2.1),
// phase volumes sum_cells phi_a dx^d, max |sum_a phi_a - 1|, min chi_k and the
// count of non-finite cells.  Sums are FP64 with Neumaier compensation; the
// grid, the per-thread stride and both tree reductions are fixed by the cell
// count alone, so the result is bitwise reproducible run to run.
#include <mutex>

#include "diag_cell.hpp"
#include "diag_static.hpp"
#include "mp_internal.hpp"

namespace mp {

// The device memory of mp_diagnostics_static: the per-block partial records
// and one result record per instance, in the library's own storage instead of
// a caller workspace.  Each GPU the library runs on holds its own copy until
// the process ends.  Host code must not pass the array's name to a kernel (it
// is a host-side stand-in there): diag_static_scratch returns its address on
// the current device.
static __device__ __align__(256) double scratch[(DIAG_BLOCKS_MAX + DIAG_STATIC_INST) * DIAG_VALS];

hipError_t diag_static_scratch(double** out) {
    constexpr int kMaxDev = 64;
    static std::mutex lock;
    static double* addr[kMaxDev] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDev) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(lock);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = (double*)p;
    }
    *out = addr[dev];
    return hipSuccess;
}


namespace {

constexpr int DT = 256;  // threads per diagnostics block

// Fixed-shape tree over the block's records in LDS.
__device__ void block_tree(DiagRec& A, double (*rec)[DIAG_VALS]) {
    const int t = threadIdx.x;
    rec_store(rec[t], A);
    __syncthreads();
    for (int w = DT / 2; w > 0; w >>= 1) {
        if (t < w) {
            DiagRec a, b;
            rec_load(a, rec[t]);
            rec_load(b, rec[t + w]);
            rec_merge(a, b);
            rec_store(rec[t], a);
        }
        __syncthreads();
    }
    rec_load(A, rec[0]);
}

template <typename R, int NP, int NM>
__global__ void __launch_bounds__(DT) k_diag(const R* __restrict__ st, int64_t ncells, DiagCoef dc,
                                             double* __restrict__ partial) {
    __shared__ double rec[DT][DIAG_VALS];
    DiagAcc A;
    acc_init(A);
    const int64_t stride = (int64_t)gridDim.x * DT;
    for (int64_t i = (int64_t)blockIdx.x * DT + threadIdx.x; i < ncells; i += stride) {
        double p[NP], mu[NM];
        for (int a = 0; a < NP; ++a) p[a] = (double)st[a * ncells + i];
        for (int k = 0; k < NM; ++k) mu[k] = (double)st[(NP + k) * ncells + i];
        // T - Te of the cell's row (the composition depends on T through B(T))
        const double tt = dc.tt0 + dc.tslope * (double)((i / dc.nx) % dc.ny);
        diag_cell<NP, NM, true>(p, mu, tt, dc, A);
    }
    DiagRec B;
    rec_from(B, A);
    block_tree(B, rec);
    if (threadIdx.x == 0) rec_store(partial + (int64_t)blockIdx.x * DIAG_VALS, B);
}

__global__ void __launch_bounds__(DT) k_diag_final(const double* __restrict__ partial, int nblocks,
                                                   double* __restrict__ result) {
    __shared__ double rec[DT][DIAG_VALS];
    DiagRec A;
    rec_init(A);
    for (int i = threadIdx.x; i < nblocks; i += DT) {
        DiagRec b;
        rec_load(b, partial + (int64_t)i * DIAG_VALS);
        rec_merge(A, b);
    }
    block_tree(A, rec);
    if (threadIdx.x == 0) rec_store(result, A);
}

template <typename R, int NP, int NM>
int launch_diag_t(const void* state, const Geom& g, const DiagCoef& dc, double* partials,
                  double* result, hipStream_t s) {
    const int64_t n = g.fstride;
    const int nb = diag_blocks(n);
    hipLaunchKernelGGL((k_diag<R, NP, NM>), dim3(nb), dim3(DT), 0, s, (const R*)state, n, dc, partials);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(DT), 0, s, (const double*)partials, nb, result);
    return MP_OK;
}

template <typename R>
int launch_diag_r(const void* state, const Geom& g, int np, int nm, const DiagCoef& dc,
                  double* partials, double* result, hipStream_t s) {
    if (np == 2 && nm == 1) return launch_diag_t<R, 2, 1>(state, g, dc, partials, result, s);
    if (np == 2 && nm == 2) return launch_diag_t<R, 2, 2>(state, g, dc, partials, result, s);
    if (np == 3 && nm == 1) return launch_diag_t<R, 3, 1>(state, g, dc, partials, result, s);
    if (np == 3 && nm == 2) return launch_diag_t<R, 3, 2>(state, g, dc, partials, result, s);
    return MP_E_PARAM;
}

}  // namespace

int diag_blocks(int64_t ncells) {
    int64_t nb = (ncells + DT - 1) / DT;
    if (nb > DIAG_BLOCKS_MAX) nb = DIAG_BLOCKS_MAX;
    if (nb < 1) nb = 1;
    return (int)nb;
}

int launch_diag_final(const double* partials, int64_t nrec, double* result, hipStream_t s) {
    if (nrec < 1 || nrec > 0x7fffffffLL) return MP_E_PARAM;
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(DT), 0, s, partials, (int)nrec, result);
    return MP_OK;
}

int launch_diag(const void* state, int precision, const Geom& g, int nphases, int nmu,
                const DiagCoef& dc, double* partials, double* result, hipStream_t s) {
    if (precision == MP_FP64)
        return launch_diag_r<double>(state, g, nphases, nmu, dc, partials, result, s);
    return launch_diag_r<float>(state, g, nphases, nmu, dc, partials, result, s);
}

}  // namespace mp
