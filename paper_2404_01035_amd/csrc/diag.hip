// Global diagnostics of a state: solute mass sum_cells c_k dx^d with
// c_k = sum_a h_a(phi) c^a_k(mu) (the composition constraint of Sec. 2.1),
// phase volumes sum_cells phi_a dx^d, max |sum_a phi_a - 1|, min chi_k and the
// count of non-finite cells.  Sums are FP64 with Neumaier compensation; the
// grid, the per-thread stride and both tree reductions are fixed by the cell
// count alone, so the result is bitwise reproducible run to run.
#include <mutex>

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

struct Neu {
    double s, c;
};

__device__ __forceinline__ void neu_add(Neu& a, double x) {
    double t = a.s + x;
    if (fabs(a.s) >= fabs(x))
        a.c += (a.s - t) + x;
    else
        a.c += (x - t) + a.s;
    a.s = t;
}

__device__ __forceinline__ void neu_merge(Neu& a, const Neu& b) {
    neu_add(a, b.s);
    a.c += b.c;
}

template <int NP>
__device__ __forceinline__ void h_fp64(const double (&p)[NP], double (&h)[NP]) {
    for (int a = 0; a < NP; ++a) {
        double o = 0.0;
        if (NP == 3) {
            int b = (a + 1) % 3, g = (a + 2) % 3;
            o = p[b] * p[g];
        }
        h[a] = 3.0 * p[a] * p[a] - 2.0 * p[a] * p[a] * p[a] + 2.0 * p[a] * o;
    }
}

struct Acc {
    Neu mass[2];
    Neu vol[3];
    double maxdev;
    double minchi[2];
    double nonfin;
};

__device__ __forceinline__ void acc_init(Acc& A) {
    for (int k = 0; k < 2; ++k) A.mass[k] = {0.0, 0.0};
    for (int a = 0; a < 3; ++a) A.vol[a] = {0.0, 0.0};
    A.maxdev = 0.0;
    A.minchi[0] = A.minchi[1] = INFINITY;
    A.nonfin = 0.0;
}

__device__ __forceinline__ void acc_merge(Acc& A, const Acc& B) {
    for (int k = 0; k < 2; ++k) neu_merge(A.mass[k], B.mass[k]);
    for (int a = 0; a < 3; ++a) neu_merge(A.vol[a], B.vol[a]);
    A.maxdev = fmax(A.maxdev, B.maxdev);
    A.minchi[0] = fmin(A.minchi[0], B.minchi[0]);
    A.minchi[1] = fmin(A.minchi[1], B.minchi[1]);
    A.nonfin += B.nonfin;
}

__device__ __forceinline__ void acc_store(double* r, const Acc& A) {
    for (int k = 0; k < 2; ++k) {
        r[DV_MASS + 2 * k] = A.mass[k].s;
        r[DV_MASS + 2 * k + 1] = A.mass[k].c;
    }
    for (int a = 0; a < 3; ++a) {
        r[DV_VOL + 2 * a] = A.vol[a].s;
        r[DV_VOL + 2 * a + 1] = A.vol[a].c;
    }
    r[DV_MAXDEV] = A.maxdev;
    r[DV_MINCHI] = A.minchi[0];
    r[DV_MINCHI + 1] = A.minchi[1];
    r[DV_NONFIN] = A.nonfin;
}

__device__ __forceinline__ void acc_load(Acc& A, const double* r) {
    for (int k = 0; k < 2; ++k) A.mass[k] = {r[DV_MASS + 2 * k], r[DV_MASS + 2 * k + 1]};
    for (int a = 0; a < 3; ++a) A.vol[a] = {r[DV_VOL + 2 * a], r[DV_VOL + 2 * a + 1]};
    A.maxdev = r[DV_MAXDEV];
    A.minchi[0] = r[DV_MINCHI];
    A.minchi[1] = r[DV_MINCHI + 1];
    A.nonfin = r[DV_NONFIN];
}

// Fixed-shape tree over the block's records in LDS.
__device__ void block_tree(Acc& A, double (*rec)[DIAG_VALS]) {
    const int t = threadIdx.x;
    acc_store(rec[t], A);
    __syncthreads();
    for (int w = DT / 2; w > 0; w >>= 1) {
        if (t < w) {
            Acc a, b;
            acc_load(a, rec[t]);
            acc_load(b, rec[t + w]);
            acc_merge(a, b);
            acc_store(rec[t], a);
        }
        __syncthreads();
    }
    acc_load(A, rec[0]);
}

template <typename R, int NP, int NM>
__global__ void __launch_bounds__(DT) k_diag(const R* __restrict__ st, int64_t ncells, DiagCoef dc,
                                             double* __restrict__ partial) {
    __shared__ double rec[DT][DIAG_VALS];
    Acc A;
    acc_init(A);
    const int64_t stride = (int64_t)gridDim.x * DT;
    for (int64_t i = (int64_t)blockIdx.x * DT + threadIdx.x; i < ncells; i += stride) {
        double p[NP], mu[NM], h[NP];
        bool fin = true;
        double sum = 0.0;
        for (int a = 0; a < NP; ++a) {
            p[a] = (double)st[a * ncells + i];
            fin = fin && isfinite(p[a]);
            sum += p[a];
        }
        for (int k = 0; k < NM; ++k) {
            mu[k] = (double)st[(NP + k) * ncells + i];
            fin = fin && isfinite(mu[k]);
        }
        if (!fin) A.nonfin += 1.0;
        h_fp64<NP>(p, h);
        A.maxdev = fmax(A.maxdev, fabs(sum - 1.0));
        for (int a = 0; a < NP; ++a) neu_add(A.vol[a], p[a] * dc.vol);
        // T - Te of the cell's row (the composition depends on T through B(T))
        const double tt = dc.tt0 + dc.tslope * (double)((i / dc.nx) % dc.ny);
        double dm[NP][NM];
        for (int a = 0; a < NP; ++a)
            for (int k = 0; k < NM; ++k) dm[a][k] = mu[k] - dc.B[a][k] - dc.Bt[a][k] * tt;
        for (int k = 0; k < NM; ++k) {
            double cc = 0.0, chi = 0.0;
            for (int a = 0; a < NP; ++a) {
                double ca = dm[a][k] * dc.chi[a][k];
                if (NM == 2) ca += dm[a][1 - k] * dc.chx[a];  // c^a = chi^a (mu - B^a(T))
                cc += h[a] * ca;
                chi += h[a] * dc.chi[a][k];
            }
            neu_add(A.mass[k], cc * dc.vol);
            A.minchi[k] = fmin(A.minchi[k], chi);
        }
    }
    block_tree(A, rec);
    if (threadIdx.x == 0) acc_store(partial + (int64_t)blockIdx.x * DIAG_VALS, A);
}

__global__ void __launch_bounds__(DT) k_diag_final(const double* __restrict__ partial, int nblocks,
                                                   double* __restrict__ result) {
    __shared__ double rec[DT][DIAG_VALS];
    Acc A;
    acc_init(A);
    for (int i = threadIdx.x; i < nblocks; i += DT) {
        Acc b;
        acc_load(b, partial + (int64_t)i * DIAG_VALS);
        acc_merge(A, b);
    }
    block_tree(A, rec);
    if (threadIdx.x == 0) acc_store(result, A);
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

int launch_diag(const void* state, int precision, const Geom& g, int nphases, int nmu,
                const DiagCoef& dc, double* partials, double* result, hipStream_t s) {
    if (precision == MP_FP64)
        return launch_diag_r<double>(state, g, nphases, nmu, dc, partials, result, s);
    return launch_diag_r<float>(state, g, nphases, nmu, dc, partials, result, s);
}

}  // namespace mp
