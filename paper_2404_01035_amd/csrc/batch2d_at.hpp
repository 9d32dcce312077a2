// Batched 2D step with the anti-trapping current of Eq. jatr folded in
// (MICROSIM, arXiv 2404.01035, Sec. 2.1): the batched kernel's persistent
// launch, work list and instance table, each item run by the single grid's
// folded strip (strip2d_at), so a batched instance is stepped bit for bit
// like a single one.  The folded strip holds one cell per lane; an item made
// for V cells per lane (60 V columns) is run as V consecutive strips.  The
// current's coefficients come from a second table, one AtCoef per instance.
#pragma once

#include "batch2d.hpp"
#include "step2d_at.hpp"

namespace mp {

// GEN: the extended model's general strip (x its terms).
template <typename R, int NP, int NM, bool ANISO, bool OBST, bool GEN>
__device__ __forceinline__ void run_strip_at(const R* src, R* dst, const InstDesc<R>& d, const AtCoef<R>& ac,
                                             const CoefX<R>* x, double tb0, int tx, int m0, int m1) {
    for (int sub = 0; sub < d.vec; ++sub) {
        const int t = tx * d.vec + sub;
        if (t * W2X_LANES_OUT >= d.g.nx) break;  // past the instance's last column
        bool fixL, fixR;
        x2_column<1>(d.g, x2_first_col<1>(t, threadIdx.x & 63), fixL, fixR);
        if (__ballot(fixL || fixR) != 0)
            strip2d_at<R, NP, NM, ANISO, OBST, true, GEN>(src, dst, d.g, d.c, ac, tb0, d.tslope, t, m0, m1, x);
        else
            strip2d_at<R, NP, NM, ANISO, OBST, false, GEN>(src, dst, d.g, d.c, ac, tb0, d.tslope, t, m0, m1, x);
    }
}

template <typename R, bool ANISO, bool OBST, bool GEN>
__device__ __forceinline__ void run_item_at(const R* src, R* dst, const InstDesc<R>& d, const AtCoef<R>& ac,
                                            const CoefX<R>* x, double tb0, int tx, int m0, int m1) {
    switch (d.np * 4 + d.nm) {
        case 2 * 4 + 1:
            run_strip_at<R, 2, 1, ANISO, OBST, GEN>(src, dst, d, ac, x, tb0, tx, m0, m1);
            break;
        case 2 * 4 + 2:
            run_strip_at<R, 2, 2, ANISO, OBST, GEN>(src, dst, d, ac, x, tb0, tx, m0, m1);
            break;
        case 3 * 4 + 1:
            run_strip_at<R, 3, 1, ANISO, OBST, GEN>(src, dst, d, ac, x, tb0, tx, m0, m1);
            break;
        default:
            run_strip_at<R, 3, 2, ANISO, OBST, GEN>(src, dst, d, ac, x, tb0, tx, m0, m1);
            break;
    }
}

// GEN: xtab holds the extended coefficients (null otherwise).
template <typename R, bool ANISO, bool OBST, bool GEN>
__device__ __forceinline__ void batch2d_at_items(const R* __restrict__ in, R* __restrict__ out,
                                                 const InstDesc<R>* __restrict__ tab,
                                                 const AtCoef<R>* __restrict__ atab, const CoefX<R>* __restrict__ xtab,
                                                 const int* __restrict__ items, const BatchCuts& cuts,
                                                 const int64_t* __restrict__ stepctr, int kstep) {
    const int nb = gridDim.x;  // a multiple of 8
    const int b = blockIdx.x;
    const int xcd = b % 8;
    const int wpx = (nb / 8) * BATCH_WPB;  // waves per XCD
    const int rank = __builtin_amdgcn_readfirstlane((b / 8) * BATCH_WPB + (threadIdx.x >> 6));
    const int lo = cuts.c[xcd];
    const int hi = cuts.c[xcd + 1];
    const int64_t n = *stepctr + kstep;
    for (int it = lo + rank; it < hi; it += wpx) {
        const int inst = __builtin_amdgcn_readfirstlane(items[2 * it]);
        const int local = __builtin_amdgcn_readfirstlane(items[2 * it + 1]);
        const InstDesc<R>& d = tab[inst];
        const int tx = local % d.ntx;
        const int m0 = (local / d.ntx) * d.seg;
        const int m1 = min(m0 + d.seg, d.g.ny);
        run_item_at<R, ANISO, OBST, GEN>(in + d.off, out + d.off, d, atab[inst], GEN ? &xtab[inst] : nullptr,
                                         d.tb0 + d.tdn * (double)n, tx, m0, m1);
    }
}

template <typename R, bool ANISO, bool OBST>
__global__ void __launch_bounds__(64 * BATCH_WPB) __attribute__((amdgpu_waves_per_eu(2)))
k_batch2d_at(const R* __restrict__ in, R* __restrict__ out, const InstDesc<R>* __restrict__ tab,
             const AtCoef<R>* __restrict__ atab, const int* __restrict__ items, BatchCuts cuts,
             const int64_t* __restrict__ stepctr, int kstep) {
    batch2d_at_items<R, ANISO, OBST, false>(in, out, tab, atab, nullptr, items, cuts, stepctr, kstep);
}

template <typename R, bool ANISO, bool OBST>
__global__ void __launch_bounds__(64 * BATCH_WPB) __attribute__((amdgpu_waves_per_eu(2)))
k_batch2d_at_gen(const R* __restrict__ in, R* __restrict__ out, const InstDesc<R>* __restrict__ tab,
                 const AtCoef<R>* __restrict__ atab, const CoefX<R>* __restrict__ xtab, const int* __restrict__ items,
                 BatchCuts cuts, const int64_t* __restrict__ stepctr, int kstep) {
    batch2d_at_items<R, ANISO, OBST, true>(in, out, tab, atab, xtab, items, cuts, stepctr, kstep);
}

// One step of the batch with the current: L as for call_batch (fuse 1), atab
// the AtCoef<R>[ninst] table in device memory.
template <typename R>
int call_batch_at(const BatchLaunch& L, const void* atab, KernelCall& k) {
    const bool obst = L.potential == MP_OBSTACLE;
    if (L.aniso)
        k.func = obst ? (const void*)&k_batch2d_at<R, true, true> : (const void*)&k_batch2d_at<R, true, false>;
    else
        k.func = obst ? (const void*)&k_batch2d_at<R, false, true> : (const void*)&k_batch2d_at<R, false, false>;
    if (L.nblocks <= 0 || L.nblocks % 8 || L.fuse != 1 || !atab) return MP_E_PARAM;
    k.grid = dim3((unsigned)L.nblocks);
    k.block = dim3(64 * BATCH_WPB);
    k.arg((const R*)L.in);
    k.arg((R*)L.out);
    k.arg((const InstDesc<R>*)L.table);
    k.arg((const AtCoef<R>*)atab);
    k.arg(L.items);
    k.arg(L.cuts);
    k.arg(L.stepctr);
    k.arg(L.kstep);
    return MP_OK;
}

// The same for a batch of the extended model (xtab: CoefX<R>[ninst] in device memory).
template <typename R>
int call_batch_at_gen(const BatchLaunch& L, const void* atab, const void* xtab, KernelCall& k) {
    const bool obst = L.potential != MP_WELL;
    if (L.aniso)
        k.func = obst ? (const void*)&k_batch2d_at_gen<R, true, true> : (const void*)&k_batch2d_at_gen<R, true, false>;
    else
        k.func = obst ? (const void*)&k_batch2d_at_gen<R, false, true> : (const void*)&k_batch2d_at_gen<R, false, false>;
    if (L.nblocks <= 0 || L.nblocks % 8 || L.fuse != 1 || !atab || !xtab) return MP_E_PARAM;
    k.grid = dim3((unsigned)L.nblocks);
    k.block = dim3(64 * BATCH_WPB);
    k.arg((const R*)L.in);
    k.arg((R*)L.out);
    k.arg((const InstDesc<R>*)L.table);
    k.arg((const AtCoef<R>*)atab);
    k.arg((const CoefX<R>*)xtab);
    k.arg(L.items);
    k.arg(L.cuts);
    k.arg(L.stepctr);
    k.arg(L.kstep);
    return MP_OK;
}

}  // namespace mp
