// Batched 2D step of the extended model (temperature-dependent B and C with
// the dT/dt term, per-pair relaxation, the active-set obstacle, off-diagonal
// susceptibility and mobility): the batched kernel's persistent launch, work
// list and instance table, each item run by the general strips of the single
// grid (one cell per lane; an item made for V cells per lane is V strips),
// with the extended coefficients from a second table, one CoefX per instance.
// A batch that holds one extended instance steps all of its instances with
// these kernels.
#pragma once

#include "batch2d.hpp"

namespace mp {

template <typename R, int NP, int NM, bool ANISO, bool OBST, int FUSE>
__device__ __forceinline__ void run_strip_gen(const R* src, R* dst, const InstDesc<R>& d, const CoefX<R>& x,
                                              double tb0, double tb1, int tx, int m0, int m1) {
    for (int sub = 0; sub < d.vec; ++sub) {
        const int t = tx * d.vec + sub;
        if (t * BATCH_W >= d.g.nx) break;  // past the instance's last column
        if constexpr (FUSE == 2)
            strip2d_x2<R, NP, NM, ANISO, OBST, 1, true, false, true>(src, dst, nullptr, d.g, d.c, tb0, tb1, d.tslope,
                                                                    t, m0, m1, &x);
        else
            strip2d<R, NP, NM, ANISO, OBST, 1, MP_STRIP_DEPTH, BATCH_W, true>(src, dst, d.g, d.c, tb0, d.tslope, t,
                                                                             m0, m1, &x);
    }
}

template <typename R, bool ANISO, bool OBST, int FUSE>
__device__ __forceinline__ void run_item_gen(const R* src, R* dst, const InstDesc<R>& d, const CoefX<R>& x,
                                             double tb0, double tb1, int tx, int m0, int m1) {
    switch (d.np * 4 + d.nm) {
        case 2 * 4 + 1:
            run_strip_gen<R, 2, 1, ANISO, OBST, FUSE>(src, dst, d, x, tb0, tb1, tx, m0, m1);
            break;
        case 2 * 4 + 2:
            run_strip_gen<R, 2, 2, ANISO, OBST, FUSE>(src, dst, d, x, tb0, tb1, tx, m0, m1);
            break;
        case 3 * 4 + 1:
            run_strip_gen<R, 3, 1, ANISO, OBST, FUSE>(src, dst, d, x, tb0, tb1, tx, m0, m1);
            break;
        default:
            run_strip_gen<R, 3, 2, ANISO, OBST, FUSE>(src, dst, d, x, tb0, tb1, tx, m0, m1);
            break;
    }
}

template <typename R, bool ANISO, bool OBST, int FUSE>
__global__ void __launch_bounds__(64 * BATCH_WPB) __attribute__((amdgpu_waves_per_eu(2)))
k_batch2d_gen(const R* __restrict__ in, R* __restrict__ out, const InstDesc<R>* __restrict__ tab,
              const CoefX<R>* __restrict__ xtab, const int* __restrict__ items, BatchCuts cuts,
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
        run_item_gen<R, ANISO, OBST, FUSE>(in + d.off, out + d.off, d, xtab[inst], d.tb0 + d.tdn * (double)n,
                                           d.tb0 + d.tdn * (double)(n + 1), tx, m0, m1);
    }
}

// One launch of the extended model's batch: L as for call_batch, xtab the
// CoefX<R>[ninst] table in device memory (both obstacle projections share one
// instance: the choice is CoefX::proj).
template <typename R>
int call_batch_gen(const BatchLaunch& L, const void* xtab, KernelCall& k) {
    const bool obst = L.potential != MP_WELL;
    if (L.fuse == 2) {
        if (L.aniso)
            k.func = obst ? (const void*)&k_batch2d_gen<R, true, true, 2> : (const void*)&k_batch2d_gen<R, true, false, 2>;
        else
            k.func = obst ? (const void*)&k_batch2d_gen<R, false, true, 2> : (const void*)&k_batch2d_gen<R, false, false, 2>;
    } else {
        if (L.aniso)
            k.func = obst ? (const void*)&k_batch2d_gen<R, true, true, 1> : (const void*)&k_batch2d_gen<R, true, false, 1>;
        else
            k.func = obst ? (const void*)&k_batch2d_gen<R, false, true, 1> : (const void*)&k_batch2d_gen<R, false, false, 1>;
    }
    if (L.nblocks <= 0 || L.nblocks % 8 || !xtab) return MP_E_PARAM;
    k.grid = dim3((unsigned)L.nblocks);
    k.block = dim3(64 * BATCH_WPB);
    k.arg((const R*)L.in);
    k.arg((R*)L.out);
    k.arg((const InstDesc<R>*)L.table);
    k.arg((const CoefX<R>*)xtab);
    k.arg(L.items);
    k.arg(L.cuts);
    k.arg(L.stepctr);
    k.arg(L.kstep);
    return MP_OK;
}

}  // namespace mp
