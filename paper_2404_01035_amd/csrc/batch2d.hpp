// Batched 2D step: many independent simulations in one persistent launch.
//
// The work list holds one item per (instance, column strip, row segment),
// strips W2X_LANES_OUT lanes wide for both the one-step and the two-step
// variant (so the list does not depend on the steps per launch), as
// (instance, local index) pairs; the instance table (InstDesc) carries each
// instance's grid, sizes, coefficients, state offset and temperature law.
// The grid is sized to what stays resident; the waves of XCD x walk their
// slice cuts[x] .. cuts[x+1]-1 of the list with a fixed stride.  The host
// deals whole instances to the slices by cost (a strip's neighbours share an
// L2) and orders each slice so that the waves' shares are even.  Each item
// runs the same strip function as the single-grid kernel, so a batched
// instance is stepped bit for bit like a single one, in any order.
#pragma once

#include "step2d.hpp"

namespace mp {

constexpr int BATCH_WPB = BATCH_WPB_HOST;  // waves per block

constexpr int BATCH_W = W2X_LANES_OUT;  // written lanes per batched strip

// One item with V cells per lane and FUSE (1 or 2) steps.
template <typename R, int NP, int NM, bool ANISO, bool OBST, int V, int FUSE>
__device__ __forceinline__ void run_strip(const R* src, R* dst, const InstDesc<R>& d, double tb0,
                                          double tb1, int tx, int m0, int m1) {
    if constexpr (FUSE == 2)
        strip2d_x2<R, NP, NM, ANISO, OBST, V, true>(src, dst, nullptr, d.g, d.c, tb0, tb1, d.tslope, tx, m0,
                                                    m1);
    else
        strip2d<R, NP, NM, ANISO, OBST, V, MP_STRIP_DEPTH, BATCH_W>(src, dst, d.g, d.c, tb0, d.tslope,
                                                                    tx, m0, m1);
}

// Cells per lane of a batched item: 1, or up to VMAX = 2 where nx is even.
// Every variant is inlined into the one kernel, whose register budget is that
// of the widest, so the kernel is instantiated per VMAX.
template <typename R, int NP, int NM, bool ANISO, bool OBST, int VMAX, int FUSE>
__device__ __forceinline__ void run_vec(const R* src, R* dst, const InstDesc<R>& d, double tb0,
                                        double tb1, int tx, int m0, int m1) {
    if (VMAX == 1 || d.vec == 1)
        run_strip<R, NP, NM, ANISO, OBST, 1, FUSE>(src, dst, d, tb0, tb1, tx, m0, m1);
    else
        run_strip<R, NP, NM, ANISO, OBST, 2, FUSE>(src, dst, d, tb0, tb1, tx, m0, m1);
}

template <typename R, bool ANISO, bool OBST, int VMAX, int FUSE>
__device__ __forceinline__ void run_item(const R* src, R* dst, const InstDesc<R>& d, double tb0,
                                         double tb1, int tx, int m0, int m1) {
    switch (d.np * 4 + d.nm) {
        case 2 * 4 + 1:
            run_vec<R, 2, 1, ANISO, OBST, VMAX, FUSE>(src, dst, d, tb0, tb1, tx, m0, m1);
            break;
        case 2 * 4 + 2:
            run_vec<R, 2, 2, ANISO, OBST, VMAX, FUSE>(src, dst, d, tb0, tb1, tx, m0, m1);
            break;
        case 3 * 4 + 1:
            run_vec<R, 3, 1, ANISO, OBST, VMAX, FUSE>(src, dst, d, tb0, tb1, tx, m0, m1);
            break;
        default:
            run_vec<R, 3, 2, ANISO, OBST, VMAX, FUSE>(src, dst, d, tb0, tb1, tx, m0, m1);
            break;
    }
}

template <typename R, bool ANISO, bool OBST, int VMAX, int FUSE>
__global__ void __launch_bounds__(64 * BATCH_WPB) __attribute__((amdgpu_waves_per_eu(2)))
k_batch2d(const R* __restrict__ in, R* __restrict__ out, const InstDesc<R>* __restrict__ tab,
          const int* __restrict__ items, BatchCuts cuts, const int64_t* __restrict__ stepctr, int kstep) {
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
        const R* src = in + d.off;
        R* dst = out + d.off;
        run_item<R, ANISO, OBST, VMAX, FUSE>(src, dst, d, d.tb0 + d.tdn * (double)n,
                                             d.tb0 + d.tdn * (double)(n + 1), tx, m0, m1);
    }
}

template <typename R, int VMAX, int FUSE>
const void* batch_func(bool aniso, bool obst) {
    if (aniso)
        return obst ? (const void*)&k_batch2d<R, true, true, VMAX, FUSE>
                    : (const void*)&k_batch2d<R, true, false, VMAX, FUSE>;
    return obst ? (const void*)&k_batch2d<R, false, true, VMAX, FUSE>
                : (const void*)&k_batch2d<R, false, false, VMAX, FUSE>;
}

template <typename R>
int call_batch(const BatchLaunch& L, KernelCall& k) {
    const bool obst = L.potential == MP_OBSTACLE;
    if (L.fuse == 2)
        k.func = L.vmax == 1 ? batch_func<R, 1, 2>(L.aniso, obst) : batch_func<R, 2, 2>(L.aniso, obst);
    else
        k.func = L.vmax == 1 ? batch_func<R, 1, 1>(L.aniso, obst) : batch_func<R, 2, 1>(L.aniso, obst);
    if (L.nblocks <= 0 || L.nblocks % 8) return MP_E_PARAM;
    k.grid = dim3((unsigned)L.nblocks);
    k.block = dim3(64 * BATCH_WPB);
    k.arg((const R*)L.in);
    k.arg((R*)L.out);
    k.arg((const InstDesc<R>*)L.table);
    k.arg(L.items);
    k.arg(L.cuts);
    k.arg(L.stepctr);
    k.arg(L.kstep);
    return MP_OK;
}

}  // namespace mp
