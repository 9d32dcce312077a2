// 2D fused phi + mu step: one wave per column strip, no LDS, no barriers.
//
// A wave owns 64 consecutive columns, x0-1 .. x0+62, and writes the 62 inner
// ones (lanes 1..62); neighbouring waves overlap by two columns.  It walks a
// segment of rows (y, the slowest axis) keeping its own column's cells of
// rows m-1 (anisotropy only), m and m+1 in registers; the x neighbours come
// from the adjacent lanes through ds_bpermute.  Every face is evaluated once:
// lane t computes the x face (t, t+1) and passes its W, J to lane t+1; the y
// face (m, m+1) is kept and becomes the lower face of row m+1.  Rows are
// loaded two at a time, two rows ahead of use, with one wait per pair (see the
// row loop).  Waves are independent, so there is
// no block-level synchronisation at all; consecutive waves of a block take
// neighbouring strips, and blocks are dealt XCD-aware so that a band of strips
// shares one XCD's L2.
#pragma once

#include "gp_device.hpp"

namespace mp {

template <typename R, int NP, int NM, bool ANISO>
struct Cell2d {
    R phi[NP];
    R mu[NM];
    R Mt[NM];
    R h[NP];
    R cdx[ANISO ? NP : 1];  // phi(x+1) - phi(x-1) on this row
};

constexpr int W2D_OUT = W2D_OUT_HOST;  // columns written per wave

// One wave's strip: columns tx*62-1 .. tx*62+62 of a 2D field, rows [m0, m1).
// Called with wave-uniform arguments by the single-grid and the batched kernel.
template <typename R, int NP, int NM, bool ANISO, bool OBST>
__device__ __forceinline__ void strip2d(const R* __restrict__ in, R* __restrict__ out, const Geom& g,
                                        const Coef<R>& c, double tbase, double tslope, int tx,
                                        int m0, int m1) {
    constexpr int NF = NP + NM;
    typedef Cell2d<R, NP, NM, ANISO> CellT;
    const int lane = threadIdx.x & 63;
    const int gx = tx * W2D_OUT - 1 + lane;
    const bool perx = g.bcx == MP_BC_PERIODIC;
    const bool pery = g.bcy == MP_BC_PERIODIC;
    const int col = gmap(gx, g.nx, perx);
    const int64_t fs = g.fstride;
    const int64_t nx = g.nx;
    const int aR = ((lane + 1) & 63) << 2;
    const int aL = ((lane + 63) & 63) << 2;
    const bool writes = lane >= 1 && lane <= W2D_OUT && gx < g.nx;

    auto load = [&](int m, R (&v)[NF]) {
        const int64_t o = (int64_t)gmap(m, g.ny, pery) * nx + col;
#pragma unroll
        for (int f = 0; f < NF; ++f) v[f] = in[f * fs + o];
    };
    auto process = [&](const R (&v)[NF], CellT& P) {
#pragma unroll
        for (int a = 0; a < NP; ++a) P.phi[a] = v[a];
#pragma unroll
        for (int k = 0; k < NM; ++k) P.mu[k] = v[NP + k];
        interp_h<R, NP>(P.phi, P.h);
        mobility<R, NP, NM>(P.h, c, P.Mt);
        if constexpr (ANISO) {
#pragma unroll
            for (int a = 0; a < NP; ++a) P.cdx[a] = lane_get(P.phi[a], aR) - lane_get(P.phi[a], aL);
        }
    };
    R Wlo0[NP], Jlo0[NM], Wlo1[NP], Jlo1[NM];  // lower y faces, alternating per row
    auto yface = [&](const CellT& A, const CellT& B, R (&U)[NP], R (&Wf)[NP], R (&J)[NM]) {
        R tau[1][NP];
        if constexpr (ANISO) {
#pragma unroll
            for (int a = 0; a < NP; ++a) tau[0][a] = A.cdx[a] + B.cdx[a];
        }
        face_core<R, NP, NM, ANISO, 1>(A.phi, B.phi, tau, A.Mt, B.Mt, A.mu, B.mu, c, U, Wf, J);
    };

    // Prologue: rows m0-1, m0, m0+1 processed, rows m0+2 and m0+3 in flight.
    R v0[NF], v1[NF], v2[NF], ldA[NF], ldB[NF], ldC[NF], ldD[NF];
    load(m0 - 1, v0);
    load(m0, v1);
    load(m0 + 1, v2);
    if (m0 + 2 <= m1) load(m0 + 2, ldA);
    if (m0 + 3 <= m1) load(m0 + 3, ldB);
    CellT cA, cB;
    R prvphi[ANISO ? NP : 1];
    {
        CellT prv;
        process(v0, prv);
        process(v1, cA);
        process(v2, cB);
        if constexpr (ANISO) {
#pragma unroll
            for (int a = 0; a < NP; ++a) prvphi[a] = prv.phi[a];
        }
        R Ud[NP];
        yface(prv, cA, Ud, Wlo0, Jlo0);
    }

    // One row.  On entry cur = row m, nxt = row m+1 and ldX holds the raw row
    // m+2; the call ends by turning ldX into the cell record of row m+2 in
    // cur's storage, so the next row is computed with the roles swapped.
    auto row = [&](int m, CellT& cur, CellT& nxt, const R (&ldX)[NF], const R (&Wlo)[NP],
                   const R (&Jlo)[NM], R (&Wy)[NP], R (&Jy)[NM]) {
        // x face (t, t+1) on row m
        R pR[NP], uR[NM], MR[NM];
#pragma unroll
        for (int a = 0; a < NP; ++a) pR[a] = lane_get(cur.phi[a], aR);
#pragma unroll
        for (int k = 0; k < NM; ++k) {
            uR[k] = lane_get(cur.mu[k], aR);
            MR[k] = lane_get(cur.Mt[k], aR);
        }
        R taux[1][NP];
        if constexpr (ANISO) {
#pragma unroll
            for (int a = 0; a < NP; ++a) {
                R cdy = nxt.phi[a] - prvphi[a];
                taux[0][a] = cdy + lane_get(cdy, aR);
            }
        }
        R Ux[NP], Wx[NP], Jx[NM];
        face_core<R, NP, NM, ANISO, 1>(cur.phi, pR, taux, cur.Mt, MR, cur.mu, uR, c, Ux, Wx, Jx);
        R Wxl[NP], Jxl[NM];  // face (t-1, t), computed by the lane on the left
#pragma unroll
        for (int a = 0; a < NP; ++a) Wxl[a] = lane_get(Wx[a], aL);
#pragma unroll
        for (int k = 0; k < NM; ++k) Jxl[k] = lane_get(Jx[k], aL);

        // y face (m, m+1)
        R Uy[NP];
        yface(cur, nxt, Uy, Wy, Jy);

        R Gs[NP], Js[NM];
#pragma unroll
        for (int a = 0; a < NP; ++a) Gs[a] = (Ux[a] - Wxl[a]) + (Uy[a] - Wlo[a]);
#pragma unroll
        for (int k = 0; k < NM; ++k) Js[k] = (Jx[k] - Jxl[k]) + (Jy[k] - Jlo[k]);

        const R tt = (R)(tbase + tslope * (double)m);
        R phin[NP], mun[NM];
        cell_update<R, NP, NM, OBST>(cur.phi, cur.mu, cur.h, Gs, Js, tt, c, phin, mun);
        if (writes) {
            const int64_t o = (int64_t)m * nx + gx;
#pragma unroll
            for (int a = 0; a < NP; ++a) out[a * fs + o] = phin[a];
#pragma unroll
            for (int k = 0; k < NM; ++k) out[(NP + k) * fs + o] = mun[k];
        }

        if constexpr (ANISO) {
#pragma unroll
            for (int a = 0; a < NP; ++a) prvphi[a] = cur.phi[a];
        }
        if (m + 2 <= m1) process(ldX, cur);
    };

    // Rows go in pairs.  Before a pair, one explicit wait drains every
    // outstanding access (the two raw rows the pair consumes, and earlier
    // stores); the loads of the next pair's rows are issued right after it, so
    // each load has two rows of arithmetic to land in.  Waiting any finer would
    // not help: with loads and stores both pending the counter completes out of
    // order and any wait on a load becomes a wait for zero.
    constexpr unsigned kWaitVm0 = 0x0F70;  // s_waitcnt vmcnt(0), expcnt/lgkmcnt untouched
    int m = m0;
    while (true) {
        __builtin_amdgcn_s_waitcnt(kWaitVm0);
        if (m + 4 <= m1) load(m + 4, ldC);
        if (m + 5 <= m1) load(m + 5, ldD);
        if (m >= m1) break;
        row(m, cA, cB, ldA, Wlo0, Jlo0, Wlo1, Jlo1);
        if (m + 1 >= m1) break;
        row(m + 1, cB, cA, ldB, Wlo1, Jlo1, Wlo0, Jlo0);
        m += 2;
        __builtin_amdgcn_s_waitcnt(kWaitVm0);
        if (m + 4 <= m1) load(m + 4, ldA);
        if (m + 5 <= m1) load(m + 5, ldB);
        if (m >= m1) break;
        row(m, cA, cB, ldC, Wlo0, Jlo0, Wlo1, Jlo1);
        if (m + 1 >= m1) break;
        row(m + 1, cB, cA, ldD, Wlo1, Jlo1, Wlo0, Jlo0);
        m += 2;
    }
}

template <typename R, int NP, int NM, bool ANISO, bool OBST>
__global__ void __launch_bounds__(256)
k_step2d(const R* __restrict__ in, R* __restrict__ out, Geom g, Coef<R> c,
         const int64_t* __restrict__ stepctr, int kstep, double tb0, double tdn, double tslope,
         int seg, int ntx, int nseg) {
    const int wpb = blockDim.x >> 6;
    const int nb = gridDim.x;
    const int q8 = nb / 8;
    const int b = blockIdx.x;
    const int blk = (b < 8 * q8) ? (b % 8) * q8 + b / 8 : b;
    // wave-uniform by construction; readfirstlane tells the compiler so, which
    // keeps every row-loop branch scalar
    const int wid = __builtin_amdgcn_readfirstlane(blk * wpb + (threadIdx.x >> 6));
    if (wid >= ntx * nseg) return;  // whole wave leaves; nothing below synchronises
    const int tx = wid % ntx;
    const int sg = wid / ntx;
    const int m0 = sg * seg;
    const double tbase = tb0 + tdn * (double)(*stepctr + kstep);
    strip2d<R, NP, NM, ANISO, OBST>(in, out, g, c, tbase, tslope, tx, m0, min(m0 + seg, g.ny));
}

template <typename R, int NP, int NM, bool ANISO, bool OBST>
int call_2d(const StepLaunch& L, const Coef<R>& c, KernelCall& k) {
    const int ntx = (L.g.nx + W2D_OUT - 1) / W2D_OUT;
    const int nseg = (L.g.ny + L.seg - 1) / L.seg;
    const int wpb = L.bx / 64;
    const long long waves = (long long)ntx * nseg;
    const long long nblocks = (waves + wpb - 1) / wpb;
    if (nblocks <= 0 || nblocks > 0x7fffffffLL) return MP_E_PARAM;
    k.func = (const void*)&k_step2d<R, NP, NM, ANISO, OBST>;
    k.grid = dim3((unsigned)nblocks);
    k.block = dim3(L.bx);
    k.arg((const R*)L.in);
    k.arg((R*)L.out);
    k.arg(L.g);
    k.arg(c);
    k.arg(L.stepctr);
    k.arg(L.kstep);
    k.arg(L.tb0);
    k.arg(L.tdn);
    k.arg(L.tslope);
    k.arg(L.seg);
    k.arg(ntx);
    k.arg(nseg);
    return MP_OK;
}

}  // namespace mp
