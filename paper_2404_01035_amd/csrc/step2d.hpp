// 2D fused phi + mu step: one wave per column strip, no LDS, no barriers.
//
// A lane owns V consecutive cells of a row (V * sizeof(R) <= 16 bytes, so a
// lane moves one aligned vector per field; V divides nx).  A wave's 64 lanes
// cover the 64 V columns xs .. xs + 64 V - 1, xs = tx * 62 V - V: lanes 1..62
// hold the strip's 62 V cells and are the ones written; lane 0 and lane 63
// hold the columns just outside it (only lane 0's last and lane 63's first
// cell matter), so neighbouring strips overlap by 2 V columns.  The wave
// walks a segment of rows [m0, m1) of the slowest axis y, keeping the cell
// records of rows m and m+1 in registers.  Every face is evaluated once per
// wave: lane t evaluates the V x faces to the right of its cells (the last one
// with lane t+1's first cell, fetched by a lane rotate) and passes the last
// face's W, J to lane t+1; the y face (m, m+1) is kept and becomes the lower
// face of row m+1.  Out-of-range columns come from the boundary map: a lane
// lying wholly outside the grid loads the aligned vector holding its ghost
// column and, for a mirror boundary, moves that value into the slot the
// neighbouring lane reads.  Consecutive waves of a block take neighbouring
// strips; blocks are dealt XCD-aware so that a band of strips shares one
// XCD's L2.
#pragma once

#include "gp_device.hpp"

namespace mp {

template <typename R, int V>
struct Vec;
template <>
struct Vec<double, 1> {
    typedef double T;
};
template <>
struct Vec<double, 2> {
    typedef double T __attribute__((ext_vector_type(2)));
};
template <>
struct Vec<float, 1> {
    typedef float T;
};
template <>
struct Vec<float, 2> {
    typedef float T __attribute__((ext_vector_type(2)));
};
template <>
struct Vec<float, 4> {
    typedef float T __attribute__((ext_vector_type(4)));
};

template <typename R, int V>
__device__ __forceinline__ void vload(const R* p, R (&v)[V]) {
    if constexpr (V == 1) {
        v[0] = *p;
    } else {
        const typename Vec<R, V>::T t = *reinterpret_cast<const typename Vec<R, V>::T*>(p);
#pragma unroll
        for (int i = 0; i < V; ++i) v[i] = t[i];
    }
}

template <typename R, int V>
__device__ __forceinline__ void vstore(R* p, const R (&v)[V]) {
    if constexpr (V == 1) {
        *p = v[0];
    } else {
        typename Vec<R, V>::T t;
#pragma unroll
        for (int i = 0; i < V; ++i) t[i] = v[i];
        *reinterpret_cast<typename Vec<R, V>::T*>(p) = t;
    }
}

constexpr int W2D_LANES_OUT = W2D_LANES_OUT_HOST;  // written lanes per strip wave

// Raw row as loaded: the lane's V cells of every field.
template <typename R, int NF, int V>
struct Raw2d {
    R v[NF][V];
};

// Cell record of one row (cell-major); for anisotropy also the x central
// differences phi(x+1) - phi(x-1).
template <typename R, int NP, int NM, int V, bool ANISO>
struct Row2d {
    R phi[V][NP];
    R mu[V][NM];
    R Mt[V][NM];
    R cdx[ANISO ? V : 1][NP];
};

#ifndef MP_STRIP_DEPTH
#define MP_STRIP_DEPTH 2
#endif

// One wave's strip: columns tx*62V .. tx*62V + 62V - 1 (lanes 1..62), rows
// [m0, m1).  Called with wave-uniform arguments by the single-grid and the
// batched kernel.  Requires nx % V == 0.
template <typename R, int NP, int NM, bool ANISO, bool OBST, int V, int DEPTH = MP_STRIP_DEPTH>
__device__ __forceinline__ void strip2d(const R* __restrict__ in, R* __restrict__ out, const Geom& g,
                                        const Coef<R>& c, double tbase, double tslope, int tx,
                                        int m0, int m1) {
    constexpr int NF = NP + NM;
    typedef Raw2d<R, NF, V> RawT;
    typedef Row2d<R, NP, NM, V, ANISO> RowT;
    const int lane = threadIdx.x & 63;
    const bool perx = g.bcx == MP_BC_PERIODIC;
    const bool pery = g.bcy == MP_BC_PERIODIC;
    const int nx = g.nx;
    const int64_t fs = g.fstride;
    const int cs = (tx * W2D_LANES_OUT - 1 + lane) * V;  // first column of the lane
    // load column: the lane's own, or the aligned vector holding its ghost
    int col = cs;
    bool fixL = false, fixR = false;  // mirror ghosts: move the ghost value into the read slot
    if (cs < 0) {
        col = perx ? nx - V : 0;
        fixL = !perx;
    } else if (cs >= nx) {
        col = perx ? 0 : nx - V;
        fixR = !perx;
    }
    const bool writes = lane >= 1 && lane <= W2D_LANES_OUT && cs < nx;

    auto load = [&](int m, RawT& r) {
        const int64_t o = (int64_t)gmap(m, g.ny, pery) * nx + col;
#pragma unroll
        for (int f = 0; f < NF; ++f) vload<R, V>(in + f * fs + o, r.v[f]);
    };
    auto process = [&](const RawT& r, RowT& P) {
#pragma unroll
        for (int i = 0; i < V; ++i) {
#pragma unroll
            for (int a = 0; a < NP; ++a) P.phi[i][a] = r.v[a][i];
#pragma unroll
            for (int k = 0; k < NM; ++k) P.mu[i][k] = r.v[NP + k][i];
        }
        if constexpr (V > 1) {
            // a mirror ghost lane on the left is read at its last slot, one on
            // the right at its first slot
#pragma unroll
            for (int a = 0; a < NP; ++a) {
                P.phi[V - 1][a] = fixL ? P.phi[0][a] : P.phi[V - 1][a];
                P.phi[0][a] = fixR ? P.phi[V - 1][a] : P.phi[0][a];
            }
#pragma unroll
            for (int k = 0; k < NM; ++k) {
                P.mu[V - 1][k] = fixL ? P.mu[0][k] : P.mu[V - 1][k];
                P.mu[0][k] = fixR ? P.mu[V - 1][k] : P.mu[0][k];
            }
        }
#pragma unroll
        for (int i = 0; i < V; ++i) {
            R hh[NP];
            interp_h<R, NP>(P.phi[i], hh);
            mobility<R, NP, NM>(hh, c, P.Mt[i]);
        }
        if constexpr (ANISO) {
#pragma unroll
            for (int a = 0; a < NP; ++a) {
                const R left = lane_prev(P.phi[V - 1][a]);
                const R right = lane_next(P.phi[0][a]);
#pragma unroll
                for (int i = 0; i < V; ++i)
                    P.cdx[i][a] = (i + 1 < V ? P.phi[i + 1][a] : right) - (i > 0 ? P.phi[i - 1][a] : left);
            }
        }
    };

    R Wlo[V][NP], Jlo[V][NM];  // lower y faces of the current row's cells
    R prvphi[ANISO ? V : 1][NP];

    auto yface = [&](const RowT& A, const RowT& B, int i, R (&U)[NP], R (&Wf)[NP], R (&J)[NM]) {
        R tau[1][NP];
        if constexpr (ANISO) {
#pragma unroll
            for (int a = 0; a < NP; ++a) tau[0][a] = A.cdx[i][a] + B.cdx[i][a];
        }
        face_core<R, NP, NM, ANISO, 1>(A.phi[i], B.phi[i], tau, A.Mt[i], B.Mt[i], A.mu[i], B.mu[i], c,
                                       U, Wf, J);
    };

    // Row m from cur (row m) and nxt (row m+1); stores row m.
    auto row = [&](int m, const RowT& cur, const RowT& nxt) {
        R cdy[ANISO ? V : 1][NP];
        if constexpr (ANISO) {
#pragma unroll
            for (int i = 0; i < V; ++i)
#pragma unroll
                for (int a = 0; a < NP; ++a) cdy[i][a] = nxt.phi[i][a] - prvphi[i][a];
        }
        // x face to the right of the last cell, with lane t+1's first cell
        R Ur[NP], Wr[NP], Jr[NM];
        {
            R pR[NP], uR[NM], MR[NM], tau[1][NP];
#pragma unroll
            for (int a = 0; a < NP; ++a) pR[a] = lane_next(cur.phi[0][a]);
#pragma unroll
            for (int k = 0; k < NM; ++k) {
                uR[k] = lane_next(cur.mu[0][k]);
                MR[k] = lane_next(cur.Mt[0][k]);
            }
            if constexpr (ANISO) {
#pragma unroll
                for (int a = 0; a < NP; ++a) tau[0][a] = cdy[V - 1][a] + lane_next(cdy[0][a]);
            }
            face_core<R, NP, NM, ANISO, 1>(cur.phi[V - 1], pR, tau, cur.Mt[V - 1], MR, cur.mu[V - 1], uR,
                                           c, Ur, Wr, Jr);
        }
        // the face on the left of the first cell is lane t-1's last face
        R Wxl[NP], Jxl[NM];
#pragma unroll
        for (int a = 0; a < NP; ++a) Wxl[a] = lane_prev(Wr[a]);
#pragma unroll
        for (int k = 0; k < NM; ++k) Jxl[k] = lane_prev(Jr[k]);

        R Cs[NP];
        psi_const<R, NP>((R)(tbase + tslope * (double)m), c, Cs);
        R phin[NP][V], mun[NM][V];
#pragma unroll
        for (int i = 0; i < V; ++i) {
            // x face (i, i+1) inside the lane, or the right face for the last cell
            R Ux[NP], Wx[NP], Jx[NM];
            if (i + 1 < V) {
                R tau[1][NP];
                if constexpr (ANISO) {
#pragma unroll
                    for (int a = 0; a < NP; ++a) tau[0][a] = cdy[i][a] + cdy[i + 1][a];
                }
                face_core<R, NP, NM, ANISO, 1>(cur.phi[i], cur.phi[i + 1], tau, cur.Mt[i], cur.Mt[i + 1],
                                               cur.mu[i], cur.mu[i + 1], c, Ux, Wx, Jx);
            } else {
#pragma unroll
                for (int a = 0; a < NP; ++a) {
                    Ux[a] = Ur[a];
                    Wx[a] = Wr[a];
                }
#pragma unroll
                for (int k = 0; k < NM; ++k) Jx[k] = Jr[k];
            }
            // y face (m, m+1) above cell i
            R Uy[NP], Wy[NP], Jy[NM];
            yface(cur, nxt, i, Uy, Wy, Jy);
            R Gs[NP], Js[NM];
#pragma unroll
            for (int a = 0; a < NP; ++a) Gs[a] = (Ux[a] - Wxl[a]) + (Uy[a] - Wlo[i][a]);
#pragma unroll
            for (int k = 0; k < NM; ++k) Js[k] = (Jx[k] - Jxl[k]) + (Jy[k] - Jlo[i][k]);
            R pn[NP], un[NM], h0[NP];
            interp_h<R, NP>(cur.phi[i], h0);
            cell_update<R, NP, NM, OBST>(cur.phi[i], cur.mu[i], h0, Gs, Js, Cs, c, pn, un);
#pragma unroll
            for (int a = 0; a < NP; ++a) {
                phin[a][i] = pn[a];
                Wlo[i][a] = Wy[a];
                Wxl[a] = Wx[a];
            }
#pragma unroll
            for (int k = 0; k < NM; ++k) {
                mun[k][i] = un[k];
                Jlo[i][k] = Jy[k];
                Jxl[k] = Jx[k];
            }
        }
        if (writes) {
            const int64_t o = (int64_t)m * nx + cs;
#pragma unroll
            for (int a = 0; a < NP; ++a) vstore<R, V>(out + a * fs + o, phin[a]);
#pragma unroll
            for (int k = 0; k < NM; ++k) vstore<R, V>(out + (NP + k) * fs + o, mun[k]);
        }
        if constexpr (ANISO) {
#pragma unroll
            for (int i = 0; i < V; ++i)
#pragma unroll
                for (int a = 0; a < NP; ++a) prvphi[i][a] = cur.phi[i][a];
        }
    };

    // Prologue: rows m0-1, m0 and m0+1 processed.
    RowT cA, cB;
    {
        RawT r0, r1, r2;
        load(m0 - 1, r0);
        load(m0, r1);
        load(m0 + 1, r2);
        RowT prv;
        process(r0, prv);
        process(r1, cA);
#pragma unroll
        for (int i = 0; i < V; ++i) {
            R Ud[NP];
            yface(prv, cA, i, Ud, Wlo[i], Jlo[i]);
        }
        if constexpr (ANISO) {
#pragma unroll
            for (int i = 0; i < V; ++i)
#pragma unroll
                for (int a = 0; a < NP; ++a) prvphi[i][a] = prv.phi[i][a];
        }
        process(r2, cB);
    }

    // Loads and stores share one counter and may complete out of order with
    // respect to each other, so the only wait that covers a load issued before
    // a store is a wait for everything.  The loop therefore waits once per
    // DEPTH rows and issues the loads of the next DEPTH rows right after that
    // wait, giving every load DEPTH rows of arithmetic to land in; a raw row
    // is turned into a cell record just before the row that needs it.
    constexpr unsigned kWaitVm0 = 0x0F70;  // s_waitcnt vmcnt(0), expcnt/lgkmcnt untouched
    int m = m0;
    if constexpr (DEPTH == 1) {
        RawT ld;
        if (m0 + 2 <= m1) load(m0 + 2, ld);
        while (true) {
            row(m, cA, cB);
            if (++m >= m1) break;
            __builtin_amdgcn_s_waitcnt(kWaitVm0);
            process(ld, cA);
            if (m + 2 <= m1) load(m + 2, ld);
            row(m, cB, cA);
            if (++m >= m1) break;
            __builtin_amdgcn_s_waitcnt(kWaitVm0);
            process(ld, cB);
            if (m + 2 <= m1) load(m + 2, ld);
        }
    } else {
        RawT X1, X2, Y1, Y2;
        if (m0 + 2 <= m1) load(m0 + 2, X1);
        if (m0 + 3 <= m1) load(m0 + 3, X2);
        while (true) {
            __builtin_amdgcn_s_waitcnt(kWaitVm0);
            if (m + 4 <= m1) load(m + 4, Y1);
            if (m + 5 <= m1) load(m + 5, Y2);
            row(m, cA, cB);
            if (++m >= m1) break;
            process(X1, cA);
            row(m, cB, cA);
            if (++m >= m1) break;
            process(X2, cB);
            __builtin_amdgcn_s_waitcnt(kWaitVm0);
            if (m + 4 <= m1) load(m + 4, X1);
            if (m + 5 <= m1) load(m + 5, X2);
            row(m, cA, cB);
            if (++m >= m1) break;
            process(Y1, cA);
            row(m, cB, cA);
            if (++m >= m1) break;
            process(Y2, cB);
        }
    }
}

#ifndef MP_WAVES_PER_EU
#define MP_WAVES_PER_EU 2
#endif

template <typename R, int NP, int NM, bool ANISO, bool OBST, int V>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MP_WAVES_PER_EU)))
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
    strip2d<R, NP, NM, ANISO, OBST, V>(in, out, g, c, tbase, tslope, tx, m0, min(m0 + seg, g.ny));
}

template <typename R, int NP, int NM, bool ANISO, bool OBST, int V>
int call_2d_v(const StepLaunch& L, const Coef<R>& c, KernelCall& k) {
    const int ntx = (L.g.nx + W2D_LANES_OUT * V - 1) / (W2D_LANES_OUT * V);
    const int nseg = (L.g.ny + L.seg - 1) / L.seg;
    const int wpb = L.bx / 64;
    const long long waves = (long long)ntx * nseg;
    const long long nblocks = (waves + wpb - 1) / wpb;
    if (nblocks <= 0 || nblocks > 0x7fffffffLL) return MP_E_PARAM;
    k.func = (const void*)&k_step2d<R, NP, NM, ANISO, OBST, V>;
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

template <typename R, int NP, int NM, bool ANISO, bool OBST>
int call_2d(const StepLaunch& L, const Coef<R>& c, KernelCall& k) {
    const int v = vec2d_width(L.g.nx, (int)sizeof(R), L.vec);
    if (v == 1) return call_2d_v<R, NP, NM, ANISO, OBST, 1>(L, c, k);
    if (v == 2) return call_2d_v<R, NP, NM, ANISO, OBST, 2>(L, c, k);
    if constexpr (sizeof(R) == 4) {
        if (v == 4) return call_2d_v<R, NP, NM, ANISO, OBST, 4>(L, c, k);
    }
    return MP_E_PARAM;
}

}  // namespace mp
