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

#include "diag_cell.hpp"
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
constexpr int W2X_LANES_OUT = W2X_LANES_OUT_HOST;  // written lanes per two-step strip wave

// Raw row as loaded: the lane's V cells of every field.
template <typename R, int NF, int V>
struct Raw2d {
    R v[NF][V];
};

// Cell record of one row (cell-major); for anisotropy also the x central
// differences phi(x+1) - phi(x-1).  GEN: the mobility is a matrix.
template <typename R, int NP, int NM, int V, bool ANISO, bool GEN = false>
struct Row2d {
    R phi[V][NP];
    R mu[V][NM];
    R Mt[V][mob_n<NM, GEN>()];
    R cdx[ANISO ? V : 1][NP];
};

// What one pass over the rows carries from a row to the next: the W, J of the
// y faces below the current row's cells and (anisotropy) phi of the row below;
// in a pass from the top down, the U, J of the faces above and phi of the row
// above.
template <typename R, int NP, int NM, int V, bool ANISO>
struct Carry2d {
    R Wlo[V][NP];
    R Jlo[V][NM];
    R prvphi[ANISO ? V : 1][NP];
};

// Cell record from the V values of every field (field-major, as loaded).
// HAVE_H: hv holds h(phi) of the cells already.
template <typename R, int NP, int NM, bool ANISO, int V, bool HAVE_H = false, bool GEN = false>
__device__ __forceinline__ void make_row(const R (&v)[NP + NM][V], Row2d<R, NP, NM, V, ANISO, GEN>& P,
                                         const Coef<R>& c, const R (*hv)[V] = nullptr,
                                         const CoefX<R>* x = nullptr) {
#pragma unroll
    for (int i = 0; i < V; ++i) {
#pragma unroll
        for (int a = 0; a < NP; ++a) P.phi[i][a] = v[a][i];
#pragma unroll
        for (int k = 0; k < NM; ++k) P.mu[i][k] = v[NP + k][i];
        R hh[NP];
        if constexpr (HAVE_H) {
#pragma unroll
            for (int a = 0; a < NP; ++a) hh[a] = hv[a][i];
        } else {
            interp_h<R, NP>(P.phi[i], hh);
        }
        mobility_any<R, NP, NM, GEN>(hh, c, x, P.Mt[i]);
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
}

// y face between rows A (below) and B (above) at slot i.
template <typename R, int NP, int NM, bool ANISO, int V, bool GEN = false>
__device__ __forceinline__ void yface(const Row2d<R, NP, NM, V, ANISO, GEN>& A,
                                      const Row2d<R, NP, NM, V, ANISO, GEN>& B, int i, const Coef<R>& c,
                                      R (&U)[NP], R (&Wf)[NP], R (&J)[NM]) {
    R tau[1][NP];
    if constexpr (ANISO) {
#pragma unroll
        for (int a = 0; a < NP; ++a) tau[0][a] = A.cdx[i][a] + B.cdx[i][a];
    }
    face_core<R, NP, NM, ANISO, 1, GEN>(A.phi[i], B.phi[i], tau, A.Mt[i], B.Mt[i], A.mu[i], B.mu[i], c, U, Wf,
                                        J);
}

// Carry of the first row of a pass, from the row before it in the pass (below
// it, or above it when DOWN).
template <typename R, int NP, int NM, bool ANISO, int V, bool GEN = false, bool DOWN = false>
__device__ __forceinline__ void carry_init(const Row2d<R, NP, NM, V, ANISO, GEN>& prv,
                                           const Row2d<R, NP, NM, V, ANISO, GEN>& cur,
                                           Carry2d<R, NP, NM, V, ANISO>& k, const Coef<R>& c) {
#pragma unroll
    for (int i = 0; i < V; ++i) {
        R Ud[NP];
        if constexpr (DOWN)
            yface<R, NP, NM, ANISO, V, GEN>(cur, prv, i, c, k.Wlo[i], Ud, k.Jlo[i]);
        else
            yface<R, NP, NM, ANISO, V, GEN>(prv, cur, i, c, Ud, k.Wlo[i], k.Jlo[i]);
    }
    if constexpr (ANISO) {
#pragma unroll
        for (int i = 0; i < V; ++i)
#pragma unroll
            for (int a = 0; a < NP; ++a) k.prvphi[i][a] = prv.phi[i][a];
    }
}

// New values of the row `cur` (nxt is the next row of the pass: the row above,
// or the row below when DOWN) and the carry moved on one row.  Cs = psi_const
// of the row, tt its T - Te; hn receives h of the new phi.
template <typename R, int NP, int NM, bool ANISO, bool OBST, int V, bool GEN = false, bool DOWN = false>
__device__ __forceinline__ void row_update(const Row2d<R, NP, NM, V, ANISO, GEN>& cur,
                                           const Row2d<R, NP, NM, V, ANISO, GEN>& nxt,
                                           Carry2d<R, NP, NM, V, ANISO>& k, const R (&Cs)[NP],
                                           const Coef<R>& c, R (&phin)[NP][V], R (&mun)[NM][V],
                                           R (&hn)[NP][V], R tt = R(0), const CoefX<R>* x = nullptr) {
    constexpr int NMM = mob_n<NM, GEN>();
    R cdy[ANISO ? V : 1][NP];
    if constexpr (ANISO) {
#pragma unroll
        for (int i = 0; i < V; ++i)
#pragma unroll
            for (int a = 0; a < NP; ++a)
                cdy[i][a] = DOWN ? k.prvphi[i][a] - nxt.phi[i][a] : nxt.phi[i][a] - k.prvphi[i][a];
    }
    // x face to the right of the last cell, with the next lane's first cell
    R Ur[NP], Wr[NP], Jr[NM];
    {
        R pR[NP], uR[NM], MR[NMM], tau[1][NP];
#pragma unroll
        for (int a = 0; a < NP; ++a) pR[a] = lane_next(cur.phi[0][a]);
#pragma unroll
        for (int kk = 0; kk < NM; ++kk) uR[kk] = lane_next(cur.mu[0][kk]);
#pragma unroll
        for (int kk = 0; kk < NMM; ++kk) MR[kk] = lane_next(cur.Mt[0][kk]);
        if constexpr (ANISO) {
#pragma unroll
            for (int a = 0; a < NP; ++a) tau[0][a] = cdy[V - 1][a] + lane_next(cdy[0][a]);
        }
        face_core<R, NP, NM, ANISO, 1, GEN>(cur.phi[V - 1], pR, tau, cur.Mt[V - 1], MR, cur.mu[V - 1], uR,
                                            c, Ur, Wr, Jr);
    }
    // the face on the left of the first cell is the previous lane's last face
    R Wxl[NP], Jxl[NM];
#pragma unroll
    for (int a = 0; a < NP; ++a) Wxl[a] = lane_prev(Wr[a]);
#pragma unroll
    for (int kk = 0; kk < NM; ++kk) Jxl[kk] = lane_prev(Jr[kk]);

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
            face_core<R, NP, NM, ANISO, 1, GEN>(cur.phi[i], cur.phi[i + 1], tau, cur.Mt[i], cur.Mt[i + 1],
                                                cur.mu[i], cur.mu[i + 1], c, Ux, Wx, Jx);
        } else {
#pragma unroll
            for (int a = 0; a < NP; ++a) {
                Ux[a] = Ur[a];
                Wx[a] = Wr[a];
            }
#pragma unroll
            for (int kk = 0; kk < NM; ++kk) Jx[kk] = Jr[kk];
        }
        // y face (m, m+1) above cell i
        R Uy[NP], Wy[NP], Jy[NM];
        if constexpr (DOWN)
            yface<R, NP, NM, ANISO, V, GEN>(nxt, cur, i, c, Uy, Wy, Jy);
        else
            yface<R, NP, NM, ANISO, V, GEN>(cur, nxt, i, c, Uy, Wy, Jy);
        R Gs[NP], Js[NM];
#pragma unroll
        for (int a = 0; a < NP; ++a)
            Gs[a] = (Ux[a] - Wxl[a]) + (DOWN ? k.Wlo[i][a] - Wy[a] : Uy[a] - k.Wlo[i][a]);
#pragma unroll
        for (int kk = 0; kk < NM; ++kk)
            Js[kk] = (Jx[kk] - Jxl[kk]) + (DOWN ? k.Jlo[i][kk] - Jy[kk] : Jy[kk] - k.Jlo[i][kk]);
        R pn[NP], un[NM], h0[NP], h1[NP];
        interp_h<R, NP>(cur.phi[i], h0);
        cell_update_any<R, NP, NM, OBST, GEN>(cur.phi[i], cur.mu[i], h0, Gs, Js, Cs, tt, c, x, pn, un, h1);
#pragma unroll
        for (int a = 0; a < NP; ++a) {
            phin[a][i] = pn[a];
            hn[a][i] = h1[a];
            k.Wlo[i][a] = DOWN ? Uy[a] : Wy[a];
            Wxl[a] = Wx[a];
        }
#pragma unroll
        for (int kk = 0; kk < NM; ++kk) {
            mun[kk][i] = un[kk];
            k.Jlo[i][kk] = Jy[kk];
            Jxl[kk] = Jx[kk];
        }
    }
    if constexpr (ANISO) {
#pragma unroll
        for (int i = 0; i < V; ++i)
#pragma unroll
            for (int a = 0; a < NP; ++a) k.prvphi[i][a] = cur.phi[i][a];
    }
}

// Mirror ghost lane: move its ghost value into the slot the neighbour reads
// (the last slot for a lane left of the grid, the first for one right of it).
template <typename R, int NF, int V>
__device__ __forceinline__ void mirror_fix(R (&v)[NF][V], bool fixL, bool fixR) {
    if constexpr (V > 1) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            v[f][V - 1] = fixL ? v[f][0] : v[f][V - 1];
            v[f][0] = fixR ? v[f][V - 1] : v[f][0];
        }
    }
}

#ifndef MP_STRIP_DEPTH
#define MP_STRIP_DEPTH 2
#endif

// Diagnostics of one stored row record (V cells of a lane), in FP64; TDEP:
// B^a depends on T (the extended model).
template <typename R, int NP, int NM, int V, bool TDEP>
__device__ __forceinline__ void diag_row(const R (&phin)[NP][V], const R (&mun)[NM][V], double tt,
                                         const DiagCoef& dc, DiagStrip<NP, NM, TDEP>& A) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
        double p[NP], u[NM];
#pragma unroll
        for (int a = 0; a < NP; ++a) p[a] = (double)phin[a][v];
#pragma unroll
        for (int k = 0; k < NM; ++k) u[k] = (double)mun[k][v];
        A.cell(p, u, tt, dc);
    }
}

constexpr unsigned kWaitVm0 = 0x0F70;  // s_waitcnt vmcnt(0), expcnt/lgkmcnt untouched

// One wave's strip of one step: columns tx*W*V .. (tx+1)*W*V - 1 (lanes
// 1..W, W <= 62), rows [m0, m1).  Called with wave-uniform arguments by the
// single-grid and the batched kernel.  Requires nx % V == 0.
template <typename R, int NP, int NM, bool ANISO, bool OBST, int V, int DEPTH = MP_STRIP_DEPTH,
          int W = W2D_LANES_OUT, bool GEN = false, bool DIAG = false>
__device__ __forceinline__ void strip2d(const R* __restrict__ in, R* __restrict__ out, const Geom& g,
                                        const Coef<R>& c, double tbase, double tslope, int tx,
                                        int m0, int m1, const CoefX<R>* x = nullptr,
                                        DiagStrip<NP, NM, GEN>* da = nullptr, const DiagCoef* dc = nullptr) {
    constexpr int NF = NP + NM;
    typedef Raw2d<R, NF, V> RawT;
    typedef Row2d<R, NP, NM, V, ANISO, GEN> RowT;
    const int lane = threadIdx.x & 63;
    const bool perx = g.bcx == MP_BC_PERIODIC;
    const bool pery = g.bcy == MP_BC_PERIODIC;
    const int nx = g.nx;
    const int64_t fs = g.fstride;
    static_assert(W >= 1 && W <= 62, "strip width");
    const int cs = (tx * W - 1 + lane) * V;  // first column of the lane
    // load column: the lane's own, or the aligned vector holding its ghost
    int col = cs;
    bool fixL = false, fixR = false;
    if (cs < 0) {
        col = perx ? nx - V : 0;
        fixL = !perx;
    } else if (cs >= nx) {
        col = perx ? 0 : nx - V;
        fixR = !perx;
    }
    const bool writes = lane >= 1 && lane <= W && cs < nx;

    auto load = [&](int m, RawT& r) {
        const int64_t o = (int64_t)gmap(m, g.ny, pery) * nx + col;
#pragma unroll
        for (int f = 0; f < NF; ++f) vload<R, V>(in + f * fs + o, r.v[f]);
    };
    auto process = [&](RawT& r, RowT& P) {
        mirror_fix<R, NF, V>(r.v, fixL, fixR);
        make_row<R, NP, NM, ANISO, V, false, GEN>(r.v, P, c, nullptr, x);
    };
    Carry2d<R, NP, NM, V, ANISO> k;
    auto row = [&](int m, const RowT& cur, const RowT& nxt) {
        R Cs[NP];
        const R tt = (R)(tbase + tslope * (double)m);
        psi_const_any<R, NP, GEN>(tt, c, x, Cs);
        R phin[NP][V], mun[NM][V], hn[NP][V];
        row_update<R, NP, NM, ANISO, OBST, V, GEN>(cur, nxt, k, Cs, c, phin, mun, hn, tt, x);
        if (writes) {
            const int64_t o = (int64_t)m * nx + cs;
#pragma unroll
            for (int a = 0; a < NP; ++a) vstore<R, V>(out + a * fs + o, phin[a]);
#pragma unroll
            for (int kk = 0; kk < NM; ++kk) vstore<R, V>(out + (NP + kk) * fs + o, mun[kk]);
            if constexpr (DIAG) diag_row<R, NP, NM, V, GEN>(phin, mun, dc->tt0 + dc->tslope * (double)m, *dc, *da);
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
        carry_init<R, NP, NM, ANISO, V, GEN>(prv, cA, k, c);
        process(r2, cB);
    }

    // Loads and stores share one counter and may complete out of order with
    // respect to each other, so the only wait that covers a load issued before
    // a store is a wait for everything.  The loop therefore waits once per
    // DEPTH rows and issues the loads of the next DEPTH rows right after that
    // wait, giving every load DEPTH rows of arithmetic to land in; a raw row
    // is turned into a cell record just before the row that needs it.
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

// Two steps in one pass.  A wave's lanes cover xs .. xs + 64 V - 1 with
// xs = tx * 60 V - 2 V; lanes 2..61 are written.  Step 1 is computed on every
// lane into registers (a row at a time, marching y as in strip2d) and step 2
// from those rows, so the state is read and written once per two steps.
// Step 1 must see exactly the ghosts a stored state would: a periodic ghost
// row or column is computed from its wrapped neighbours (the same operands in
// the same order as where it lives, so the same bits); a mirror ghost is an
// exact copy of the cell it mirrors (made by a lane shuffle in x and by
// reusing the row record in y), so a boundary face sees two identical cells
// and carries nothing, as in the one-step kernel.  The output rows [m0, m1)
// need step-1 rows m0-1 .. m1 and state rows m0-2 .. m1+1.
// Column loaded by a lane of a two-step strip wave whose first column is cs,
// and whether the lane holds a mirror ghost column (fixL: ghost -1 in its
// last slot, fixR: ghost nx in its first slot).
template <int V>
__device__ __forceinline__ int x2_column(const Geom& g, int cs, bool& fixL, bool& fixR) {
    const int nx = g.nx;
    fixL = fixR = false;
    if (g.bcx == MP_BC_PERIODIC) return wrap(cs, nx);
    if (cs >= 0 && cs < nx) return cs;
    if (cs == -V) {
        fixL = true;  // holds ghost column -1 = column 0 in its last slot
        return 0;
    }
    if (cs == nx) {
        fixR = true;  // holds ghost column nx = column nx-1 in its first slot
        return nx - V;
    }
    return cs < 0 ? 0 : nx - V;  // farther out: never read by a written lane
}

// First column of a lane of two-step strip wave tx.
template <int V>
__device__ __forceinline__ int x2_first_col(int tx, int lane) {
    return (tx * W2X_LANES_OUT - 2 + lane) * V;
}

// XEDGE: the wave holds a mirror ghost column (wave-uniform; only then are
// the mirror copies of step 1 made).  STORE1: the step-1 rows of the segment
// are also written, to out1 (the state between the two steps).  DOWN: the
// rows are visited from the top of the segment down (the y face below a row
// is formed there and its lower-cell part carried to the next row).
template <typename R, int NP, int NM, bool ANISO, bool OBST, int V, bool XEDGE, bool STORE1 = false,
          bool GEN = false, bool DIAG = false, bool DOWN = false>
__device__ __forceinline__ void strip2d_x2(const R* __restrict__ in, R* __restrict__ out, R* __restrict__ out1,
                                           const Geom& g, const Coef<R>& c, double tbase0, double tbase1,
                                           double tslope, int tx, int m0, int m1, const CoefX<R>* x = nullptr,
                                           DiagStrip<NP, NM, GEN>* da = nullptr, const DiagCoef* dc = nullptr) {
    constexpr int NF = NP + NM;
    typedef Raw2d<R, NF, V> RawT;
    typedef Row2d<R, NP, NM, V, ANISO, GEN> RowT;
    const int lane = threadIdx.x & 63;
    const bool pery = g.bcy == MP_BC_PERIODIC;
    const int nx = g.nx, ny = g.ny;
    const int64_t fs = g.fstride;
    const int cs = x2_first_col<V>(tx, lane);
    bool fixL, fixR;
    const int col = x2_column<V>(g, cs, fixL, fixR);
    const bool writes = lane >= 2 && lane <= W2X_LANES_OUT + 1 && cs < nx;
    const bool top = !pery && m0 == 0;   // step-1 row -1 is a copy of row 0
    const bool bot = !pery && m1 == ny;  // step-1 row ny is a copy of row ny-1
    // step-1 rows computed: (top ? 0 : m0 - 1) .. (bot ? ny - 1 : m1), from the
    // bottom up, or from the top down (DOWN)
    constexpr int dir = DOWN ? -1 : 1;
    const bool first_edge = DOWN ? bot : top;  // the start row's outer neighbour is the row itself
    const int r_first = DOWN ? (bot ? ny - 1 : m1) : (top ? 0 : m0 - 1);

    auto rowmap = [&](int s) { return pery ? wrap(s, ny) : gmap(s, ny, false); };
    auto load = [&](int s, RawT& r) {
        const int64_t o = (int64_t)rowmap(s) * nx + col;
#pragma unroll
        for (int f = 0; f < NF; ++f) vload<R, V>(in + f * fs + o, r.v[f]);
    };
    auto process = [&](RawT& r, RowT& P) {
        if constexpr (XEDGE) mirror_fix<R, NF, V>(r.v, fixL, fixR);
        make_row<R, NP, NM, ANISO, V, false, GEN>(r.v, P, c, nullptr, x);
    };

    // step 0 -> 1: rows of the state in c0 (row r) and n0 (row r+1)
    Carry2d<R, NP, NM, V, ANISO> k0, k1;
    RowT c0, n0;
    RawT ld;
    {
        RawT a, b, d;
        load(r_first - dir, a);
        load(r_first, b);
        load(r_first + dir, d);
        RowT prv;
        process(a, prv);
        process(b, c0);
        carry_init<R, NP, NM, ANISO, V, GEN, DOWN>(prv, c0, k0, c);
        process(d, n0);
    }
    load(r_first + 2 * dir, ld);

    // Step-1 row r into P, then the state window moves on one row.  The
    // window always moves (past the last row needed it reads clamped rows that
    // go unused), so that the row loop below has a single path and the rows in
    // flight stay in the registers they are loaded into.
    auto step1 = [&](int r, RowT& P) {
        R Cs[NP];
        const R tt = (R)(tbase0 + tslope * (double)rowmap(r));
        psi_const_any<R, NP, GEN>(tt, c, x, Cs);
        R phin[NP][V], mun[NM][V], hn[NP][V];
        row_update<R, NP, NM, ANISO, OBST, V, GEN, DOWN>(c0, n0, k0, Cs, c, phin, mun, hn, tt, x);
        R v[NF][V];
#pragma unroll
        for (int i = 0; i < V; ++i) {
#pragma unroll
            for (int a = 0; a < NP; ++a) v[a][i] = phin[a][i];
#pragma unroll
            for (int kk = 0; kk < NM; ++kk) v[NP + kk][i] = mun[kk][i];
        }
        // mirror ghost columns of step 1: copies of the cells they mirror
        // (only the waves at a no-flux x edge hold such a column; elsewhere
        // the record takes h of the new phi from the update)
        if constexpr (XEDGE) {
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const R nextFirst = lane_next(v[f][0]);
                const R prevLast = lane_prev(v[f][V - 1]);
                v[f][V - 1] = fixL ? nextFirst : v[f][V - 1];
                v[f][0] = fixR ? prevLast : v[f][0];
            }
            make_row<R, NP, NM, ANISO, V, false, GEN>(v, P, c, nullptr, x);
        } else {
            make_row<R, NP, NM, ANISO, V, true, GEN>(v, P, c, hn, x);
        }
        if constexpr (STORE1) {
            if (writes && r >= m0 && r < m1) {
                const int64_t o = (int64_t)r * nx + cs;
#pragma unroll
                for (int f = 0; f < NF; ++f) vstore<R, V>(out1 + f * fs + o, v[f]);
            }
        }
        c0 = n0;
        __builtin_amdgcn_s_waitcnt(kWaitVm0);
        process(ld, n0);
        load(r + 3 * dir, ld);
    };

    // step 1 -> 2: step-1 rows in c1 (row q) and n1 (row q+1)
    RowT c1, n1;
    {
        RowT outer;
        step1(r_first, outer);
        if (first_edge) {
            c1 = outer;
        } else {
            step1(r_first + dir, c1);
        }
        carry_init<R, NP, NM, ANISO, V, GEN, DOWN>(outer, c1, k1, c);
    }
    auto step2 = [&](int q) {
        R Cs[NP];
        const R tt = (R)(tbase1 + tslope * (double)q);
        psi_const_any<R, NP, GEN>(tt, c, x, Cs);
        R phin[NP][V], mun[NM][V], hn[NP][V];
        row_update<R, NP, NM, ANISO, OBST, V, GEN, DOWN>(c1, n1, k1, Cs, c, phin, mun, hn, tt, x);
        if (writes) {
            const int64_t o = (int64_t)q * nx + cs;
#pragma unroll
            for (int a = 0; a < NP; ++a) vstore<R, V>(out + a * fs + o, phin[a]);
#pragma unroll
            for (int kk = 0; kk < NM; ++kk) vstore<R, V>(out + (NP + kk) * fs + o, mun[kk]);
            if constexpr (DIAG) diag_row<R, NP, NM, V, GEN>(phin, mun, dc->tt0 + dc->tslope * (double)q, *dc, *da);
        }
        c1 = n1;
    };
    if constexpr (DOWN) {
        for (int q = m1 - 1; q > m0; --q) {
            step1(q - 1, n1);
            step2(q);
        }
        // last row: above a no-flux bottom edge step-1 row -1 is a copy of row 0
        if (top)
            n1 = c1;
        else
            step1(m0 - 1, n1);
        step2(m0);
    } else {
        for (int q = m0; q < m1 - 1; ++q) {
            step1(q + 1, n1);
            step2(q);
        }
        // last row: below a no-flux top edge step-1 row ny is a copy of row ny-1
        if (bot)
            n1 = c1;
        else
            step1(m1, n1);
        step2(m1 - 1);
    }
}

#ifndef MP_WAVES_PER_EU
#define MP_WAVES_PER_EU 2
#endif

// XCD-aware block order: the hardware deals blocks round-robin to the 8 XCDs,
// so block b works on (b mod 8) * (nb/8) + b/8 and each XCD gets a contiguous
// band of strips.
__device__ __forceinline__ int xcd_block() {
    const int nb = gridDim.x;
    const int q8 = nb / 8;
    const int b = blockIdx.x;
    return (b < 8 * q8) ? (b % 8) * q8 + b / 8 : b;
}

template <typename R, int NP, int NM, bool ANISO, bool OBST, int V>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MP_WAVES_PER_EU)))
k_step2d(const R* __restrict__ in, R* __restrict__ out, Geom g, Coef<R> c,
         const int64_t* __restrict__ stepctr, int kstep, double tb0, double tdn, double tslope,
         int seg, int ntx, int nseg) {
    const int wpb = blockDim.x >> 6;
    // wave-uniform by construction; readfirstlane tells the compiler so, which
    // keeps every row-loop branch scalar
    const int wid = __builtin_amdgcn_readfirstlane(xcd_block() * wpb + (threadIdx.x >> 6));
    if (wid >= ntx * nseg) return;  // whole wave leaves; nothing below synchronises
    const int tx = wid % ntx;
    const int sg = wid / ntx;
    const int m0 = sg * seg;
    const double tbase = tb0 + tdn * (double)(*stepctr + kstep);
    strip2d<R, NP, NM, ANISO, OBST, V>(in, out, g, c, tbase, tslope, tx, m0, min(m0 + seg, g.ny));
}

// Odd row segments march from the top down, so that the two segments on either
// side of a segment border reach the rows around it at about the same time and
// the second reads them from L2 (the results do not depend on the direction:
// every face takes the same operands in the same order).
template <typename R, int NP, int NM, bool ANISO, bool OBST, int V, bool STORE1 = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MP_WAVES_PER_EU)))
k_step2d_x2(const R* __restrict__ in, R* __restrict__ out, R* __restrict__ out1, Geom g, Coef<R> c,
            const int64_t* __restrict__ stepctr, int kstep, double tb0, double tdn, double tslope,
            int seg, int ntx, int nseg) {
    const int wpb = blockDim.x >> 6;
    const int wid = __builtin_amdgcn_readfirstlane(xcd_block() * wpb + (threadIdx.x >> 6));
    if (wid >= ntx * nseg) return;
    const int tx = wid % ntx;
    const int sg = wid / ntx;
    const int m0 = sg * seg;
    const double n = (double)(*stepctr + kstep);
    bool fixL, fixR;
    x2_column<V>(g, x2_first_col<V>(tx, threadIdx.x & 63), fixL, fixR);
    const bool xe = __ballot(fixL || fixR) != 0;
    const double t0 = tb0 + tdn * n, t1 = tb0 + tdn * (n + 1.0);
    const int m1 = min(m0 + seg, g.ny);
    if (sg & 1) {
        if (xe)
            strip2d_x2<R, NP, NM, ANISO, OBST, V, true, STORE1, false, false, true>(in, out, out1, g, c, t0, t1,
                                                                                   tslope, tx, m0, m1);
        else
            strip2d_x2<R, NP, NM, ANISO, OBST, V, false, STORE1, false, false, true>(in, out, out1, g, c, t0, t1,
                                                                                    tslope, tx, m0, m1);
    } else {
        if (xe)
            strip2d_x2<R, NP, NM, ANISO, OBST, V, true, STORE1>(in, out, out1, g, c, t0, t1, tslope, tx, m0, m1);
        else
            strip2d_x2<R, NP, NM, ANISO, OBST, V, false, STORE1>(in, out, out1, g, c, t0, t1, tslope, tx, m0, m1);
    }
}

// The general kernels of the extended model (one cell per lane): the same
// strips with the GEN cell and face arithmetic, and the extended
// coefficients as a further argument.
template <typename R, int NP, int NM, bool ANISO, bool OBST>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MP_WAVES_PER_EU)))
k_step2d_gen(const R* __restrict__ in, R* __restrict__ out, Geom g, Coef<R> c,
             const int64_t* __restrict__ stepctr, int kstep, double tb0, double tdn, double tslope,
             int seg, int ntx, int nseg, CoefX<R> x) {
    const int wpb = blockDim.x >> 6;
    const int wid = __builtin_amdgcn_readfirstlane(xcd_block() * wpb + (threadIdx.x >> 6));
    if (wid >= ntx * nseg) return;
    const int tx = wid % ntx;
    const int sg = wid / ntx;
    const int m0 = sg * seg;
    const double tbase = tb0 + tdn * (double)(*stepctr + kstep);
    strip2d<R, NP, NM, ANISO, OBST, 1, MP_STRIP_DEPTH, W2D_LANES_OUT, true>(in, out, g, c, tbase, tslope, tx, m0,
                                                                          min(m0 + seg, g.ny), &x);
}

template <typename R, int NP, int NM, bool ANISO, bool OBST>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MP_WAVES_PER_EU)))
k_step2d_x2_gen(const R* __restrict__ in, R* __restrict__ out, Geom g, Coef<R> c,
                const int64_t* __restrict__ stepctr, int kstep, double tb0, double tdn, double tslope,
                int seg, int ntx, int nseg, CoefX<R> x) {
    const int wpb = blockDim.x >> 6;
    const int wid = __builtin_amdgcn_readfirstlane(xcd_block() * wpb + (threadIdx.x >> 6));
    if (wid >= ntx * nseg) return;
    const int tx = wid % ntx;
    const int sg = wid / ntx;
    const int m0 = sg * seg;
    const double n = (double)(*stepctr + kstep);
    bool fixL, fixR;
    x2_column<1>(g, x2_first_col<1>(tx, threadIdx.x & 63), fixL, fixR);
    if (__ballot(fixL || fixR) != 0)
        strip2d_x2<R, NP, NM, ANISO, OBST, 1, true, false, true>(in, out, nullptr, g, c, tb0 + tdn * n,
                                                                 tb0 + tdn * (n + 1.0), tslope, tx, m0,
                                                                 min(m0 + seg, g.ny), &x);
    else
        strip2d_x2<R, NP, NM, ANISO, OBST, 1, false, false, true>(in, out, nullptr, g, c, tb0 + tdn * n,
                                                                  tb0 + tdn * (n + 1.0), tslope, tx, m0,
                                                                  min(m0 + seg, g.ny), &x);
}

// The same launches writing, beside the state, one partial diagnostics record
// per strip wave: the diagnostics of the state they store, so that it need
// not be read again (the record of wave w at d.part + w * DIAG_VALS).  The
// lanes' accumulators live in LDS (DiagStrip), 256 slots per sum.
template <int NP, int NM, bool TDEP>
__device__ __forceinline__ void diag_finish(const DiagStrip<NP, NM, TDEP>& A, const DiagOut& d, int wid) {
    DiagRec R;
    A.record(d.dc, R);
    rec_wave_reduce(R);
    if ((threadIdx.x & 63) == 0) rec_store(d.part + (int64_t)wid * DIAG_VALS, R);
}

// One cell per lane: at least the occupancy of the plain kernels with the most
// fields (FP64 3 waves per SIMD, FP32 5); the LDS accumulators take no VGPRs.
#define MP_DIAG_WAVES(R, V) ((V) == 1 ? (sizeof(R) == 8 ? 3 : 5) : MP_WAVES_PER_EU)

template <typename R, int NP, int NM, bool ANISO, bool OBST, int V, bool GEN>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MP_DIAG_WAVES(R, V))))
k_step2d_diag(const R* __restrict__ in, R* __restrict__ out, Geom g, Coef<R> c,
              const int64_t* __restrict__ stepctr, int kstep, double tb0, double tdn, double tslope,
              int seg, int ntx, int nseg, CoefX<R> x, DiagOut d) {
    const int wpb = blockDim.x >> 6;
    const int wid = __builtin_amdgcn_readfirstlane(xcd_block() * wpb + (threadIdx.x >> 6));
    if (wid >= ntx * nseg) return;
    const int tx = wid % ntx;
    const int sg = wid / ntx;
    const int m0 = sg * seg;
    const double tbase = tb0 + tdn * (double)(*stepctr + kstep);
    typedef DiagStrip<NP, NM, GEN> DS;
    __shared__ double dls[DS::WORDS];
    DS A;
    A.init(dls, threadIdx.x);
    strip2d<R, NP, NM, ANISO, OBST, V, MP_STRIP_DEPTH, W2D_LANES_OUT, GEN, true>(
        in, out, g, c, tbase, tslope, tx, m0, min(m0 + seg, g.ny), GEN ? &x : nullptr, &A, &d.dc);
    diag_finish(A, d, wid);
}

template <typename R, int NP, int NM, bool ANISO, bool OBST, int V, bool GEN>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MP_DIAG_WAVES(R, V))))
k_step2d_x2_diag(const R* __restrict__ in, R* __restrict__ out, Geom g, Coef<R> c,
                 const int64_t* __restrict__ stepctr, int kstep, double tb0, double tdn, double tslope,
                 int seg, int ntx, int nseg, CoefX<R> x, DiagOut d) {
    const int wpb = blockDim.x >> 6;
    const int wid = __builtin_amdgcn_readfirstlane(xcd_block() * wpb + (threadIdx.x >> 6));
    if (wid >= ntx * nseg) return;
    const int tx = wid % ntx;
    const int sg = wid / ntx;
    const int m0 = sg * seg;
    const double n = (double)(*stepctr + kstep);
    const CoefX<R>* xp = GEN ? &x : nullptr;
    typedef DiagStrip<NP, NM, GEN> DS;
    __shared__ double dls[DS::WORDS];
    DS A;
    A.init(dls, threadIdx.x);
    bool fixL, fixR;
    x2_column<V>(g, x2_first_col<V>(tx, threadIdx.x & 63), fixL, fixR);
    if (__ballot(fixL || fixR) != 0)
        strip2d_x2<R, NP, NM, ANISO, OBST, V, true, false, GEN, true>(in, out, nullptr, g, c, tb0 + tdn * n,
                                                                      tb0 + tdn * (n + 1.0), tslope, tx, m0,
                                                                      min(m0 + seg, g.ny), xp, &A, &d.dc);
    else
        strip2d_x2<R, NP, NM, ANISO, OBST, V, false, false, GEN, true>(in, out, nullptr, g, c, tb0 + tdn * n,
                                                                       tb0 + tdn * (n + 1.0), tslope, tx, m0,
                                                                       min(m0 + seg, g.ny), xp, &A, &d.dc);
    diag_finish(A, d, wid);
}

// Launch of a diagnostics instance: the plain or general strips, one or two
// steps, V cells per lane.
template <typename R, int NP, int NM, bool ANISO, bool OBST, int V, bool GEN>
int call_2d_diag(const StepLaunch& L, const Coef<R>& c, const CoefX<R>& x, KernelCall& k) {
    const int wout = L.fuse == 2 ? W2X_LANES_OUT : W2D_LANES_OUT;
    const int ntx = (L.g.nx + wout * V - 1) / (wout * V);
    const int nseg = (L.g.ny + L.seg - 1) / L.seg;
    const int wpb = L.bx / 64;
    const long long waves = (long long)ntx * nseg;
    const long long nblocks = (waves + wpb - 1) / wpb;
    // the lanes' LDS accumulators hold 256 slots per sum
    if (nblocks <= 0 || nblocks > 0x7fffffffLL || L.out1 || !L.diag || L.bx > 256) return MP_E_PARAM;
    k.func = L.fuse == 2 ? (const void*)&k_step2d_x2_diag<R, NP, NM, ANISO, OBST, V, GEN>
                         : (const void*)&k_step2d_diag<R, NP, NM, ANISO, OBST, V, GEN>;
    k.grid = dim3((unsigned)nblocks);
    k.block = dim3(L.bx);
    k.nrec = waves;
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
    k.arg(x);
    k.arg(*L.diag);
    return MP_OK;
}

template <typename R, int NP, int NM, bool ANISO, bool OBST, bool DIAG = false>
int call_2d_gen(const StepLaunch& L, const Coef<R>& c, const CoefX<R>& x, KernelCall& k) {
    if constexpr (DIAG) return call_2d_diag<R, NP, NM, ANISO, OBST, 1, true>(L, c, x, k);
    const int wout = L.fuse == 2 ? W2X_LANES_OUT : W2D_LANES_OUT;
    const int ntx = (L.g.nx + wout - 1) / wout;
    const int nseg = (L.g.ny + L.seg - 1) / L.seg;
    const int wpb = L.bx / 64;
    const long long waves = (long long)ntx * nseg;
    const long long nblocks = (waves + wpb - 1) / wpb;
    if (nblocks <= 0 || nblocks > 0x7fffffffLL || L.out1) return MP_E_PARAM;
    k.func = L.fuse == 2 ? (const void*)&k_step2d_x2_gen<R, NP, NM, ANISO, OBST>
                         : (const void*)&k_step2d_gen<R, NP, NM, ANISO, OBST>;
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
    k.arg(x);
    return MP_OK;
}

template <typename R, int NP, int NM, bool ANISO, bool OBST, int V>
int call_2d_v(const StepLaunch& L, const Coef<R>& c, KernelCall& k) {
    const int wout = L.fuse == 2 ? W2X_LANES_OUT : W2D_LANES_OUT;
    const int ntx = (L.g.nx + wout * V - 1) / (wout * V);
    const int nseg = (L.g.ny + L.seg - 1) / L.seg;
    const int wpb = L.bx / 64;
    const long long waves = (long long)ntx * nseg;
    const long long nblocks = (waves + wpb - 1) / wpb;
    if (nblocks <= 0 || nblocks > 0x7fffffffLL) return MP_E_PARAM;
    if (L.out1) {
        // the state between the two steps as well: built for the adjoint's
        // recomputation (isotropic, multi-well, one cell per lane)
        if constexpr (V == 1 && !ANISO && !OBST) {
            if (L.fuse != 2) return MP_E_PARAM;
            k.func = (const void*)&k_step2d_x2<R, NP, NM, ANISO, OBST, V, true>;
        } else {
            return MP_E_PARAM;
        }
    } else {
        k.func = L.fuse == 2 ? (const void*)&k_step2d_x2<R, NP, NM, ANISO, OBST, V>
                             : (const void*)&k_step2d<R, NP, NM, ANISO, OBST, V>;
    }
    k.grid = dim3((unsigned)nblocks);
    k.block = dim3(L.bx);
    k.arg((const R*)L.in);
    k.arg((R*)L.out);
    if (L.fuse == 2) k.arg((R*)L.out1);
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

template <typename R, int NP, int NM, bool ANISO, bool OBST, bool DIAG = false>
int call_2d(const StepLaunch& L, const Coef<R>& c, KernelCall& k) {
    const int v = vec2d_width(L.g.nx, (int)sizeof(R), L.vec);
    if constexpr (DIAG) {
        const CoefX<R> none{};
        if (v == 1) return call_2d_diag<R, NP, NM, ANISO, OBST, 1, false>(L, c, none, k);
        if (v == 2) return call_2d_diag<R, NP, NM, ANISO, OBST, 2, false>(L, c, none, k);
        if constexpr (sizeof(R) == 4) {
            if (v == 4) return call_2d_diag<R, NP, NM, ANISO, OBST, 4, false>(L, c, none, k);
        }
        return MP_E_PARAM;
    } else {
        if (v == 1) return call_2d_v<R, NP, NM, ANISO, OBST, 1>(L, c, k);
        if (v == 2) return call_2d_v<R, NP, NM, ANISO, OBST, 2>(L, c, k);
        if constexpr (sizeof(R) == 4) {
            if (v == 4) return call_2d_v<R, NP, NM, ANISO, OBST, 4>(L, c, k);
        }
        return MP_E_PARAM;
    }
}

}  // namespace mp
