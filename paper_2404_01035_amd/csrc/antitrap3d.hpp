// Anti-trapping current of Eq. jatr applied after a 3D step (MICROSIM,
// arXiv 2404.01035, Sec. 2.1): the 3D counterpart of k_antitrap2d, with the
// same face definition (antitrap2d.hpp's header comment) and the tangential
// components in x, y, z order.
//
// A wave owns a strip of 62 x columns (lanes 1..62; lanes 0 and 63 hold the x
// neighbours) by BY rows and marches a segment of z planes.  Per plane it keeps
// rows y0-1 .. y0+BY of phi^n, phi^{n+1} and mu^n of planes m-1 (phi^n only),
// m and m+1 in registers, with plane m+2 in flight.  On plane m:
//   x faces: each lane evaluates the face on its left (the left cell's values
//     by lane shuffles) and takes the one on its right from its right
//     neighbour;
//   y faces: the BY + 1 faces between consecutive rows of the wave, each once
//     (the two at the ends of the wave's rows are also evaluated by the waves
//     above and below);
//   z faces: the face to plane m+1 is evaluated once and carried as the lower
//     face of the next plane.
// Work items run strip-fastest (strip, then row group, then z segment) and
// blocks are dealt XCD-aware, so the strips of one row group run together on
// one XCD: the 128-byte lines where two strips' 64-column rows overlap (a
// strip's rows start one column before its first column) are fetched once
// into that XCD's L2, and the row groups above and below, a few blocks away,
// share their halo rows there too.
#pragma once

#include "antitrap2d.hpp"

namespace mp {

// Current of one face normal to axis AX between cells L and R: s and t are the
// two cells' central differences (already x 1/(2 dx)) along the tangential axes
// in increasing axis order.  Adds the face's j_k to j.  GEN: the extended
// model's compositions (x its terms, ttL/ttR = T - Te of the two cells' rows).
template <typename R, int NP, int NM, int AX, bool GEN = false>
__device__ __forceinline__ void at_face3(const R (&pL)[NP], const R (&pR)[NP], const R (&sL)[NP], const R (&sR)[NP],
                                         const R (&tL)[NP], const R (&tR)[NP], const R (&qL)[NP],
                                         const R (&qR)[NP], const R (&uL)[NM], const R (&uR)[NM],
                                         const AtCoef<R>& c, R (&j)[NM], const CoefX<R>* x = nullptr,
                                         R ttL = R(0), R ttR = R(0)) {
    constexpr int LIQ = NP - 1;
    R u[3][NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        const R gn = (pR[a] - pL[a]) * c.rdx;
        const R g1 = R(0.5) * (sL[a] + sR[a]);
        const R g2 = R(0.5) * (tL[a] + tR[a]);
        const R gx = AX == 0 ? gn : g1;
        const R gy = AX == 0 ? g1 : (AX == 1 ? gn : g2);
        const R gz = AX == 2 ? gn : g2;
        R n2 = R(0);
        n2 += gx * gx;
        n2 += gy * gy;
        n2 += gz * gz;
        const R inv = at_inv_norm(n2);
        u[0][a] = gx * inv;
        u[1][a] = gy * inv;
        u[2][a] = gz * inv;
    }
    // the composition at the mean mu (and T) is the mean composition (at_face)
    R ub[NM];
#pragma unroll
    for (int k = 0; k < NM; ++k) ub[k] = R(0.5) * (uL[k] + uR[k]);
    R cb[NP][NM];
    if constexpr (GEN) {
        at_comp_gen<R, NP, NM>(ub, R(0.5) * (ttL + ttR), c, *x, cb);
    } else {
#pragma unroll
        for (int a = 0; a < NP; ++a)
#pragma unroll
            for (int k = 0; k < NM; ++k) cb[a][k] = c.chi[a][k] * (ub[k] - c.B[a][k]);
    }
    const R hrdt = R(0.5) * c.rdt;
#pragma unroll
    for (int a = 0; a < NP - 1; ++a) {
        const R weight = -((u[0][a] * u[0][LIQ] + u[1][a] * u[1][LIQ]) + u[2][a] * u[2][LIQ]);
        const R rate = ((qL[a] + qR[a]) - (pL[a] + pR[a])) * hrdt;
        const R common = at_prefactor(R(0.5) * (pL[a] + pR[a]), c) * rate * u[AX][a] * weight;
#pragma unroll
        for (int k = 0; k < NM; ++k) j[k] += common * (cb[a][k] - cb[LIQ][k]);
    }
}

constexpr int AT3_LANES_OUT = 62;  // written lanes per wave
constexpr int AT3_WAVES = 4;       // waves per block: consecutive row groups of one strip
#ifndef MP_AT3_SEG
#define MP_AT3_SEG 64
#endif
constexpr int AT3_SEG = MP_AT3_SEG;  // z planes per wave

// Rows y0-1 .. y0+BY of one z plane at this lane.
template <typename R, int NP, int NM, int BY>
struct At3Plane {
    R p[BY + 2][NP];  // phi^n
    R q[BY + 2][NP];  // phi^{n+1}
    R u[BY + 2][NM];  // mu^n
};

template <typename R, int NP, int NM, int BY>
__device__ __forceinline__ void at3_fetch(const R* __restrict__ prev, const R* __restrict__ next, const Geom& g,
                                          int col, int y0, int z, At3Plane<R, NP, NM, BY>& P) {
    const int64_t fs = g.fstride;
    const int64_t zo = (int64_t)at_wrap(z, g.nz, g.bcz) * g.ny;
#pragma unroll
    for (int r = 0; r < BY + 2; ++r) {
        const int64_t o = (zo + at_wrap(y0 - 1 + r, g.ny, g.bcy)) * g.nx + col;
#pragma unroll
        for (int a = 0; a < NP; ++a) {
            P.p[r][a] = prev[a * fs + o];
            P.q[r][a] = next[a * fs + o];
        }
#pragma unroll
        for (int k = 0; k < NM; ++k) P.u[r][k] = prev[(NP + k) * fs + o];
    }
}

// Central difference along x (x 1/(2 dx)) of phi^n at every row, from the neighbouring lanes.
template <typename R, int NP, int NROW>
__device__ __forceinline__ void at3_dx(const R (&p)[NROW][NP], R h2, R (&t)[NROW][NP]) {
#pragma unroll
    for (int r = 0; r < NROW; ++r)
#pragma unroll
        for (int a = 0; a < NP; ++a) t[r][a] = (lane_next(p[r][a]) - lane_prev(p[r][a])) * h2;
}

// GEN: the extended model (x its terms, T - Te = tbase + tslope * row).
template <typename R, int NP, int NM, int BY, bool GEN>
__device__ __forceinline__ void antitrap3d_wave(const R* __restrict__ prev, R* __restrict__ next, const Geom& g,
                                                const AtCoef<R>& c, int nstrips, int nygroups, int nitems,
                                                const CoefX<R>* x, double tbase, double tslope) {
    const int nb = gridDim.x;
    const int q8 = nb / 8;
    const int b = blockIdx.x;
    const int blk = (b < 8 * q8) ? (b % 8) * q8 + b / 8 : b;  // XCD-aware block order
    const int item = __builtin_amdgcn_readfirstlane(blk * AT3_WAVES + (int)(threadIdx.x >> 6));
    if (item >= nitems) return;  // whole waves only; nothing below synchronises
    const int lane = (int)(threadIdx.x & 63);
    const int strip = item % nstrips;
    const int rest = item / nstrips;
    const int yg = rest % nygroups;
    const int z0 = (rest / nygroups) * AT3_SEG;
    const int z1 = z0 + AT3_SEG < g.nz ? z0 + AT3_SEG : g.nz;
    const int y0 = yg * BY;
    const int craw = strip * AT3_LANES_OUT - 1 + lane;  // -1 .. nx + 62
    const bool ownx = lane >= 1 && lane <= AT3_LANES_OUT && craw < g.nx;
    const int col = at_wrap(craw < g.nx ? craw : g.nx, g.nx, g.bcx);  // lanes past the right ghost repeat it
    const R h2 = R(0.5) * c.rdx;
    const int64_t fs = g.fstride;
    // T - Te of the wave's rows y0-1 .. y0+BY (the extended model; T depends on y only)
    R ttr[BY + 2];
#pragma unroll
    for (int r = 0; r < BY + 2; ++r)
        ttr[r] = GEN ? (R)(tbase + tslope * (double)at_wrap(y0 - 1 + r, g.ny, g.bcy)) : R(0);

    At3Plane<R, NP, NM, BY> A, B, C, D;
    at3_fetch<R, NP, NM, BY>(prev, next, g, col, y0, z0 - 1, A);
    at3_fetch<R, NP, NM, BY>(prev, next, g, col, y0, z0, B);
    at3_fetch<R, NP, NM, BY>(prev, next, g, col, y0, z0 + 1, C);

    // z face between planes z0 - 1 and z0, rows y0 .. y0 + BY - 1
    R jzlo[BY][NM];
    {
        R txa[BY + 2][NP], txb[BY + 2][NP];
        at3_dx<R, NP, BY + 2>(A.p, h2, txa);
        at3_dx<R, NP, BY + 2>(B.p, h2, txb);
#pragma unroll
        for (int r = 1; r <= BY; ++r) {
            R tya[NP], tyb[NP];
#pragma unroll
            for (int a = 0; a < NP; ++a) {
                tya[a] = (A.p[r + 1][a] - A.p[r - 1][a]) * h2;
                tyb[a] = (B.p[r + 1][a] - B.p[r - 1][a]) * h2;
            }
#pragma unroll
            for (int k = 0; k < NM; ++k) jzlo[r - 1][k] = R(0);
            at_face3<R, NP, NM, 2, GEN>(A.p[r], B.p[r], txa[r], txb[r], tya, tyb, A.q[r], B.q[r], A.u[r], B.u[r], c,
                                        jzlo[r - 1], x, ttr[r], ttr[r]);
        }
    }

    for (int m = z0; m < z1; ++m) {
        // plane m + 2 for the next pass (past the grid's ghost plane it is a
        // wrapped or clamped plane that goes unused), and mu^{n+1} of plane m
        at3_fetch<R, NP, NM, BY>(prev, next, g, col, y0, m + 2 < g.nz + 1 ? m + 2 : g.nz, D);
        const int64_t zo = (int64_t)m * g.ny;
        R mn[BY][NM];
#pragma unroll
        for (int r = 0; r < BY; ++r) {
            const int yy = y0 + r < g.ny ? y0 + r : g.ny - 1;
#pragma unroll
            for (int k = 0; k < NM; ++k) mn[r][k] = next[(NP + k) * fs + (zo + yy) * g.nx + col];
        }
        // tangential differences: along x on planes m and m+1, along z on
        // plane m, along y on planes m and m+1
        R txm[BY + 2][NP], txc[BY + 2][NP], tz[BY + 2][NP];
        at3_dx<R, NP, BY + 2>(B.p, h2, txm);
        at3_dx<R, NP, BY + 2>(C.p, h2, txc);
#pragma unroll
        for (int r = 0; r < BY + 2; ++r)
#pragma unroll
            for (int a = 0; a < NP; ++a) tz[r][a] = (C.p[r][a] - A.p[r][a]) * h2;
        // y faces between rows r and r+1 (local rows 0 .. BY+1)
        R jy[BY + 1][NM];
#pragma unroll
        for (int r = 0; r <= BY; ++r) {
#pragma unroll
            for (int k = 0; k < NM; ++k) jy[r][k] = R(0);
            at_face3<R, NP, NM, 1, GEN>(B.p[r], B.p[r + 1], txm[r], txm[r + 1], tz[r], tz[r + 1], B.q[r],
                                        B.q[r + 1], B.u[r], B.u[r + 1], c, jy[r], x, ttr[r], ttr[r + 1]);
        }
#pragma unroll
        for (int r = 1; r <= BY; ++r) {
            R tym[NP], tyc[NP];
#pragma unroll
            for (int a = 0; a < NP; ++a) {
                tym[a] = (B.p[r + 1][a] - B.p[r - 1][a]) * h2;
                tyc[a] = (C.p[r + 1][a] - C.p[r - 1][a]) * h2;
            }
            // x face between the left lane's cell and this one
            R pl[NP], ql[NP], ul[NM], tyl[NP], tzl[NP];
#pragma unroll
            for (int a = 0; a < NP; ++a) {
                pl[a] = lane_prev(B.p[r][a]);
                ql[a] = lane_prev(B.q[r][a]);
                tyl[a] = lane_prev(tym[a]);
                tzl[a] = lane_prev(tz[r][a]);
            }
#pragma unroll
            for (int k = 0; k < NM; ++k) ul[k] = lane_prev(B.u[r][k]);
            R jxl[NM], jzh[NM];
#pragma unroll
            for (int k = 0; k < NM; ++k) jxl[k] = jzh[k] = R(0);
            at_face3<R, NP, NM, 0, GEN>(pl, B.p[r], tyl, tym, tzl, tz[r], ql, B.q[r], ul, B.u[r], c, jxl, x, ttr[r],
                                        ttr[r]);
            // z face to plane m + 1
            at_face3<R, NP, NM, 2, GEN>(B.p[r], C.p[r], txm[r], txc[r], tym, tyc, B.q[r], C.q[r], B.u[r], C.u[r], c,
                                        jzh, x, ttr[r], ttr[r]);
            // chi_k(phi^{n+1}) = sum_b h_b chi^b_k, h of Eq. hphi
            R hb[NP];
#pragma unroll
            for (int a = 0; a < NP; ++a) {
                const R f = B.q[r][a];
                R cross = R(0);
                if constexpr (NP == 3) cross = B.q[r][(a + 1) % 3] * B.q[r][(a + 2) % 3];
                hb[a] = R(3) * f * f - R(2) * f * f * f + R(2) * f * cross;
            }
            const int yy = y0 + r - 1;
            if constexpr (GEN) {
                R dv[NM], mc[NM];
#pragma unroll
                for (int k = 0; k < NM; ++k) {
                    const R jxh = lane_next(jxl[k]);
                    R div = R(0);
                    div += (jxh - jxl[k]) * c.rdx;
                    div += (jy[r][k] - jy[r - 1][k]) * c.rdx;
                    div += (jzh[k] - jzlo[r - 1][k]) * c.rdx;
                    dv[k] = div;
                    mc[k] = mn[r - 1][k];
                    jzlo[r - 1][k] = jzh[k];
                }
                at_correct_gen<R, NP, NM>(hb, dv, c, *x, mc);
                if (ownx && yy < g.ny) {
#pragma unroll
                    for (int k = 0; k < NM; ++k) next[(NP + k) * fs + (zo + yy) * g.nx + col] = mc[k];
                }
            } else {
#pragma unroll
                for (int k = 0; k < NM; ++k) {
                    const R jxh = lane_next(jxl[k]);
                    if (ownx && yy < g.ny) {
                        R chik = R(0);
#pragma unroll
                        for (int a = 0; a < NP; ++a) chik += hb[a] * c.chi[a][k];
                        R div = R(0);
                        div += (jxh - jxl[k]) * c.rdx;
                        div += (jy[r][k] - jy[r - 1][k]) * c.rdx;
                        div += (jzh[k] - jzlo[r - 1][k]) * c.rdx;
                        next[(NP + k) * fs + (zo + yy) * g.nx + col] = mn[r - 1][k] - (c.dt * div) * fast_rcp(chik);
                    }
                    jzlo[r - 1][k] = jzh[k];
                }
            }
        }
        A = B;
        B = C;
        C = D;
    }
}

template <typename R, int NP, int NM, int BY>
__global__ void __launch_bounds__(64 * AT3_WAVES) k_antitrap3d(const R* __restrict__ prev, R* __restrict__ next,
                                                               Geom g, AtCoef<R> c, int nstrips, int nygroups,
                                                               int nitems) {
    antitrap3d_wave<R, NP, NM, BY, false>(prev, next, g, c, nstrips, nygroups, nitems, nullptr, 0.0, 0.0);
}

// The extended model: the time level and temperature law as the step kernels take them.
template <typename R, int NP, int NM, int BY>
__global__ void __launch_bounds__(64 * AT3_WAVES)
k_antitrap3d_gen(const R* __restrict__ prev, R* __restrict__ next, Geom g, AtCoef<R> c, int nstrips, int nygroups,
                 int nitems, CoefX<R> x, const int64_t* __restrict__ stepctr, int kstep, double tb0, double tdn,
                 double tslope) {
    antitrap3d_wave<R, NP, NM, BY, true>(prev, next, g, c, nstrips, nygroups, nitems, &x,
                                         tb0 + tdn * (double)(*stepctr + kstep), tslope);
}

// Rows per wave: the planes held in registers grow with it (2 rows: 125 VGPRs
// for the binary FP32 case; FP64 takes 1 row so that its ternary variants do
// not spill).
template <typename R>
constexpr int at3_rows() {
    return sizeof(R) == 4 ? 2 : 1;
}

template <typename R, int NP, int NM, int BY, bool GEN>
void at_launch3d_kernel(const AtLaunch& L, const AtCoef<R>& c, const CoefX<R>* x, const AtTime* t, dim3 grid,
                        dim3 block, int nstrips, int nyg, int nitems, hipStream_t s) {
    const R* prev = (const R*)L.prev;
    R* next = (R*)L.next;
    if constexpr (GEN)
        hipLaunchKernelGGL((k_antitrap3d_gen<R, NP, NM, BY>), grid, block, 0, s, prev, next, L.g, c, nstrips, nyg,
                           nitems, *x, t->stepctr, t->kstep, t->tb0, t->tdn, t->tslope);
    else
        hipLaunchKernelGGL((k_antitrap3d<R, NP, NM, BY>), grid, block, 0, s, prev, next, L.g, c, nstrips, nyg, nitems);
}

// GEN: the extended model, x and t its terms and time (unused otherwise).
template <typename R, bool GEN = false>
int at_launch3d(const AtLaunch& L, const AtCoef<R>& c, hipStream_t s, const CoefX<R>* x = nullptr,
                const AtTime* t = nullptr) {
    constexpr int BY = at3_rows<R>();
    if (L.g.nx < 1 || L.g.ny < 1 || L.g.nz < 1 || (GEN && (!x || !t))) return MP_E_PARAM;
    const int nstrips = (L.g.nx + AT3_LANES_OUT - 1) / AT3_LANES_OUT;
    const int nyg = (L.g.ny + BY - 1) / BY;
    const int64_t items = (int64_t)nstrips * nyg * ((L.g.nz + AT3_SEG - 1) / AT3_SEG);
    if (items > INT32_MAX - AT3_WAVES) return MP_E_PARAM;
    const int nitems = (int)items;
    dim3 block(64 * AT3_WAVES);
    dim3 grid((unsigned)((nitems + AT3_WAVES - 1) / AT3_WAVES));
    if (L.nphases == 2 && L.nmu == 1)
        at_launch3d_kernel<R, 2, 1, BY, GEN>(L, c, x, t, grid, block, nstrips, nyg, nitems, s);
    else if (L.nphases == 2 && L.nmu == 2)
        at_launch3d_kernel<R, 2, 2, BY, GEN>(L, c, x, t, grid, block, nstrips, nyg, nitems, s);
    else if (L.nphases == 3 && L.nmu == 1)
        at_launch3d_kernel<R, 3, 1, BY, GEN>(L, c, x, t, grid, block, nstrips, nyg, nitems, s);
    else if (L.nphases == 3 && L.nmu == 2)
        at_launch3d_kernel<R, 3, 2, BY, GEN>(L, c, x, t, grid, block, nstrips, nyg, nitems, s);
    else
        return MP_E_PARAM;
    return hipGetLastError() == hipSuccess ? MP_OK : MP_E_HIP;
}

}  // namespace mp
