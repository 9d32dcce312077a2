// Anti-trapping current of Eq. jatr applied after a 2D step (MICROSIM,
// arXiv 2404.01035, Sec. 2.1, Eq. Mu_explicit_temperature and Eq. jatr).
//
// The step kernel has written phi^{n+1} and the mu^{n+1} of the update without
// the current.  This kernel reads phi^n, mu^n (the step's input) and
// phi^{n+1}, forms the current on the four faces of every cell and corrects
// mu^{n+1} in place by -dt div(j_at) / chi(phi^{n+1}), so that the pair makes
// mu^{n+1} = mu^n + (dt div(M grad mu - j_at) - sum_a c^a dh_a) / chi.
//
// On a face between cells L and R (normal axis n, tangential axis t):
//   grad phi . e_n = (phi_R - phi_L) / dx, grad phi . e_t = mean over L, R of
//   the cells' central differences along t (the anisotropy stencil);
//   unit normal = grad phi / |grad phi|, zero where |grad phi|^2 <= 1e-30;
//   dphi_a/dt, c^a(mu^n) and the obstacle prefactor's phi are means of L, R;
//   j_k = sum over solids a of P(phi_a) (c^a_k - c^liq_k) dphi_a/dt
//         n_a . e_n (-n_a . n_liq), the liquid being the last phase.
// Ghost cells (periodic wrap or zero-flux mirror) come from index arithmetic.
// One wave per strip of 62 columns by 12 rows: each field is read once per cell
// (plus the halo) and each face is evaluated once.
#pragma once

#include "gp_device.hpp"

namespace mp {

__device__ inline int at_wrap(int i, int n, int bc) {
    if (i < 0) return bc == MP_BC_PERIODIC ? n - 1 : 0;
    if (i >= n) return bc == MP_BC_PERIODIC ? 0 : n - 1;
    return i;
}

// 1 / |grad phi| on a face, zero where |grad phi|^2 <= 1e-30 (the unit normal
// is then zero): the hardware reciprocal square root refined as in the step's
// anisotropy (the guard keeps its argument normal).
template <typename R>
__device__ __forceinline__ R at_inv_norm(R n2) {
    const bool on = n2 > R(1e-30);
    const R r = rsqrt_ok(on ? n2 : R(1));
    return on ? r : R(0);
}

template <typename R>
__device__ inline R at_prefactor(R f, const AtCoef<R>& c) {
    if (!c.obstacle) return c.prefw;
    if (!(f > R(0) && f < R(1))) return R(0);
    const R h1 = f * f * (R(3) - R(2) * f);
    return c.prefo * f * (R(1) - h1) / sqrt(f * (R(1) - f));
}

// Composition c^a_k(mu, T) = sum_j chi^a_kj (mu_j - B^a_j(T)) of a cell of the
// extended model (B^a(T) = B^a + Bt^a (T - Te), tt = T - Te of the cell's row;
// the off-diagonal chi^a_01 for two mu fields).
template <typename R, int NP, int NM>
__device__ __forceinline__ void at_comp_gen(const R* u, R tt, const AtCoef<R>& c, const CoefX<R>& x,
                                            R (&cc)[NP][NM]) {
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        R d[NM];
#pragma unroll
        for (int k = 0; k < NM; ++k) d[k] = u[k] - (c.B[a][k] + x.Bt[a][k] * tt);
#pragma unroll
        for (int k = 0; k < NM; ++k) {
            R v = c.chi[a][k] * d[k];
            if constexpr (NM == 2) v = v + x.chx[a] * d[1 - k];
            cc[a][k] = v;
        }
    }
}

// Current on one face.  pL/pR: phi^n of the two cells, tL/tR: their central
// differences along the tangential axis (already / (2 dx)), qL/qR: phi^{n+1},
// uL/uR: mu^n.  Adds the face's j_k to j.  GEN: the extended model's
// compositions (x its terms, ttL/ttR = T - Te of the two cells' rows).
template <typename R, int NP, int NM, bool GEN = false>
__device__ inline void at_face(const R* pL, const R* pR, const R* tL, const R* tR, const R* qL, const R* qR,
                               const R* uL, const R* uR, const AtCoef<R>& c, R* j, const CoefX<R>* x = nullptr,
                               R ttL = R(0), R ttR = R(0)) {
    constexpr int LIQ = NP - 1;
    R un[NP], ut[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        const R gn = (pR[a] - pL[a]) * c.rdx;
        const R gt = R(0.5) * (tL[a] + tR[a]);
        const R n2 = gn * gn + gt * gt;
        const R inv = at_inv_norm(n2);
        un[a] = gn * inv;
        ut[a] = gt * inv;
    }
    // The compositions are affine in mu (and B^a(T) in T), so the mean of the
    // two cells' compositions is the composition at the mean mu (and T).
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
    // dphi/dt of the face: (mean phi^{n+1} - mean phi^n) / dt
    const R hrdt = R(0.5) * c.rdt;
#pragma unroll
    for (int a = 0; a < NP - 1; ++a) {
        const R weight = -(un[a] * un[LIQ] + ut[a] * ut[LIQ]);
        const R rate = ((qL[a] + qR[a]) - (pL[a] + pR[a])) * hrdt;
        const R common = at_prefactor(R(0.5) * (pL[a] + pR[a]), c) * rate * un[a] * weight;
#pragma unroll
        for (int k = 0; k < NM; ++k) j[k] += common * (cb[a][k] - cb[LIQ][k]);
    }
}

// mu^{n+1} - dt chi(phi^{n+1})^-1 div j_at for the extended model: chi = sum_b h_b
// chi^b with the off-diagonal chi^b_01 for two mu fields (the step's 2 x 2
// solve), hb = h(phi^{n+1}), dv = div j_at.
template <typename R, int NP, int NM>
__device__ __forceinline__ void at_correct_gen(const R (&hb)[NP], const R (&dv)[NM], const AtCoef<R>& c,
                                               const CoefX<R>& x, R (&mn)[NM]) {
    R c00 = R(0);
#pragma unroll
    for (int b = 0; b < NP; ++b) c00 = c00 + hb[b] * c.chi[b][0];
    if constexpr (NM == 2) {
        R c11 = R(0), c01 = R(0);
#pragma unroll
        for (int b = 0; b < NP; ++b) {
            c11 = c11 + hb[b] * c.chi[b][1];
            c01 = c01 + hb[b] * x.chx[b];
        }
        const R r0 = c.dt * dv[0], r1 = c.dt * dv[1];
        const R inv = fast_rcp(c00 * c11 - c01 * c01);
        const R d0 = (c11 * r0 - c01 * r1) * inv;
        const R d1 = (c00 * r1 - c01 * r0) * inv;
        mn[0] = mn[0] - d0;
        mn[1] = mn[1] - d1;
    } else {
        mn[0] = mn[0] - (c.dt * dv[0]) * fast_rcp(c00);
    }
}

constexpr int AT_LANES_OUT = 62;  // written lanes per wave (lanes 0 and 63 hold the x halo)
#ifndef MP_AT_SEG
#define MP_AT_SEG 12
#endif
constexpr int AT_SEG = MP_AT_SEG;  // rows per wave
constexpr int AT_WAVES = 4;       // waves per block

// One row of one wave: every field of the row's cell at this lane.
template <typename R, int NP, int NM>
struct AtRow {
    R p[NP];   // phi^n
    R q[NP];   // phi^{n+1}
    R u[NM];   // mu^n
    R m[NM];   // mu^{n+1} of the step without the current
    R tx[NP];  // central difference of phi^n along x, / (2 dx)
};

// Loads of one row (issued early: the march keeps one row in flight ahead of the one it uses).
template <typename R, int NP, int NM>
__device__ inline void at_fetch(const R* __restrict__ prev, const R* __restrict__ next, const Geom& g, int col,
                                int row, AtRow<R, NP, NM>& r) {
    const int64_t o = (int64_t)row * g.nx + col;
    const int64_t fs = g.fstride;
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        r.p[a] = prev[a * fs + o];
        r.q[a] = next[a * fs + o];
    }
#pragma unroll
    for (int k = 0; k < NM; ++k) {
        r.u[k] = prev[(NP + k) * fs + o];
        r.m[k] = next[(NP + k) * fs + o];
    }
}

// The row's central differences along x, from the neighbouring lanes.
template <typename R, int NP, int NM>
__device__ inline void at_finish(AtRow<R, NP, NM>& r, R h2) {
#pragma unroll
    for (int a = 0; a < NP; ++a) r.tx[a] = (lane_next(r.p[a]) - lane_prev(r.p[a])) * h2;
}

// A wave owns columns x0 .. x0 + 61 (lanes 1..62; lane 0 and 63 are the x
// neighbours) over rows y0 .. y0 + AT_SEG - 1, and walks them top-down with
// rows y - 1, y, y + 1 in registers.  The x face below a lane (between its
// cell and the one to its left) is evaluated by that lane, the one above is
// its right neighbour's; the y face below a row is the one above the row
// before it.  Each face is evaluated once, with the operands and operations
// of the per-face definition, whichever cell it serves.
// GEN: the extended model (x its terms): the compositions at each row's
// temperature of time level n, T - Te = tbase + tslope * row, and the 2 x 2
// susceptibility in the correction.
template <typename R, int NP, int NM, bool GEN>
__device__ __forceinline__ void antitrap2d_strip(const R* __restrict__ prev, R* __restrict__ next, const Geom& g,
                                                 const AtCoef<R>& c, int nstrips, int nitems, const CoefX<R>* x,
                                                 double tbase, double tslope) {
    const int item = (int)blockIdx.x * AT_WAVES + (int)(threadIdx.x >> 6);
    if (item >= nitems) return;  // whole waves only
    const int lane = (int)(threadIdx.x & 63);
    const int strip = item % nstrips;
    const int y0 = (item / nstrips) * AT_SEG;
    const int y1 = y0 + AT_SEG < g.ny ? y0 + AT_SEG : g.ny;
    const int craw = strip * AT_LANES_OUT - 1 + lane;  // -1 .. nx + 62
    const bool own = lane >= 1 && lane <= AT_LANES_OUT && craw < g.nx;
    const int col = at_wrap(craw < g.nx ? craw : g.nx, g.nx, g.bcx);  // lanes past the right ghost repeat it
    const R h2 = R(0.5) * c.rdx;
    // T - Te of a row (the extended model)
    auto rowtt = [&](int row) { return GEN ? (R)(tbase + tslope * (double)row) : R(0); };
    AtRow<R, NP, NM> lo, mid, hi, ahead;
    const int ylo = at_wrap(y0 - 1, g.ny, g.bcy), yhi = at_wrap(y0 + 1, g.ny, g.bcy);
    at_fetch<R, NP, NM>(prev, next, g, col, ylo, lo);
    at_fetch<R, NP, NM>(prev, next, g, col, y0, mid);
    at_fetch<R, NP, NM>(prev, next, g, col, yhi, hi);
    R tlo = rowtt(ylo), tmid = rowtt(y0), thi = rowtt(yhi), tah = R(0);
    at_finish<R, NP, NM>(lo, h2);
    at_finish<R, NP, NM>(mid, h2);
    at_finish<R, NP, NM>(hi, h2);
    // y face between rows y0 - 1 and y0
    R jylo[NM] = {};
    at_face<R, NP, NM, GEN>(lo.p, mid.p, lo.tx, mid.tx, lo.q, mid.q, lo.u, mid.u, c, jylo, x, tlo, tmid);
    for (int y = y0; y < y1; ++y) {
        // row y + 2, needed by the next pass (past the grid's ghost row it is
        // a clamped or wrapped row that goes unused)
        const int ya = at_wrap(y + 2 < g.ny + 1 ? y + 2 : g.ny, g.ny, g.bcy);
        at_fetch<R, NP, NM>(prev, next, g, col, ya, ahead);
        if constexpr (GEN) tah = rowtt(ya);
        // x face between this lane's cell and the left neighbour, on row y
        R ty[NP], tyl[NP], pl[NP], ql[NP], ul[NM];
#pragma unroll
        for (int a = 0; a < NP; ++a) {
            ty[a] = (hi.p[a] - lo.p[a]) * h2;
            tyl[a] = lane_prev(ty[a]);
            pl[a] = lane_prev(mid.p[a]);
            ql[a] = lane_prev(mid.q[a]);
        }
#pragma unroll
        for (int k = 0; k < NM; ++k) ul[k] = lane_prev(mid.u[k]);
        R jxl[NM] = {};
        at_face<R, NP, NM, GEN>(pl, mid.p, tyl, ty, ql, mid.q, ul, mid.u, c, jxl, x, tmid, tmid);
        R jyhi[NM] = {};
        at_face<R, NP, NM, GEN>(mid.p, hi.p, mid.tx, hi.tx, mid.q, hi.q, mid.u, hi.u, c, jyhi, x, tmid, thi);
        // chi_k(phi^{n+1}) = sum_b h_b chi^b_k, h of Eq. hphi
        R hb[NP];
#pragma unroll
        for (int b = 0; b < NP; ++b) {
            const R f = mid.q[b];
            R cross = R(0);
            if constexpr (NP == 3) cross = mid.q[(b + 1) % 3] * mid.q[(b + 2) % 3];
            hb[b] = R(3) * f * f - R(2) * f * f * f + R(2) * f * cross;
        }
        const int64_t oc = (int64_t)y * g.nx + col;
        if constexpr (GEN) {
            R dv[NM], mn[NM];
#pragma unroll
            for (int k = 0; k < NM; ++k) {
                const R jxh = lane_next(jxl[k]);
                dv[k] = (jxh - jxl[k]) * c.rdx + (jyhi[k] - jylo[k]) * c.rdx;
                mn[k] = mid.m[k];
                jylo[k] = jyhi[k];
            }
            at_correct_gen<R, NP, NM>(hb, dv, c, *x, mn);
            if (own) {
#pragma unroll
                for (int k = 0; k < NM; ++k) next[(NP + k) * g.fstride + oc] = mn[k];
            }
        } else {
#pragma unroll
            for (int k = 0; k < NM; ++k) {
                const R jxh = lane_next(jxl[k]);
                if (own) {
                    R chik = R(0);
#pragma unroll
                    for (int b = 0; b < NP; ++b) chik += hb[b] * c.chi[b][k];
                    const R div = (jxh - jxl[k]) * c.rdx + (jyhi[k] - jylo[k]) * c.rdx;
                    next[(NP + k) * g.fstride + oc] = mid.m[k] - (c.dt * div) * fast_rcp(chik);
                }
                jylo[k] = jyhi[k];
            }
        }
        at_finish<R, NP, NM>(ahead, h2);
        lo = mid;
        mid = hi;
        hi = ahead;
        if constexpr (GEN) {
            tlo = tmid;
            tmid = thi;
            thi = tah;
        }
    }
}

template <typename R, int NP, int NM>
__global__ void __launch_bounds__(64 * AT_WAVES) k_antitrap2d(const R* __restrict__ prev, R* __restrict__ next,
                                                              Geom g, AtCoef<R> c, int nstrips, int nitems) {
    antitrap2d_strip<R, NP, NM, false>(prev, next, g, c, nstrips, nitems, nullptr, 0.0, 0.0);
}

// The extended model: the time level and temperature law as the step kernels take them.
template <typename R, int NP, int NM>
__global__ void __launch_bounds__(64 * AT_WAVES)
k_antitrap2d_gen(const R* __restrict__ prev, R* __restrict__ next, Geom g, AtCoef<R> c, int nstrips, int nitems,
                 CoefX<R> x, const int64_t* __restrict__ stepctr, int kstep, double tb0, double tdn, double tslope) {
    antitrap2d_strip<R, NP, NM, true>(prev, next, g, c, nstrips, nitems, &x, tb0 + tdn * (double)(*stepctr + kstep),
                                      tslope);
}

// The time level and temperature law of the extended model's correction.
struct AtTime {
    const int64_t* stepctr;
    int kstep;
    double tb0, tdn, tslope;
};

template <typename R, int NP, int NM, bool GEN>
void at_launch2d_kernel(const AtLaunch& L, const AtCoef<R>& c, const CoefX<R>* x, const AtTime* t, dim3 grid,
                        dim3 block, int nstrips, int nitems, hipStream_t s) {
    const R* prev = (const R*)L.prev;
    R* next = (R*)L.next;
    if constexpr (GEN)
        hipLaunchKernelGGL((k_antitrap2d_gen<R, NP, NM>), grid, block, 0, s, prev, next, L.g, c, nstrips, nitems, *x,
                           t->stepctr, t->kstep, t->tb0, t->tdn, t->tslope);
    else
        hipLaunchKernelGGL((k_antitrap2d<R, NP, NM>), grid, block, 0, s, prev, next, L.g, c, nstrips, nitems);
}

// GEN: the extended model, x and t its terms and time (unused otherwise).
template <typename R, bool GEN = false>
int at_launch2d(const AtLaunch& L, const AtCoef<R>& c, hipStream_t s, const CoefX<R>* x = nullptr,
                const AtTime* t = nullptr) {
    if (L.g.nz != 1 || L.g.nx < 1 || L.g.ny < 1 || (GEN && (!x || !t))) return MP_E_PARAM;
    const int nstrips = (L.g.nx + AT_LANES_OUT - 1) / AT_LANES_OUT;
    const int64_t items = (int64_t)nstrips * ((L.g.ny + AT_SEG - 1) / AT_SEG);
    if (items > INT32_MAX - AT_WAVES) return MP_E_PARAM;
    const int nitems = (int)items;
    dim3 block(64 * AT_WAVES);
    dim3 grid((unsigned)((nitems + AT_WAVES - 1) / AT_WAVES));
    if (L.nphases == 2 && L.nmu == 1)
        at_launch2d_kernel<R, 2, 1, GEN>(L, c, x, t, grid, block, nstrips, nitems, s);
    else if (L.nphases == 2 && L.nmu == 2)
        at_launch2d_kernel<R, 2, 2, GEN>(L, c, x, t, grid, block, nstrips, nitems, s);
    else if (L.nphases == 3 && L.nmu == 1)
        at_launch2d_kernel<R, 3, 1, GEN>(L, c, x, t, grid, block, nstrips, nitems, s);
    else if (L.nphases == 3 && L.nmu == 2)
        at_launch2d_kernel<R, 3, 2, GEN>(L, c, x, t, grid, block, nstrips, nitems, s);
    else
        return MP_E_PARAM;
    return hipGetLastError() == hipSuccess ? MP_OK : MP_E_HIP;
}

}  // namespace mp
