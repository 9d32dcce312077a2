// One 2D step with the anti-trapping current of Eq. jatr folded in (MICROSIM,
// arXiv 2404.01035, Sec. 2.1, Eq. Mu_explicit_temperature and Eq. jatr): the
// step of the strip kernels and the correction of the separate correction
// kernel in one pass, so the state is read once and written once per step
// (the pair of kernels reads it twice and mu^{n+1} three times).
#pragma once

#include "antitrap2d.hpp"
#include "step2d.hpp"

namespace mp {

// One step with the anti-trapping current of Eq. jatr folded in (one cell
// per lane, the two-step strip's lane layout: lanes 2..61 written).  The step
// of row r is computed as in strip2d_x2's first step; the correction of
// mu^{n+1} at row q needs phi^{n+1} of rows q-1..q+1 and of the neighbouring
// lanes, so it runs one row behind: after the step of row q+1 the current on
// the y face (q, q+1) and on the x face left of each lane of row q is formed
// (at_face, the correction kernel's face arithmetic), the face (q-1, q) having
// been formed for row q-1, and row q is corrected and written.  phi^n and mu^n
// of rows q-1..q+1 and phi^{n+1}, mu^{n+1} of rows q, q+1 are kept in
// registers.  A no-flux edge's ghost row or column is an exact copy of the
// cell it mirrors, so its face carries no current, as in the correction
// kernel; a periodic ghost row is stepped from its wrapped neighbours.  The
// arithmetic is that of strip2d followed by k_antitrap2d, operation for
// operation.  GEN: the extended model (x its terms): the general step, and
// compositions at each row's temperature of time level n with the 2 x 2
// susceptibility in the correction.
template <typename R, int NP, int NM, bool ANISO, bool OBST, bool XEDGE, bool GEN = false>
__device__ __forceinline__ void strip2d_at(const R* __restrict__ in, R* __restrict__ out, const Geom& g,
                                           const Coef<R>& c, const AtCoef<R>& ac, double tbase, double tslope,
                                           int tx, int m0, int m1, const CoefX<R>* x = nullptr) {
    constexpr int V = 1;
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
    const bool top = !pery && m0 == 0;   // row -1 is a copy of row 0: its face carries nothing
    const bool bot = !pery && m1 == ny;  // row ny is a copy of row ny-1
    const int r_first = top ? 0 : m0 - 1;
    const R h2 = R(0.5) * ac.rdx;

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

    Carry2d<R, NP, NM, V, ANISO> k0;
    RowT c0, n0;
    // rows of phi^n (hp[0] the newest), mu^n, and phi^{n+1}, mu^{n+1} before the correction
    R hp[3][NP], hu[2][NM], nq[2][NP], nm[2][NM];
    R htt[2] = {R(0), R(0)};  // T - Te of the rows of hu (extended model)
    {
        RawT a, b, d;
        load(r_first - 1, a);
        load(r_first, b);
        load(r_first + 1, d);
        RowT prv;
        process(a, prv);
        process(b, c0);
        carry_init<R, NP, NM, ANISO, V, GEN>(prv, c0, k0, c);
        process(d, n0);
#pragma unroll
        for (int q = 0; q < NP; ++q) hp[0][q] = prv.phi[0][q];
    }

    // The step of row r (c0 = state row r), pushed onto the row history; the
    // window then moves up one row, raw holding state row r + 2.
    auto step = [&](int r, RawT& raw) {
        R Cs[NP];
        const R tt = (R)(tbase + tslope * (double)rowmap(r));
        psi_const_any<R, NP, GEN>(tt, c, x, Cs);
        R phin[NP][V], mun[NM][V], hn[NP][V];
        row_update<R, NP, NM, ANISO, OBST, V, GEN>(c0, n0, k0, Cs, c, phin, mun, hn, tt, x);
        if constexpr (GEN) {
            htt[1] = htt[0];
            htt[0] = tt;
        }
        R v[NF][V];
#pragma unroll
        for (int a = 0; a < NP; ++a) v[a][0] = phin[a][0];
#pragma unroll
        for (int kk = 0; kk < NM; ++kk) v[NP + kk][0] = mun[kk][0];
        if constexpr (XEDGE) {
            // mirror ghost columns: copies of the cells they mirror
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const R nextFirst = lane_next(v[f][0]);
                const R prevLast = lane_prev(v[f][0]);
                v[f][0] = fixL ? nextFirst : (fixR ? prevLast : v[f][0]);
            }
        }
#pragma unroll
        for (int a = 0; a < NP; ++a) {
            hp[2][a] = hp[1][a];
            hp[1][a] = hp[0][a];
            hp[0][a] = c0.phi[0][a];
            nq[1][a] = nq[0][a];
            nq[0][a] = v[a][0];
        }
#pragma unroll
        for (int kk = 0; kk < NM; ++kk) {
            hu[1][kk] = hu[0][kk];
            hu[0][kk] = c0.mu[0][kk];
            nm[1][kk] = nm[0][kk];
            nm[0][kk] = v[NP + kk][0];
        }
        c0 = n0;
        process(raw, n0);
    };
    // row ny beyond a no-flux edge: a copy of row ny - 1
    auto mirror_row = [&]() {
#pragma unroll
        for (int a = 0; a < NP; ++a) {
            hp[2][a] = hp[1][a];
            hp[1][a] = hp[0][a];
            nq[1][a] = nq[0][a];
        }
#pragma unroll
        for (int kk = 0; kk < NM; ++kk) {
            hu[1][kk] = hu[0][kk];
            nm[1][kk] = nm[0][kk];
        }
        if constexpr (GEN) htt[1] = htt[0];
    };
    // central difference along x (x 1/(2 dx)) of a row of phi^n
    auto ddx = [&](const R (&p)[NP], R (&t)[NP]) {
#pragma unroll
        for (int a = 0; a < NP; ++a) t[a] = (lane_next(p[a]) - lane_prev(p[a])) * h2;
    };

    // jylo: the current on the face below the row being corrected; tq: the x
    // differences of the next row to be corrected (carried from the row above)
    R jylo[NM], tq[NP];
    // the face below row m0, once row m0 has been stepped
    auto first_face = [&]() {
        if (top) {
            // row -1 mirrors row 0: hp[1] stands for it, and the face (-1, 0) carries nothing
#pragma unroll
            for (int a = 0; a < NP; ++a) hp[1][a] = hp[0][a];
#pragma unroll
            for (int kk = 0; kk < NM; ++kk) jylo[kk] = R(0);
            ddx(hp[0], tq);
        } else {
            R ta[NP];
            ddx(hp[1], ta);
            ddx(hp[0], tq);
#pragma unroll
            for (int kk = 0; kk < NM; ++kk) jylo[kk] = R(0);
            at_face<R, NP, NM, GEN>(hp[1], hp[0], ta, tq, nq[1], nq[0], hu[1], hu[0], ac, jylo, x, htt[1], htt[0]);
        }
    };
    // the current around row q (rows q-1, q, q+1 of phi^n are hp[2], hp[1],
    // hp[0]) and the corrected row q written
    auto correct = [&](int q) {
        R ty[NP], tyl[NP], pl[NP], ql[NP], ul[NM], txh[NP];
#pragma unroll
        for (int a = 0; a < NP; ++a) {
            ty[a] = (hp[0][a] - hp[2][a]) * h2;
            tyl[a] = lane_prev(ty[a]);
            pl[a] = lane_prev(hp[1][a]);
            ql[a] = lane_prev(nq[1][a]);
        }
#pragma unroll
        for (int kk = 0; kk < NM; ++kk) ul[kk] = lane_prev(hu[1][kk]);
        R jxl[NM] = {};
        at_face<R, NP, NM, GEN>(pl, hp[1], tyl, ty, ql, nq[1], ul, hu[1], ac, jxl, x, htt[1], htt[1]);
        ddx(hp[0], txh);
        R jyhi[NM] = {};
        at_face<R, NP, NM, GEN>(hp[1], hp[0], tq, txh, nq[1], nq[0], hu[1], hu[0], ac, jyhi, x, htt[1], htt[0]);
#pragma unroll
        for (int a = 0; a < NP; ++a) tq[a] = txh[a];
        R hb[NP];
#pragma unroll
        for (int b = 0; b < NP; ++b) {
            const R f = nq[1][b];
            R cross = R(0);
            if constexpr (NP == 3) cross = nq[1][(b + 1) % 3] * nq[1][(b + 2) % 3];
            hb[b] = R(3) * f * f - R(2) * f * f * f + R(2) * f * cross;
        }
        const int64_t o = (int64_t)q * nx + cs;
        if (writes) {
#pragma unroll
            for (int a = 0; a < NP; ++a) out[a * fs + o] = nq[1][a];
        }
        if constexpr (GEN) {
            R dv[NM], mn[NM];
#pragma unroll
            for (int kk = 0; kk < NM; ++kk) {
                const R jxh = lane_next(jxl[kk]);
                dv[kk] = (jxh - jxl[kk]) * ac.rdx + (jyhi[kk] - jylo[kk]) * ac.rdx;
                mn[kk] = nm[1][kk];
                jylo[kk] = jyhi[kk];
            }
            at_correct_gen<R, NP, NM>(hb, dv, ac, *x, mn);
            if (writes) {
#pragma unroll
                for (int kk = 0; kk < NM; ++kk) out[(NP + kk) * fs + o] = mn[kk];
            }
            return;
        }
#pragma unroll
        for (int kk = 0; kk < NM; ++kk) {
            const R jxh = lane_next(jxl[kk]);
            if (writes) {
                R chik = R(0);
#pragma unroll
                for (int b = 0; b < NP; ++b) chik += hb[b] * ac.chi[b][kk];
                const R div = (jxh - jxl[kk]) * ac.rdx + (jyhi[kk] - jylo[kk]) * ac.rdx;
                out[(NP + kk) * fs + o] = nm[1][kk] - (ac.dt * div) * fast_rcp(chik);
            }
            jylo[kk] = jyhi[kk];
        }
    };

    // Step rows r_first .. m1 (row m1 = ny at a no-flux edge is the mirror
    // copy); after the step of row r > m0 row r - 1 is corrected.  Loads and
    // stores share one counter, so the march waits for everything once per two
    // rows and issues the loads of the two rows after next right after the
    // wait, giving every load two rows of arithmetic to land in.
    auto one = [&](int row, RawT& raw) {
        if (bot && row == ny)
            mirror_row();
        else
            step(row, raw);
        if (row == m0)
            first_face();
        else if (row > m0)
            correct(row - 1);
    };
    RawT X1, X2, Y1, Y2;
    int r = r_first;
    load(r + 2, X1);
    load(r + 3, X2);
    while (true) {
        __builtin_amdgcn_s_waitcnt(kWaitVm0);
        load(r + 4, Y1);
        load(r + 5, Y2);
        one(r, X1);
        if (r++ == m1) break;
        one(r, X2);
        if (r++ == m1) break;
        __builtin_amdgcn_s_waitcnt(kWaitVm0);
        load(r + 4, X1);
        load(r + 5, X2);
        one(r, Y1);
        if (r++ == m1) break;
        one(r, Y2);
        if (r++ == m1) break;
    }
}

template <typename R, int NP, int NM, bool ANISO, bool OBST>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MP_WAVES_PER_EU)))
k_step2d_at(const R* __restrict__ in, R* __restrict__ out, Geom g, Coef<R> c, AtCoef<R> ac,
            const int64_t* __restrict__ stepctr, int kstep, double tb0, double tdn, double tslope,
            int seg, int ntx, int nseg) {
    const int wpb = blockDim.x >> 6;
    const int wid = __builtin_amdgcn_readfirstlane(xcd_block() * wpb + (threadIdx.x >> 6));
    if (wid >= ntx * nseg) return;
    const int tx = wid % ntx;
    const int sg = wid / ntx;
    const int m0 = sg * seg;
    const double tbase = tb0 + tdn * (double)(*stepctr + kstep);
    bool fixL, fixR;
    x2_column<1>(g, x2_first_col<1>(tx, threadIdx.x & 63), fixL, fixR);
    if (__ballot(fixL || fixR) != 0)
        strip2d_at<R, NP, NM, ANISO, OBST, true>(in, out, g, c, ac, tbase, tslope, tx, m0, min(m0 + seg, g.ny));
    else
        strip2d_at<R, NP, NM, ANISO, OBST, false>(in, out, g, c, ac, tbase, tslope, tx, m0, min(m0 + seg, g.ny));
}

// The extended model's general form: the same strip with the GEN arithmetic
// and the extended coefficients as a further argument.
template <typename R, int NP, int NM, bool ANISO, bool OBST>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MP_WAVES_PER_EU)))
k_step2d_at_gen(const R* __restrict__ in, R* __restrict__ out, Geom g, Coef<R> c, AtCoef<R> ac,
                const int64_t* __restrict__ stepctr, int kstep, double tb0, double tdn, double tslope,
                int seg, int ntx, int nseg, CoefX<R> x) {
    const int wpb = blockDim.x >> 6;
    const int wid = __builtin_amdgcn_readfirstlane(xcd_block() * wpb + (threadIdx.x >> 6));
    if (wid >= ntx * nseg) return;
    const int tx = wid % ntx;
    const int sg = wid / ntx;
    const int m0 = sg * seg;
    const double tbase = tb0 + tdn * (double)(*stepctr + kstep);
    bool fixL, fixR;
    x2_column<1>(g, x2_first_col<1>(tx, threadIdx.x & 63), fixL, fixR);
    if (__ballot(fixL || fixR) != 0)
        strip2d_at<R, NP, NM, ANISO, OBST, true, true>(in, out, g, c, ac, tbase, tslope, tx, m0,
                                                        min(m0 + seg, g.ny), &x);
    else
        strip2d_at<R, NP, NM, ANISO, OBST, false, true>(in, out, g, c, ac, tbase, tslope, tx, m0,
                                                         min(m0 + seg, g.ny), &x);
}

// GEN: the general kernel with the extended model's terms x (null otherwise).
template <typename R, int NP, int NM, bool ANISO, bool OBST, bool GEN>
int call_2d_at_v(const StepLaunch& L, const Coef<R>& c, const AtCoef<R>& ac, const CoefX<R>* x, KernelCall& k) {
    const int ntx = (L.g.nx + W2X_LANES_OUT - 1) / W2X_LANES_OUT;
    const int nseg = (L.g.ny + L.seg - 1) / L.seg;
    const int wpb = L.bx / 64;
    const long long waves = (long long)ntx * nseg;
    const long long nblocks = (waves + wpb - 1) / wpb;
    if (nblocks <= 0 || nblocks > 0x7fffffffLL || L.out1 || L.fuse != 1 || L.g.nz != 1) return MP_E_PARAM;
    if constexpr (GEN)
        k.func = (const void*)&k_step2d_at_gen<R, NP, NM, ANISO, OBST>;
    else
        k.func = (const void*)&k_step2d_at<R, NP, NM, ANISO, OBST>;
    k.grid = dim3((unsigned)nblocks);
    k.block = dim3(L.bx);
    k.arg((const R*)L.in);
    k.arg((R*)L.out);
    k.arg(L.g);
    k.arg(c);
    k.arg(ac);
    k.arg(L.stepctr);
    k.arg(L.kstep);
    k.arg(L.tb0);
    k.arg(L.tdn);
    k.arg(L.tslope);
    k.arg(L.seg);
    k.arg(ntx);
    k.arg(nseg);
    if constexpr (GEN) k.arg(*x);
    return MP_OK;
}

// (both obstacle projections of the general kernel share one instance: the choice is CoefX::proj)
template <typename R, int NP, int NM, bool GEN>
int call_2d_at_flags(const StepLaunch& L, const Coef<R>& c, const AtCoef<R>& ac, const CoefX<R>* x, KernelCall& k) {
    const bool obst = GEN ? L.potential != MP_WELL : L.potential == MP_OBSTACLE;
    if (L.aniso)
        return obst ? call_2d_at_v<R, NP, NM, true, true, GEN>(L, c, ac, x, k)
                    : call_2d_at_v<R, NP, NM, true, false, GEN>(L, c, ac, x, k);
    return obst ? call_2d_at_v<R, NP, NM, false, true, GEN>(L, c, ac, x, k)
                : call_2d_at_v<R, NP, NM, false, false, GEN>(L, c, ac, x, k);
}

template <typename R, bool GEN>
int call_step_at_any(const StepLaunch& L, const Coef<R>& c, const AtCoef<R>& ac, const CoefX<R>* x, KernelCall& k) {
    if (L.dim != 2) return MP_E_PARAM;
    if (L.nphases == 2 && L.nmu == 1) return call_2d_at_flags<R, 2, 1, GEN>(L, c, ac, x, k);
    if (L.nphases == 2 && L.nmu == 2) return call_2d_at_flags<R, 2, 2, GEN>(L, c, ac, x, k);
    if (L.nphases == 3 && L.nmu == 1) return call_2d_at_flags<R, 3, 1, GEN>(L, c, ac, x, k);
    if (L.nphases == 3 && L.nmu == 2) return call_2d_at_flags<R, 3, 2, GEN>(L, c, ac, x, k);
    return MP_E_PARAM;
}

// One 2D step with the current: the kernel instance for (N, K-1, anisotropy, potential).
template <typename R>
int call_step_at(const StepLaunch& L, const Coef<R>& c, const AtCoef<R>& ac, KernelCall& k) {
    return call_step_at_any<R, false>(L, c, ac, nullptr, k);
}

// The same for the extended model (the general kernels).
template <typename R>
int call_step_at_gen(const StepLaunch& L, const Coef<R>& c, const AtCoef<R>& ac, const CoefX<R>& x,
                     KernelCall& k) {
    return call_step_at_any<R, true>(L, c, ac, &x, k);
}

}  // namespace mp
