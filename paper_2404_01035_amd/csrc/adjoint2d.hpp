// Discrete adjoint of the 2D step (isotropic gradient energy, multi-well
// potential): lambda^n = (dF/ds^n)^T lambda^{n+1} and this step's share of the
// gradients in gamma_ab, D^a_k and tau.
//
// The step is a composition of cell terms and face terms, so its transpose
// has two parts:
//   part A (cell) recomputes the forward step at the cell (its four faces in
//     the forward direction) and runs the cell's own backward: the projection
//     of the Lagrange multiplier, the phase-change source and chi, the
//     potential and the driving force (with the second derivatives of h).  It
//     leaves the cotangents X of the cell's gradient term and flux divergence
//     (for the faces) and the cell-local part of lambda^n;
//   part B (faces) backpropagates every face (q_n, G_n, the flux F and source
//     s of the gradient term, the mu flux J) from the two cells' cotangents X
//     into both cells, then the mobility M_k = sum_a D^a_k chi^a_k h_a of each
//     cell.
// A face whose two cells coincide (zero-flux ghost, or a periodic axis one
// cell long) carries no flux and contributes nothing in either direction.
//
// Layout of the work: as in the forward strip kernel, one wave per column
// strip (lanes 1..62 own the strip's columns, lanes 0 and 63 hold the
// neighbouring columns) marches up a segment of rows.  Each face is evaluated
// once: an x face by the lane on its left, which hands the right cell's share
// to the next lane by a lane rotate; a y face by the row below it, which
// carries the upper cell's share to the next row in registers.  B of step n
// and A of step n-1 run in one pass (A needs lambda^n only at its own cell).
// Parameter gradients are accumulated per lane in FP64 over the rows, summed
// per block in a fixed order and added to that block's own accumulator row,
// so the result is deterministic.
#pragma once

#include "gp_device.hpp"

namespace mp {

// Plain (unfolded) coefficients of the adjoint.
template <typename R>
struct AdjCoef {
    R inv_dx, eps, inv_eps, kphi, dt;
    R ktau;        // dt / (tau^2 eps)
    R gam[3];      // gamma_ab by pair
    R w18[3];      // 18 gamma_ab by pair
    R gamma3;
    R chi[3][2], halfchi[3][2], B[3][2], C[3], s[3], Dchi[3][2];
};

constexpr int ADJ_NPAR = 10;  // gamma 01, 02, 12; D[a][k] (a < 3, k < 2); tau
constexpr int ADJ_W = 62;     // columns owned by a strip wave (lanes 1..62)
#ifndef MP_ADJ_WPB
#define MP_ADJ_WPB 4
#endif
constexpr int ADJ_WPB = MP_ADJ_WPB;  // waves per block

template <typename R, int NP>
__device__ __forceinline__ void h_of(const R (&p)[NP], R (&h)[NP]) {
    R e3x2 = R(0);  // 2 phi_a phi_b phi_c, the same for every phase
    if constexpr (NP == 3) e3x2 = R(2) * (p[0] * p[1] * p[2]);
#pragma unroll
    for (int a = 0; a < NP; ++a) h[a] = p[a] * p[a] * (R(3) - R(2) * p[a]) + e3x2;
}

// dh[b][a] = dh_b / dphi_a
template <typename R, int NP>
__device__ __forceinline__ void dh_of(const R (&p)[NP], R (&d)[NP][NP]) {
#pragma unroll
    for (int b = 0; b < NP; ++b)
#pragma unroll
        for (int a = 0; a < NP; ++a) {
            if (a == b) {
                R v = R(6) * p[b] - R(6) * p[b] * p[b];
                if constexpr (NP == 3) {
                    const int u = b == 0 ? 1 : 0, w = b == 2 ? 1 : 2;
                    v = v + R(2) * (p[u] * p[w]);
                }
                d[b][a] = v;
            } else {
                d[b][a] = NP == 3 ? R(2) * p[b] * p[3 - a - b] : R(0);
            }
        }
}

template <typename R, int NP, int NM>
__device__ __forceinline__ void mob_of(const R (&h)[NP], const AdjCoef<R>& c, R (&M)[NM]) {
#pragma unroll
    for (int k = 0; k < NM; ++k) {
        R m = R(0);
#pragma unroll
        for (int a = 0; a < NP; ++a) m = m + c.Dchi[a][k] * h[a];
        M[k] = m;
    }
}

// Forward face in plain form: F, S of the gradient term and J of the mu flux.
template <typename R, int NP, int NM>
__device__ __forceinline__ void face_fwd(const R (&pL)[NP], const R (&pR)[NP], const R (&ML)[NM],
                                         const R (&MR)[NM], const R (&uL)[NM], const R (&uR)[NM],
                                         const AdjCoef<R>& c, R (&F)[NP], R (&S)[NP], R (&J)[NM]) {
    R pb[NP], g[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        pb[a] = R(0.5) * (pL[a] + pR[a]);
        g[a] = (pR[a] - pL[a]) * c.inv_dx;
        F[a] = R(0);
        S[a] = R(0);
    }
#pragma unroll
    for (int i = 0; i < NP; ++i)
#pragma unroll
        for (int j = i + 1; j < NP; ++j) {
            const R qn = pb[i] * g[j] - pb[j] * g[i];
            const R gG = c.gam[pair_index(i, j)] * (R(2) * qn);
            F[i] = F[i] - gG * pb[j];
            F[j] = F[j] + gG * pb[i];
            S[i] = S[i] + gG * g[j];
            S[j] = S[j] - gG * g[i];
        }
#pragma unroll
    for (int k = 0; k < NM; ++k) J[k] = R(0.5) * (ML[k] + MR[k]) * (uR[k] - uL[k]) * c.inv_dx;
}

// Sum over the 64 lanes of a wave, complete in lane 63: DPP steps in a fixed
// pattern (pairs, quads, half rows, rows, then rows 0+1 into row 1 and rows
// 2+3 into row 3, then row 1 into row 3), so the rounding does not depend on
// timing.  Each step moves the two halves of the double and adds in FP64.
template <unsigned CTRL, unsigned ROWS>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double wave_sum_last(double x) {
    x = x + dpp_f64<0xB1, 0xF>(x);   // quad_perm [1,0,3,2]
    x = x + dpp_f64<0x4E, 0xF>(x);   // quad_perm [2,3,0,1]
    x = x + dpp_f64<0x141, 0xF>(x);  // row_half_mirror
    x = x + dpp_f64<0x140, 0xF>(x);  // row_mirror
    x = x + dpp_f64<0x142, 0xA>(x);  // row_bcast:15 into rows 1 and 3
    x = x + dpp_f64<0x143, 0xC>(x);  // row_bcast:31 into rows 2 and 3
    return x;
}

// Block-wide sums of the parameter terms, added to this block's accumulator
// row: the wave sums above, then the wave sums in wave order; B's slots
// (0..8) first, then A's (0, 1, 2, 9).  rowq: slot q of the row, read by lane
// q of the block's first wave at the kernel's start (no other block touches
// the row).
template <bool DOB, bool DOA>
__device__ __forceinline__ void adj_block_add(const double (&pb)[ADJ_NPAR], const double (&pa)[ADJ_NPAR],
                                              double rowq, double* __restrict__ acc) {
    constexpr int NB = DOB ? 9 : 0, NA = DOA ? 4 : 0;
    constexpr int SA[4] = {0, 1, 2, 9};
    __shared__ double red[ADJ_WPB][NB + NA];
    const int t = threadIdx.x;
    double w[NB + NA > 0 ? NB + NA : 1];
#pragma unroll
    for (int q = 0; q < NB; ++q) w[q] = wave_sum_last(pb[q]);
#pragma unroll
    for (int q = 0; q < NA; ++q) w[NB + q] = wave_sum_last(pa[SA[q]]);
    if ((t & 63) == 63)
#pragma unroll
        for (int q = 0; q < NB + NA; ++q) red[t >> 6][q] = w[q];
    __syncthreads();
    if (t < ADJ_NPAR) {
        double r = rowq;
        if (DOB && t < 9) {
            double sum = red[0][t];
#pragma unroll
            for (int k = 1; k < ADJ_WPB; ++k) sum = sum + red[k][t];
            r = r + sum;
        }
        if (DOA && (t < 3 || t == 9)) {
            const int j = NB + (t < 3 ? t : 3);
            double sum = red[0][j];
#pragma unroll
            for (int k = 1; k < ADJ_WPB; ++k) sum = sum + red[k][j];
            r = r + sum;
        }
        if ((DOB && t < 9) || (DOA && (t < 3 || t == 9))) acc[(size_t)blockIdx.x * ADJ_NPAR + t] = r;
    }
}


struct AdjGeom {
    int nx, ny;
    bool perx, pery;
    int64_t fs;
    int seg;  // rows per strip segment
};

// Rows per segment of the adjoint strips: long segments where the grid gives
// enough waves to fill the chip (about two per SIMD), short ones otherwise.
#ifndef MP_ADJ_WAVES
#define MP_ADJ_WAVES 1536
#endif
inline int adj_seg(int nx, int ny) {
    const long long ntx = (nx + ADJ_W - 1) / ADJ_W;
    const long long s = ntx * ny / MP_ADJ_WAVES;
    return s < 1 ? 1 : (s > 32 ? 32 : (int)s);
}

inline int adj_blocks(const AdjGeom& g) {
    const long long ntx = (g.nx + ADJ_W - 1) / ADJ_W;
    const long long nsg = (g.ny + g.seg - 1) / g.seg;
    return (int)((ntx * nsg + ADJ_WPB - 1) / ADJ_WPB);
}

// One face's backward.  A is the lower cell (smaller coordinate), B the
// upper; X are the cells' cotangents of the gradient term (NP) and flux
// divergence (NM).  lpA, luA / lpB, luB receive the face's share of lambda at
// A / B, lM the share of the mobility cotangent (the same for both cells), gp
// the face's gamma terms by pair.
template <typename R, int NP, int NM>
__device__ __forceinline__ void face_bwd(const R (&pA)[NP], const R (&pB)[NP], const R (&uA)[NM],
                                         const R (&uB)[NM], const R (&MA)[NM], const R (&MB)[NM],
                                         const R (&XA)[NP + NM], const R (&XB)[NP + NM], const AdjCoef<R>& c,
                                         R (&lpA)[NP], R (&lpB)[NP], R (&luA)[NM], R (&luB)[NM], R (&lM)[NM],
                                         R (&gp)[3]) {
    R pb[NP], g[NP], lF[NP], lS[NP], lpb[NP], lg[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        pb[a] = R(0.5) * (pA[a] + pB[a]);
        g[a] = (pB[a] - pA[a]) * c.inv_dx;
        lF[a] = (XA[a] - XB[a]) * c.inv_dx;
        lS[a] = -R(0.5) * (XA[a] + XB[a]);
        lpb[a] = R(0);
        lg[a] = R(0);
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) gp[q] = R(0);
#pragma unroll
    for (int i = 0; i < NP; ++i)
#pragma unroll
        for (int j = i + 1; j < NP; ++j) {
            const int pi = pair_index(i, j);
            const R qn = pb[i] * g[j] - pb[j] * g[i];
            const R Gn = R(2) * qn;
            const R gG = c.gam[pi] * Gn;
            const R lgG = -lF[i] * pb[j] + lF[j] * pb[i] + lS[i] * g[j] - lS[j] * g[i];
            lpb[j] = lpb[j] - lF[i] * gG;
            lpb[i] = lpb[i] + lF[j] * gG;
            lg[j] = lg[j] + lS[i] * gG;
            lg[i] = lg[i] - lS[j] * gG;
            gp[pi] = lgG * Gn;
            const R lqn = R(2) * c.gam[pi] * lgG;
            lpb[i] = lpb[i] + lqn * g[j];
            lg[j] = lg[j] + lqn * pb[i];
            lpb[j] = lpb[j] - lqn * g[i];
            lg[i] = lg[i] - lqn * pb[j];
        }
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        lpA[a] = R(0.5) * lpb[a] - lg[a] * c.inv_dx;
        lpB[a] = R(0.5) * lpb[a] + lg[a] * c.inv_dx;
    }
#pragma unroll
    for (int k = 0; k < NM; ++k) {
        const R lJ = (XA[NP + k] - XB[NP + k]) * c.inv_dx;
        lM[k] = lJ * R(0.5) * (uB[k] - uA[k]) * c.inv_dx;
        const R lu = lJ * R(0.5) * (MA[k] + MB[k]) * c.inv_dx;
        luA[k] = -lu;
        luB[k] = lu;
    }
}

// Part A's backward at one cell (phi, mu, h(phi)) from the forward step's gradient term grad
// and flux divergence divJ there.  l1in = lambda^{n+1} at the cell; Xo
// receives [lambda of grad_a (NP)][lambda of divJ_k (NM)], lo the cell-local
// part of lambda^n; par collects the cell's gamma (potential) and tau terms.
template <typename R, int NP, int NM>
__device__ __forceinline__ void adj_cell_back(const R (&phi)[NP], const R (&mu)[NM], const R (&hphi)[NP],
                                              const R (&grad)[NP], const R (&divJ)[NM], const AdjCoef<R>& c, R ttc,
                                              const R (&l1in)[NP + NM], R (&Xo)[NP + NM], R (&lo)[NP + NM],
                                              double (&par)[ADJ_NPAR]) {
    const R tt = ttc;
    R dmu[NP][NM], psi[NP];
#pragma unroll
    for (int b = 0; b < NP; ++b) {
        R v = c.C[b] + c.s[b] * tt;
#pragma unroll
        for (int k = 0; k < NM; ++k) {
            dmu[b][k] = mu[k] - c.B[b][k];
            v = v - c.halfchi[b][k] * dmu[b][k] * dmu[b][k];
        }
        psi[b] = v;
    }
    R P[NP];
    R psum = R(0);
    if constexpr (NP == 3) {
        P[0] = phi[1] * phi[2];
        P[1] = phi[0] * phi[2];
        P[2] = phi[0] * phi[1];
        psum = psi[0] + psi[1] + psi[2];
    }
    R Rr[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        R dw = R(0);
#pragma unroll
        for (int b = 0; b < NP; ++b)
            if (b != a) dw = dw + c.w18[pair_index(a < b ? a : b, a < b ? b : a)] * phi[b] * phi[b];
        dw = dw * phi[a];
        R dps = R(6) * psi[a] * (phi[a] * (R(1) - phi[a]));
        if constexpr (NP == 3) {
            dw = dw + c.gamma3 * P[a];
            dps = dps + R(2) * P[a] * psum;
        }
        Rr[a] = c.eps * grad[a] - c.inv_eps * dw - dps;
    }
    double lam = 0.0;
#pragma unroll
    for (int a = 0; a < NP; ++a) lam = lam + (double)Rr[a];
    lam = lam * (1.0 / NP);
    R dR[NP], phin[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        dR[a] = (R)((double)Rr[a] - lam);
        phin[a] = phi[a] + c.kphi * dR[a];
    }
    R h0[NP], h1[NP], dh0[NP][NP], dh1[NP][NP];
    R phi0[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) phi0[a] = phi[a];
#pragma unroll
    for (int a = 0; a < NP; ++a) h0[a] = hphi[a];
    h_of<R, NP>(phin, h1);
    dh_of<R, NP>(phi0, dh0);
    dh_of<R, NP>(phin, dh1);

    // ---- mu update -------------------------------------------------------
    R lmu[NM], ldiv[NM], lh1[NP], lh0[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        lh1[a] = R(0);
        lh0[a] = R(0);
    }
#pragma unroll
    for (int k = 0; k < NM; ++k) {
        R src = R(0), chik = R(0);
#pragma unroll
        for (int b = 0; b < NP; ++b) {
            src = src + (dmu[b][k] * c.chi[b][k]) * (h1[b] - h0[b]);
            chik = chik + h1[b] * c.chi[b][k];
        }
        const R Q = c.dt * divJ[k] - src;
        const R l1 = l1in[NP + k];
        const R r = fast_rcp(chik);
        const R lQ = l1 * r;
        const R lchi = -l1 * Q * r * r;
        ldiv[k] = c.dt * lQ;
        const R lsrc = -lQ;
        R lm = l1;
#pragma unroll
        for (int b = 0; b < NP; ++b) {
            const R cab = dmu[b][k] * c.chi[b][k];
            lh1[b] = lh1[b] + lsrc * cab + lchi * c.chi[b][k];
            lh0[b] = lh0[b] - lsrc * cab;
            lm = lm + lsrc * (h1[b] - h0[b]) * c.chi[b][k];
        }
        lmu[k] = lm;
    }

    // ---- phi update ------------------------------------------------------
    R lphin[NP], lphi[NP];
    R lmean = R(0);
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        R v = l1in[a];
#pragma unroll
        for (int b = 0; b < NP; ++b) v = v + lh1[b] * dh1[b][a];
        lphin[a] = v;
        lmean = lmean + v;
    }
    lmean = lmean * (R(1) / R(NP));
    R lR[NP];
    double gtau = 0.0;
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        R v = lphin[a];
#pragma unroll
        for (int b = 0; b < NP; ++b) v = v + lh0[b] * dh0[b][a];
        lphi[a] = v;
        lR[a] = c.kphi * (lphin[a] - lmean);
        gtau -= (double)(c.ktau * lphin[a] * dR[a]);
    }
    par[9] += gtau;
    // potential
#pragma unroll
    for (int cc = 0; cc < NP; ++cc)
#pragma unroll
        for (int a = 0; a < NP; ++a) {
            R d;
            if (a == cc) {
                d = R(0);
#pragma unroll
                for (int b = 0; b < NP; ++b)
                    if (b != cc) d = d + c.w18[pair_index(cc < b ? cc : b, cc < b ? b : cc)] * phi[b] * phi[b];
            } else {
                d = R(2) * c.w18[pair_index(cc < a ? cc : a, cc < a ? a : cc)] * phi[cc] * phi[a];
                if constexpr (NP == 3) d = d + c.gamma3 * phi[3 - a - cc];
            }
            lphi[a] = lphi[a] - lR[cc] * c.inv_eps * d;
        }
#pragma unroll
    for (int cc = 0; cc < NP; ++cc)
#pragma unroll
        for (int b = 0; b < NP; ++b)
            if (b != cc)
                par[pair_index(cc < b ? cc : b, cc < b ? b : cc)] -=
                    (double)(lR[cc] * c.inv_eps * R(18) * phi[cc] * phi[b] * phi[b]);
    // driving force sum_b psi_b dh_b/dphi_c, differentiated in phi and psi
#pragma unroll
    for (int cc = 0; cc < NP; ++cc)
#pragma unroll
        for (int a = 0; a < NP; ++a) {
            R d = a == cc ? R(6) * psi[cc] * (R(1) - R(2) * phi[cc]) : R(0);
            if constexpr (NP == 3)
                if (a != cc) d = R(2) * phi[3 - a - cc] * psum;
            lphi[a] = lphi[a] - lR[cc] * d;
        }
#pragma unroll
    for (int b = 0; b < NP; ++b) {
        R lpsi = R(0);
#pragma unroll
        for (int cc = 0; cc < NP; ++cc) lpsi = lpsi - lR[cc] * dh0[b][cc];
#pragma unroll
        for (int k = 0; k < NM; ++k) lmu[k] = lmu[k] - lpsi * (dmu[b][k] * c.chi[b][k]);
    }

#pragma unroll
    for (int a = 0; a < NP; ++a) {
        Xo[a] = c.eps * lR[a];
        lo[a] = lphi[a];
    }
#pragma unroll
    for (int k = 0; k < NM; ++k) {
        Xo[NP + k] = ldiv[k];
        lo[NP + k] = lmu[k];
    }
}


// A cell of one row of a state: phi, mu, the mobility and h(phi).
template <typename R, int NP, int NM>
struct ACell {
    R phi[NP], mu[NM], M[NM], h[NP];
};

template <typename R, int NP, int NM>
__device__ __forceinline__ void adj_fetch(const R* __restrict__ s, int64_t fs, int64_t o, ACell<R, NP, NM>& q) {
#pragma unroll
    for (int a = 0; a < NP; ++a) q.phi[a] = s[a * fs + o];
#pragma unroll
    for (int k = 0; k < NM; ++k) q.mu[k] = s[(NP + k) * fs + o];
}

// The cell's h and mobility, once its phi is in.
template <typename R, int NP, int NM>
__device__ __forceinline__ void adj_finish(const AdjCoef<R>& c, ACell<R, NP, NM>& q) {
    h_of<R, NP>(q.phi, q.h);
    mob_of<R, NP, NM>(q.h, c, q.M);
}

template <typename R, int NP, int NM>
__device__ __forceinline__ void adj_load(const R* __restrict__ s, int64_t fs, int64_t o, const AdjCoef<R>& c,
                                         ACell<R, NP, NM>& q) {
    adj_fetch<R, NP, NM>(s, fs, o, q);
    adj_finish<R, NP, NM>(c, q);
}

// Adjoint strip kernel.  DOB: part B of step n (sB = s^n, XB = part A's
// cotangents of step n); DOA: part A at sA (step n-1 when fused, else the
// step itself), writing its cotangents to XA.  lam: lambda, updated in place
// at each owned cell (A alone: lambda^{n+1} in, the cell-local part out; B
// alone: that part in, lambda^n out; both: lambda^{n+1} in, step n-1's
// cell-local part out).  The two parts' parameter sums are added B first, as
// separate launches add them.
#ifndef MP_ADJ_WAVES_PER_EU
#define MP_ADJ_WAVES_PER_EU 2
#endif
template <typename R, int NP, int NM, bool DOA, bool DOB>
__global__ void __launch_bounds__(64 * ADJ_WPB) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? MP_ADJ_WAVES_PER_EU : 1)))
k_adj_strip(const R* __restrict__ sB, const R* __restrict__ XB, const R* __restrict__ sA, R* __restrict__ XA,
            R* __restrict__ lam, AdjGeom G, AdjCoef<R> c, double tt_row0, double tt_slope,
            double* __restrict__ acc) {
    constexpr int NF = NP + NM;
    typedef ACell<R, NP, NM> Cell;
    double parB[ADJ_NPAR], parA[ADJ_NPAR];
#pragma unroll
    for (int q = 0; q < ADJ_NPAR; ++q) {
        parB[q] = 0.0;
        parA[q] = 0.0;
    }
    // part B adds to slots 0..8 and part A to 0, 1, 2, 9 of this block's
    // accumulator row; its old values are read now, used at the end
    double rowq = 0.0;
    if (threadIdx.x < ADJ_NPAR) rowq = acc[(size_t)blockIdx.x * ADJ_NPAR + threadIdx.x];
    const int lane = threadIdx.x & 63;
    const int ntx = (G.nx + ADJ_W - 1) / ADJ_W;
    const int nsg = (G.ny + G.seg - 1) / G.seg;
    // wave-uniform by construction
    const int wid = __builtin_amdgcn_readfirstlane(blockIdx.x * ADJ_WPB + (int)(threadIdx.x >> 6));
    if (wid < ntx * nsg) {
        const int tx = wid % ntx;
        const int m0 = (wid / ntx) * G.seg;
        const int m1 = min(m0 + G.seg, G.ny);
        const int nx = G.nx, ny = G.ny;
        const int64_t fs = G.fs;
        const int cs = tx * ADJ_W - 1 + lane;  // this lane's column
        // loaded column: wrapped, or (zero-flux) the ghost columns -1 and nx as
        // copies of 0 and nx-1; farther out clamped (never owned)
        const int col = G.perx ? wrap(cs, nx) : (cs < 0 ? 0 : (cs >= nx ? nx - 1 : cs));
        const bool xsame = col == rot_next(col);  // face (lane, lane+1) joins a cell with itself
        const bool own = lane >= 1 && lane <= ADJ_W && cs < nx;
        // row index of rows m0-1 .. m1+1 (selects, no branches: periodic rows
        // lie within one period plus two rows of the grid)
        auto rowmap = [&](int r) {
            int w = r >= ny ? r - ny : r;
            w = w >= ny ? w - ny : w;
            w = w < 0 ? w + ny : w;
            const int cl = r < 0 ? 0 : (r >= ny ? ny - 1 : r);
            return G.pery ? w : cl;
        };
        auto at = [&](int r) { return (int64_t)rowmap(r) * nx + col; };
        auto ldX = [&](int r, R (&x)[NF]) {
            const int64_t o = at(r);
#pragma unroll
            for (int f = 0; f < NF; ++f) x[f] = XB[f * fs + o];
        };

        // rows m and m+1: B's state and cotangents, A's state
        Cell b0, b1, a0, a1;
        R x0[NF], x1[NF];
        // carries from the face (m-1, m): B's share for the upper cell, A's
        // forward F, S, J
        R cpB[NP], cuB[NM], cMB[NM], cF[NP], cS[NP], cJ[NM];
        {
            const bool ysame = rowmap(m0 - 1) == rowmap(m0);
            Cell bl, al;
            R xl[NF];
            if constexpr (DOB) {
                adj_fetch<R, NP, NM>(sB, fs, at(m0 - 1), bl);
                adj_fetch<R, NP, NM>(sB, fs, at(m0), b0);
                adj_fetch<R, NP, NM>(sB, fs, at(m0 + 1), b1);
                ldX(m0 - 1, xl);
                ldX(m0, x0);
                ldX(m0 + 1, x1);
            }
            if constexpr (DOA) {
                adj_fetch<R, NP, NM>(sA, fs, at(m0 - 1), al);
                adj_fetch<R, NP, NM>(sA, fs, at(m0), a0);
                adj_fetch<R, NP, NM>(sA, fs, at(m0 + 1), a1);
            }
            if constexpr (DOB) {
                adj_finish<R, NP, NM>(c, bl);
                adj_finish<R, NP, NM>(c, b0);
                adj_finish<R, NP, NM>(c, b1);
                R lpA[NP], luA[NM];
                R gp[3];
                face_bwd<R, NP, NM>(bl.phi, b0.phi, bl.mu, b0.mu, bl.M, b0.M, xl, x0, c, lpA, cpB, luA, cuB, cMB,
                                    gp);
                if (ysame) {
#pragma unroll
                    for (int a = 0; a < NP; ++a) cpB[a] = R(0);
#pragma unroll
                    for (int k = 0; k < NM; ++k) cuB[k] = cMB[k] = R(0);
                }
            }
            if constexpr (DOA) {
                adj_finish<R, NP, NM>(c, al);
                adj_finish<R, NP, NM>(c, a0);
                adj_finish<R, NP, NM>(c, a1);
                // a face between a cell and its copy has no flux: F, S, J vanish
                face_fwd<R, NP, NM>(al.phi, a0.phi, al.M, a0.M, al.mu, a0.mu, c, cF, cS, cJ);
            }
        }

        // Row m with rows m, m+1 in (b0, b1), (x0, x1), (a0, a1); row m+2 is
        // then loaded into the row-m slots, so that consecutive rows swap the
        // roles of the two slots instead of copying records.
        auto row = [&](int m, Cell& b0, Cell& b1, R (&x0)[NF], R (&x1)[NF], Cell& a0, Cell& a1) {
            const int64_t o = (int64_t)m * nx + cs;  // the owned cell (own lanes only)
            const bool ysame = rowmap(m) == rowmap(m + 1);
            R lv[NF];  // lambda at the cell (used at owned cells only)
            {
                const int64_t oc = at(m);  // = o at owned cells, in bounds elsewhere
#pragma unroll
                for (int f = 0; f < NF; ++f) lv[f] = lam[f * fs + oc];
            }
            R lf[NF];
            if constexpr (DOB) {
                // x face (lane, lane+1)
                R pR[NP], uR[NM], MR[NM], XR[NF];
#pragma unroll
                for (int a = 0; a < NP; ++a) pR[a] = lane_next(b0.phi[a]);
#pragma unroll
                for (int k = 0; k < NM; ++k) {
                    uR[k] = lane_next(b0.mu[k]);
                    MR[k] = lane_next(b0.M[k]);
                }
#pragma unroll
                for (int f = 0; f < NF; ++f) XR[f] = lane_next(x0[f]);
                R lpx[NP], lpxR[NP], lux[NM], luxR[NM], lMx[NM];
                R gpx[3];
                face_bwd<R, NP, NM>(b0.phi, pR, b0.mu, uR, b0.M, MR, x0, XR, c, lpx, lpxR, lux, luxR, lMx, gpx);
                const R xm = xsame ? R(0) : R(1);  // mask: see the y face below
#pragma unroll
                for (int a = 0; a < NP; ++a) {
                    lpx[a] = lpx[a] * xm;
                    lpxR[a] = lpxR[a] * xm;
                }
#pragma unroll
                for (int k = 0; k < NM; ++k) {
                    lux[k] = lux[k] * xm;
                    luxR[k] = luxR[k] * xm;
                    lMx[k] = lMx[k] * xm;
                }
#pragma unroll
                for (int q = 0; q < 3; ++q) gpx[q] = gpx[q] * xm;
                // y face (m, m+1)
                R lpy[NP], lpyU[NP], luy[NM], luyU[NM], lMy[NM];
                R gpy[3];
                face_bwd<R, NP, NM>(b0.phi, b1.phi, b0.mu, b1.mu, b0.M, b1.M, x0, x1, c, lpy, lpyU, luy, luyU, lMy,
                                    gpy);
                // masks multiply (a select would let the compiler branch around the
                // face, splitting the row body the scheduler interleaves)
                const R ym = ysame ? R(0) : R(1);
#pragma unroll
                for (int a = 0; a < NP; ++a) {
                    lpy[a] = lpy[a] * ym;
                    lpyU[a] = lpyU[a] * ym;
                }
#pragma unroll
                for (int k = 0; k < NM; ++k) {
                    luy[k] = luy[k] * ym;
                    luyU[k] = luyU[k] * ym;
                    lMy[k] = lMy[k] * ym;
                }
#pragma unroll
                for (int q = 0; q < 3; ++q) gpy[q] = gpy[q] * ym;
                // the cell's four faces: x-hi (own), x-lo (from the previous
                // lane), y-hi (own), y-lo (carried)
                R lphi[NP], lmu[NM], lM[NM];
#pragma unroll
                for (int a = 0; a < NP; ++a) lphi[a] = (lpx[a] + lane_prev(lpxR[a])) + (lpy[a] + cpB[a]);
#pragma unroll
                for (int k = 0; k < NM; ++k) {
                    lmu[k] = (lux[k] + lane_prev(luxR[k])) + (luy[k] + cuB[k]);
                    lM[k] = (lMx[k] + lane_prev(lMx[k])) + (lMy[k] + cMB[k]);
                }
                // mobility M_k = sum_b D_bk chi_bk h_b(phi)
                const R(&hi)[NP] = b0.h;
                R dhi[NP][NP];
                dh_of<R, NP>(b0.phi, dhi);
                if (own) {
#pragma unroll
                    for (int q = 0; q < 3; ++q) parB[q] += (double)gpx[q] + (double)gpy[q];
#pragma unroll
                    for (int k = 0; k < NM; ++k)
#pragma unroll
                        for (int b = 0; b < NP; ++b)
                            parB[3 + 2 * b + k] += (double)(lM[k] * c.chi[b][k] * hi[b]);
                }
#pragma unroll
                for (int k = 0; k < NM; ++k)
#pragma unroll
                    for (int b = 0; b < NP; ++b)
#pragma unroll
                        for (int a = 0; a < NP; ++a) lphi[a] = lphi[a] + lM[k] * c.Dchi[b][k] * dhi[b][a];
#pragma unroll
                for (int a = 0; a < NP; ++a) {
                    lf[a] = lphi[a];
                    cpB[a] = lpyU[a];
                }
#pragma unroll
                for (int k = 0; k < NM; ++k) {
                    lf[NP + k] = lmu[k];
                    cuB[k] = luyU[k];
                    cMB[k] = lMy[k];
                }
                // row m's slots are free: row m+2 is fetched into them while
                // part A runs
                // (past the segment's last row the clamped rows go unused)
                adj_fetch<R, NP, NM>(sB, fs, at(m + 2), b0);
                ldX(m + 2, x0);
            }
            if constexpr (DOA) {
                // forward faces of sA: x-hi here, x-lo from the previous lane,
                // y-hi here, y-lo carried
                R pR[NP], uR[NM], MR[NM];
#pragma unroll
                for (int a = 0; a < NP; ++a) pR[a] = lane_next(a0.phi[a]);
#pragma unroll
                for (int k = 0; k < NM; ++k) {
                    uR[k] = lane_next(a0.mu[k]);
                    MR[k] = lane_next(a0.M[k]);
                }
                R Fx[NP], Sx[NP], Jx[NM], Fy[NP], Sy[NP], Jy[NM];
                face_fwd<R, NP, NM>(a0.phi, pR, a0.M, MR, a0.mu, uR, c, Fx, Sx, Jx);
                face_fwd<R, NP, NM>(a0.phi, a1.phi, a0.M, a1.M, a0.mu, a1.mu, c, Fy, Sy, Jy);
                R grad[NP], divJ[NM];
#pragma unroll
                for (int a = 0; a < NP; ++a) {
                    const R Fl = lane_prev(Fx[a]), Sl = lane_prev(Sx[a]);
                    grad[a] = ((Fx[a] - Fl) * c.inv_dx - R(0.5) * (Sx[a] + Sl)) +
                              ((Fy[a] - cF[a]) * c.inv_dx - R(0.5) * (Sy[a] + cS[a]));
                    cF[a] = Fy[a];
                    cS[a] = Sy[a];
                }
#pragma unroll
                for (int k = 0; k < NM; ++k) {
                    const R Jl = lane_prev(Jx[k]);
                    divJ[k] = (Jx[k] - Jl) * c.inv_dx + (Jy[k] - cJ[k]) * c.inv_dx;
                    cJ[k] = Jy[k];
                }
                R ph[NP], mu[NM], hA[NP];
#pragma unroll
                for (int a = 0; a < NP; ++a) {
                    ph[a] = a0.phi[a];
                    hA[a] = a0.h[a];
                }
#pragma unroll
                for (int k = 0; k < NM; ++k) mu[k] = a0.mu[k];
                adj_fetch<R, NP, NM>(sA, fs, at(m + 2), a0);
                R l1[NF], Xo[NF], lo[NF];
#pragma unroll
                for (int f = 0; f < NF; ++f) l1[f] = lv[f];
                if constexpr (DOB)
#pragma unroll
                    for (int f = 0; f < NF; ++f) l1[f] = l1[f] + lf[f];
                double pc[ADJ_NPAR];
#pragma unroll
                for (int q = 0; q < ADJ_NPAR; ++q) pc[q] = 0.0;
                adj_cell_back<R, NP, NM>(ph, mu, hA, grad, divJ, c, (R)(tt_row0 + tt_slope * (double)m), l1, Xo,
                                         lo, pc);
                if (own) {
#pragma unroll
                    for (int q = 0; q < ADJ_NPAR; ++q) parA[q] += pc[q];
#pragma unroll
                    for (int f = 0; f < NF; ++f) {
                        XA[f * fs + o] = Xo[f];
                        lam[f * fs + o] = lo[f];
                    }
                }
            } else {
                if (own)
#pragma unroll
                    for (int f = 0; f < NF; ++f) lam[f * fs + o] = lv[f] + lf[f];
            }
            // the window moves up one row: row m+2's mobilities
            if constexpr (DOB) adj_finish<R, NP, NM>(c, b0);
            if constexpr (DOA) adj_finish<R, NP, NM>(c, a0);
        };
        int m = m0;
        for (; m + 1 < m1; m += 2) {
            row(m, b0, b1, x0, x1, a0, a1);
            row(m + 1, b1, b0, x1, x0, a1, a0);
        }
        if (m < m1) row(m, b0, b1, x0, x1, a0, a1);
    }
    adj_block_add<DOB, DOA>(parB, parA, rowq, acc);
}

// One adjoint launch: part A of a step (which = 0), part B (which = 1) or
// part B of step n with part A of step n-1 (which = 2).
struct AdjLaunch {
    int which;
    const void* sB;    // s^n for part B
    const void* XB;    // part A's cotangents of step n, for part B
    const void* sA;    // the state part A differentiates at
    void* XA;          // receives part A's cotangents
    void* lam;         // lambda, updated in place
    AdjGeom g;
    int nphases, nmu;
    double tt_row0, tt_slope;  // T - Te at row j for part A's step: tt_row0 + tt_slope * j
    double* acc;               // per-block parameter accumulators
};

template <typename R, int NP, int NM>
int adj_launch_t(const AdjLaunch& L, const AdjCoef<R>& c, hipStream_t st) {
    const int nb = adj_blocks(L.g);
    const dim3 grid(nb), block(64 * ADJ_WPB);
    if (L.which == 0)
        hipLaunchKernelGGL((k_adj_strip<R, NP, NM, true, false>), grid, block, 0, st, nullptr, nullptr,
                           (const R*)L.sA, (R*)L.XA, (R*)L.lam, L.g, c, L.tt_row0, L.tt_slope, L.acc);
    else if (L.which == 1)
        hipLaunchKernelGGL((k_adj_strip<R, NP, NM, false, true>), grid, block, 0, st, (const R*)L.sB,
                           (const R*)L.XB, nullptr, nullptr, (R*)L.lam, L.g, c, L.tt_row0, L.tt_slope, L.acc);
    else
        hipLaunchKernelGGL((k_adj_strip<R, NP, NM, true, true>), grid, block, 0, st, (const R*)L.sB,
                           (const R*)L.XB, (const R*)L.sA, (R*)L.XA, (R*)L.lam, L.g, c, L.tt_row0, L.tt_slope,
                           L.acc);
    return MP_OK;
}

template <typename R>
int adj_launch(const AdjLaunch& L, const AdjCoef<R>& c, hipStream_t st) {
    if (L.nphases == 2 && L.nmu == 1) return adj_launch_t<R, 2, 1>(L, c, st);
    if (L.nphases == 2 && L.nmu == 2) return adj_launch_t<R, 2, 2>(L, c, st);
    if (L.nphases == 3 && L.nmu == 1) return adj_launch_t<R, 3, 1>(L, c, st);
    if (L.nphases == 3 && L.nmu == 2) return adj_launch_t<R, 3, 2>(L, c, st);
    return MP_E_PARAM;
}

}  // namespace mp
