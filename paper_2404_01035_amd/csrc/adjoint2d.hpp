// Discrete adjoint of the 2D step (isotropic gradient energy, multi-well
// potential): lambda^n = (dF/ds^n)^T lambda^{n+1} and this step's share of the
// gradients in gamma_ab, D^a_k and tau.
//
// The step is a composition of cell terms and face terms, so its transpose
// runs in two passes over the cells:
//   pass A (one thread per cell) recomputes the forward step at the cell and
//     runs the cell's own backward: the projection of the Lagrange
//     multiplier, the phase-change source and chi, the potential and the
//     driving force (with the second derivatives of h).  It leaves the
//     cotangents of the cell's gradient term and flux divergence (for the
//     faces) and the cell-local part of lambda^n;
//   pass B (one thread per cell) walks the cell's faces, backpropagates each
//     face (q_n, G_n, the flux F and source s of the gradient term, the mu flux
//     J) from the two cells' cotangents, keeps the contributions that land on
//     its own cell, and finishes with the mobility M_k = sum_a D^a_k chi^a_k h_a.
// A face whose two cells coincide (zero-flux ghost, or a periodic axis one
// cell long) carries no flux and contributes nothing in either direction.
// Parameter gradients are reduced per block in FP64 and added to that block's
// own accumulator row, so the result is deterministic.  Inside a segment of
// recomputed states, pass B of step n and pass A of step n-1 run as one
// kernel (pass A needs lambda^n only at its own cell).
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
constexpr int ADJ_BX = 64, ADJ_BY = 4;

template <typename R, int NP>
__device__ __forceinline__ void h_of(const R (&p)[NP], R (&h)[NP]) {
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        h[a] = R(3) * p[a] * p[a] - R(2) * p[a] * p[a] * p[a];
        if constexpr (NP == 3) {
            const int b = a == 0 ? 1 : 0, g = a == 2 ? 1 : 2;
            h[a] = h[a] + R(2) * p[a] * (p[b] * p[g]);
        }
    }
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

// Block-wide sum of the slots `idx` of v, added to this block's accumulator
// row: a fixed xor butterfly inside each wave, then the four wave sums in
// wave order, so the result does not depend on timing.
template <int NS>
__device__ __forceinline__ void adj_block_add(const int (&idx)[NS], const double (&v)[ADJ_NPAR],
                                              double* __restrict__ acc) {
    __shared__ double red[ADJ_BX * ADJ_BY / 64][NS];
    const int t = threadIdx.x;
    double w[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        double x = v[idx[q]];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) x = x + __shfl_xor(x, m, 64);
        w[q] = x;
    }
    if ((t & 63) == 0)
#pragma unroll
        for (int q = 0; q < NS; ++q) red[t >> 6][q] = w[q];
    __syncthreads();
    if (t == 0) {
        double* row = acc + (size_t)blockIdx.x * ADJ_NPAR;
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            double sum = red[0][q];
#pragma unroll
            for (int k = 1; k < ADJ_BX * ADJ_BY / 64; ++k) sum = sum + red[k][q];
            row[idx[q]] = row[idx[q]] + sum;
        }
    }
    __syncthreads();  // red may be reused by a second call in the same kernel
}

// Parameter slots each pass touches: A the potential's gamma and tau, B the
// gradient term's gamma and the mobilities.
constexpr int ADJ_SLOTS_A[4] = {0, 1, 2, 9};
constexpr int ADJ_SLOTS_B[9] = {0, 1, 2, 3, 4, 5, 6, 7, 8};

struct AdjGeom {
    int nx, ny;
    bool perx, pery;
    int64_t fs;
};

__device__ __forceinline__ int64_t cell_at(const AdjGeom& G, int x, int y) {
    return (int64_t)gmap(y, G.ny, G.pery) * G.nx + gmap(x, G.nx, G.perx);
}

template <typename R, int NP, int NM>
__device__ __forceinline__ void load_cell(const R* __restrict__ s, int64_t fs, int64_t o, R (&phi)[NP],
                                          R (&mu)[NM]) {
#pragma unroll
    for (int a = 0; a < NP; ++a) phi[a] = s[a * fs + o];
#pragma unroll
    for (int k = 0; k < NM; ++k) mu[k] = s[(NP + k) * fs + o];
}

// Pass A at cell (x, y), o = its offset: the forward step recomputed at the
// cell, then the cell's own backward.  l1in = lambda^{n+1} at the cell; Xo
// receives [lambda of grad_a (NP)][lambda of divJ_k (NM)], lo the cell-local
// part of lambda^n; par collects this cell's gamma (potential) and tau terms.
template <typename R, int NP, int NM>
__device__ __forceinline__ void adj_pass_a(const R* __restrict__ s, int x, int y, int64_t o,
                                           const AdjGeom& G, const AdjCoef<R>& c, R ttc,
                                           const R (&l1in)[NP + NM], R (&Xo)[NP + NM],
                                           R (&lo)[NP + NM], double (&par)[ADJ_NPAR]) {
    const int64_t fs = G.fs;
    // the cell and its four neighbours: 0 centre, 1 x-, 2 x+, 3 y-, 4 y+
    const int64_t on[5] = {o, cell_at(G, x - 1, y), cell_at(G, x + 1, y), cell_at(G, x, y - 1),
                           cell_at(G, x, y + 1)};
    R ph[5][NP], uu[5][NM], MM[5][NM];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        load_cell<R, NP, NM>(s, fs, on[q], ph[q], uu[q]);
        R hq[NP];
        h_of<R, NP>(ph[q], hq);
        mob_of<R, NP, NM>(hq, c, MM[q]);
    }
    R grad[NP], divJ[NM];
    {
        R Fl[NP], Sl[NP], Jl[NM], Fh[NP], Sh[NP], Jh[NM];
        face_fwd<R, NP, NM>(ph[1], ph[0], MM[1], MM[0], uu[1], uu[0], c, Fl, Sl, Jl);
        face_fwd<R, NP, NM>(ph[0], ph[2], MM[0], MM[2], uu[0], uu[2], c, Fh, Sh, Jh);
#pragma unroll
        for (int a = 0; a < NP; ++a) grad[a] = (Fh[a] - Fl[a]) * c.inv_dx - R(0.5) * (Sh[a] + Sl[a]);
#pragma unroll
        for (int k = 0; k < NM; ++k) divJ[k] = (Jh[k] - Jl[k]) * c.inv_dx;
        face_fwd<R, NP, NM>(ph[3], ph[0], MM[3], MM[0], uu[3], uu[0], c, Fl, Sl, Jl);
        face_fwd<R, NP, NM>(ph[0], ph[4], MM[0], MM[4], uu[0], uu[4], c, Fh, Sh, Jh);
#pragma unroll
        for (int a = 0; a < NP; ++a)
            grad[a] = grad[a] + ((Fh[a] - Fl[a]) * c.inv_dx - R(0.5) * (Sh[a] + Sl[a]));
#pragma unroll
        for (int k = 0; k < NM; ++k) divJ[k] = divJ[k] + (Jh[k] - Jl[k]) * c.inv_dx;
    }
    const R* phi = ph[0];
    const R* mu = uu[0];
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
    lam = lam / NP;
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
    h_of<R, NP>(phi0, h0);
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
        const R r = R(1) / chik;
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
    lmean = lmean / R(NP);
    R lR[NP];
    double gtau = 0.0;
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        R v = lphin[a];
#pragma unroll
        for (int b = 0; b < NP; ++b) v = v + lh0[b] * dh0[b][a];
        lphi[a] = v;
        lR[a] = c.kphi * (lphin[a] - lmean);
        gtau -= (double)c.ktau * (double)lphin[a] * (double)dR[a];
    }
    par[9] = gtau;
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
                    (double)lR[cc] * (double)c.inv_eps * 18.0 * (double)phi[cc] * (double)phi[b] *
                    (double)phi[b];
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

// Pass B at cell (x, y): the backward of the cell's four faces (from the
// cotangents X of pass A at the cell and its neighbours) and of its mobility.
// lf receives the faces' and mobility's share of lambda^n at the cell; par
// collects the gradient-term gamma and mobility terms.
template <typename R, int NP, int NM>
__device__ __forceinline__ void adj_pass_b(const R* __restrict__ s, const R* __restrict__ X, int x, int y,
                                           int64_t o, const AdjGeom& G, const AdjCoef<R>& c,
                                           R (&lf)[NP + NM], double (&par)[ADJ_NPAR]) {
    const int64_t fs = G.fs;
    R phi[NP], mu[NM], hi[NP], Mi[NM], Xi[NP + NM];
    load_cell<R, NP, NM>(s, fs, o, phi, mu);
    h_of<R, NP>(phi, hi);
    mob_of<R, NP, NM>(hi, c, Mi);
#pragma unroll
    for (int f = 0; f < NP + NM; ++f) Xi[f] = X[f * fs + o];
    R lphi[NP], lmu[NM], lM[NM];
#pragma unroll
    for (int a = 0; a < NP; ++a) lphi[a] = R(0);
#pragma unroll
    for (int k = 0; k < NM; ++k) {
        lmu[k] = R(0);
        lM[k] = R(0);
    }
    // faces: 0 x-lo, 1 x-hi, 2 y-lo, 3 y-hi; on a hi face this cell is the lower one
#pragma unroll
    for (int fc = 0; fc < 4; ++fc) {
        const int nxp = x + (fc == 0 ? -1 : fc == 1 ? 1 : 0);
        const int nyp = y + (fc == 2 ? -1 : fc == 3 ? 1 : 0);
        const int64_t oj = cell_at(G, nxp, nyp);
        if (oj == o) continue;
        const bool lower = fc == 1 || fc == 3;
        R pj[NP], uj[NM], hj[NP], Mj[NM], Xj[NP + NM];
        load_cell<R, NP, NM>(s, fs, oj, pj, uj);
        h_of<R, NP>(pj, hj);
        mob_of<R, NP, NM>(hj, c, Mj);
#pragma unroll
        for (int f = 0; f < NP + NM; ++f) Xj[f] = X[f * fs + oj];
        // A = lower cell, B = upper cell of the face
        const R* pA = lower ? phi : pj;
        const R* pB = lower ? pj : phi;
        const R* uA = lower ? mu : uj;
        const R* uB = lower ? uj : mu;
        const R* MA = lower ? Mi : Mj;
        const R* MB = lower ? Mj : Mi;
        const R* XA = lower ? Xi : Xj;
        const R* XB = lower ? Xj : Xi;
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
                if (lower) par[pi] += (double)lgG * (double)Gn;
                const R lqn = R(2) * c.gam[pi] * lgG;
                lpb[i] = lpb[i] + lqn * g[j];
                lg[j] = lg[j] + lqn * pb[i];
                lpb[j] = lpb[j] - lqn * g[i];
                lg[i] = lg[i] - lqn * pb[j];
            }
#pragma unroll
        for (int a = 0; a < NP; ++a)
            lphi[a] = lphi[a] + (lower ? R(0.5) * lpb[a] - lg[a] * c.inv_dx
                                       : R(0.5) * lpb[a] + lg[a] * c.inv_dx);
#pragma unroll
        for (int k = 0; k < NM; ++k) {
            const R lJ = (XA[NP + k] - XB[NP + k]) * c.inv_dx;
            lM[k] = lM[k] + lJ * R(0.5) * (uB[k] - uA[k]) * c.inv_dx;
            const R lu = lJ * R(0.5) * (MA[k] + MB[k]) * c.inv_dx;
            lmu[k] = lower ? lmu[k] - lu : lmu[k] + lu;
        }
    }
    // mobility M_k = sum_b D_bk chi_bk h_b(phi)
    R dhi[NP][NP];
    dh_of<R, NP>(phi, dhi);
#pragma unroll
    for (int k = 0; k < NM; ++k)
#pragma unroll
        for (int b = 0; b < NP; ++b) {
            par[3 + 2 * b + k] += (double)lM[k] * (double)c.chi[b][k] * (double)hi[b];
#pragma unroll
            for (int a = 0; a < NP; ++a) lphi[a] = lphi[a] + lM[k] * c.Dchi[b][k] * dhi[b][a];
        }
#pragma unroll
    for (int a = 0; a < NP; ++a) lf[a] = lphi[a];
#pragma unroll
    for (int k = 0; k < NM; ++k) lf[NP + k] = lmu[k];
}

// Cell of this thread: ADJ_BX x ADJ_BY tiles, one per block.
__device__ __forceinline__ void adj_cell_of(const AdjGeom& G, int& x, int& y) {
    const int ntx = (G.nx + ADJ_BX - 1) / ADJ_BX;
    x = blockIdx.x % ntx * ADJ_BX + (int)(threadIdx.x % ADJ_BX);
    y = blockIdx.x / ntx * ADJ_BY + (int)(threadIdx.x / ADJ_BX);
}

// Pass A of one step: lam holds lambda^{n+1} on entry and the cell-local part
// of lambda^n on exit (each thread reads and writes its own cell only).
template <typename R, int NP, int NM>
__global__ void __launch_bounds__(ADJ_BX* ADJ_BY)
k_adj_cell(const R* __restrict__ s, R* __restrict__ lam, R* __restrict__ X, AdjGeom G, AdjCoef<R> c,
           double tt_row0, double tt_slope, double* __restrict__ acc) {
    constexpr int NF = NP + NM;
    int x, y;
    adj_cell_of(G, x, y);
    double par[ADJ_NPAR];
#pragma unroll
    for (int q = 0; q < ADJ_NPAR; ++q) par[q] = 0.0;
    if (x < G.nx && y < G.ny) {
        const int64_t o = (int64_t)y * G.nx + x;
        R l1[NF], Xo[NF], lo[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) l1[f] = lam[f * G.fs + o];
        adj_pass_a<R, NP, NM>(s, x, y, o, G, c, (R)(tt_row0 + tt_slope * (double)y), l1, Xo, lo, par);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            X[f * G.fs + o] = Xo[f];
            lam[f * G.fs + o] = lo[f];
        }
    }
    adj_block_add(ADJ_SLOTS_A, par, acc);
}

// Pass B of one step: lam (the cell-local part from pass A) becomes lambda^n.
template <typename R, int NP, int NM>
__global__ void __launch_bounds__(ADJ_BX* ADJ_BY)
k_adj_face(const R* __restrict__ s, const R* __restrict__ X, R* __restrict__ lam, AdjGeom G,
           AdjCoef<R> c, double* __restrict__ acc) {
    constexpr int NF = NP + NM;
    int x, y;
    adj_cell_of(G, x, y);
    double par[ADJ_NPAR];
#pragma unroll
    for (int q = 0; q < ADJ_NPAR; ++q) par[q] = 0.0;
    if (x < G.nx && y < G.ny) {
        const int64_t o = (int64_t)y * G.nx + x;
        R lf[NF];
        adj_pass_b<R, NP, NM>(s, X, x, y, o, G, c, lf, par);
#pragma unroll
        for (int f = 0; f < NF; ++f) lam[f * G.fs + o] = lam[f * G.fs + o] + lf[f];
    }
    adj_block_add(ADJ_SLOTS_B, par, acc);
}

// Pass B of step n followed by pass A of step n-1 at the same cell: pass A
// needs lambda^n only at its own cell, which pass B has just completed.  sB =
// s^n, XB = pass A's cotangents of step n; sA = s^{n-1}, XA receives those of
// step n-1.  The two passes' parameter sums are added B first, as separate
// launches would add them.
template <typename R, int NP, int NM>
__global__ void __launch_bounds__(ADJ_BX* ADJ_BY)
k_adj_fused(const R* __restrict__ sB, const R* __restrict__ XB, const R* __restrict__ sA,
            R* __restrict__ XA, R* __restrict__ lam, AdjGeom G, AdjCoef<R> c, double tt_row0,
            double tt_slope, double* __restrict__ acc) {
    constexpr int NF = NP + NM;
    int x, y;
    adj_cell_of(G, x, y);
    double parB[ADJ_NPAR], parA[ADJ_NPAR];
#pragma unroll
    for (int q = 0; q < ADJ_NPAR; ++q) {
        parB[q] = 0.0;
        parA[q] = 0.0;
    }
    if (x < G.nx && y < G.ny) {
        const int64_t o = (int64_t)y * G.nx + x;
        R lf[NF], l1[NF], Xo[NF], lo[NF];
        adj_pass_b<R, NP, NM>(sB, XB, x, y, o, G, c, lf, parB);
#pragma unroll
        for (int f = 0; f < NF; ++f) l1[f] = lam[f * G.fs + o] + lf[f];
        adj_pass_a<R, NP, NM>(sA, x, y, o, G, c, (R)(tt_row0 + tt_slope * (double)y), l1, Xo, lo, parA);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            XA[f * G.fs + o] = Xo[f];
            lam[f * G.fs + o] = lo[f];
        }
    }
    adj_block_add(ADJ_SLOTS_B, parB, acc);
    adj_block_add(ADJ_SLOTS_A, parA, acc);
}

// One adjoint launch: pass A of a step (which = 0), pass B (which = 1) or
// pass B of step n with pass A of step n-1 (which = 2).
struct AdjLaunch {
    int which;
    const void* sB;    // s^n for pass B
    const void* XB;    // pass A's cotangents of step n, for pass B
    const void* sA;    // the state pass A differentiates at
    void* XA;          // receives pass A's cotangents
    void* lam;         // lambda, updated in place
    AdjGeom g;
    int nphases, nmu;
    double tt_row0, tt_slope;  // T - Te at row j for pass A's step: tt_row0 + tt_slope * j
    double* acc;               // per-block parameter accumulators
};

inline int adj_blocks(const AdjGeom& g) {
    return ((g.nx + ADJ_BX - 1) / ADJ_BX) * ((g.ny + ADJ_BY - 1) / ADJ_BY);
}

template <typename R, int NP, int NM>
int adj_launch_t(const AdjLaunch& L, const AdjCoef<R>& c, hipStream_t st) {
    const int nb = adj_blocks(L.g);
    if (L.which == 0)
        hipLaunchKernelGGL((k_adj_cell<R, NP, NM>), dim3(nb), dim3(ADJ_BX * ADJ_BY), 0, st, (const R*)L.sA,
                           (R*)L.lam, (R*)L.XA, L.g, c, L.tt_row0, L.tt_slope, L.acc);
    else if (L.which == 1)
        hipLaunchKernelGGL((k_adj_face<R, NP, NM>), dim3(nb), dim3(ADJ_BX * ADJ_BY), 0, st, (const R*)L.sB,
                           (const R*)L.XB, (R*)L.lam, L.g, c, L.acc);
    else
        hipLaunchKernelGGL((k_adj_fused<R, NP, NM>), dim3(nb), dim3(ADJ_BX * ADJ_BY), 0, st, (const R*)L.sB,
                           (const R*)L.XB, (const R*)L.sA, (R*)L.XA, (R*)L.lam, L.g, c, L.tt_row0,
                           L.tt_slope, L.acc);
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
