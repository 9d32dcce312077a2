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
//   part B (faces) backpropagates every face (the gradient-term flux and
//     source, the mu flux J) from the two cells' cotangents X into both
//     cells, then the mobility M_k = sum_a D^a_k chi^a_k h_a of each cell.
// Both parts work on the step rearranged into closed forms (see AdjCoef and
// dh_parts): on a face, pair (i, j) of the gradient term depends on the two
// cells only through K = phi_i^L phi_j^R - phi_i^R phi_j^L, and for N = 3
// every derivative of h_b is one diagonal term plus twice the product of the
// other phases.  A face whose two cells coincide (zero-flux ghost, or a
// periodic axis one cell long) carries no flux; it is evaluated like any
// other and its terms vanish up to rounding.
//
// Layout of the work: as in the forward strip kernel, one wave per column
// strip (lanes 1..62 own the strip's columns, lanes 0 and 63 hold the
// neighbouring columns) marches up a segment of rows.  Each face is evaluated
// once: an x face by the lane on its left, which hands the right cell's share
// to the next lane by a lane rotate; a y face by the row below it, which
// carries the upper cell's share to the next row in registers.  B of step n
// and A of step n-1 run in one pass (A needs lambda^n only at its own cell).
// Segments are planned so that every wave of the chip starts at once (two per
// SIMD in FP32, one in FP64).  Parameter gradients are accumulated per lane in
// FP64 over the rows, summed per block in a fixed order and added to that
// block's own accumulator row, so the result is deterministic.
#pragma once

#include "gp_device.hpp"

namespace mp {

// Coefficients of the adjoint, with the grid and interface scalings folded in
// (the same step as the plain form of Sec. 2.1, rearranged):
//   on a face between cells L and R the gradient term of pair (i, j) reduces
//   to K = phi_i^L phi_j^R - phi_i^R phi_j^L (q_n = K / dx), and the cell
//   term eps [(F_hi - F_lo) / dx - (s_hi + s_lo) / 2] of that pair becomes
//   w = c4e K times a neighbour's phi, c4e = 2 eps gamma_ij / dx^2;
//   the mu flux of a face is J = (M_L + M_R)(mu_R - mu_L), its 1 / (2 dx^2)
//   folded into ktj = dt / (2 dx^2).
template <typename R>
struct AdjCoef {
    R kphi;     // dt / (tau eps): the phi update
    R ktj;      // dt / (2 dx^2): the mu update from the unscaled flux divergence
    R c4e[3];   // 2 eps gamma_ab / dx^2 by pair
    R w18e[3];  // 18 gamma_ab / eps by pair
    R g3e;      // gamma3 / eps
    R chi[3][2], B[3][2], C[3], s[3], Dchi[3][2];
    // factors of the parameter sums, applied once at the end: part B (faces:
    // gamma from K T, D from lM h) and part A (gamma from the potential, tau)
    double scB[10], scA[10];
};

constexpr int ADJ_NPAR = 10;  // gamma 01, 02, 12; D[a][k] (a < 3, k < 2); tau
constexpr int ADJ_W = 62;     // columns owned by a strip wave (lanes 1..62)

// Waves per block: the FP32 kernels hold two waves per SIMD (a block of 8
// fills one CU), the FP64 ones one (a block of 4).
template <typename R>
constexpr int adj_wpb() {
    return sizeof(R) == 4 ? 8 : 4;
}

template <typename R, int NP>
__device__ __forceinline__ void h_of(const R (&p)[NP], R (&h)[NP]) {
    R e3x2 = R(0);  // 2 phi_a phi_b phi_c, the same for every phase
    if constexpr (NP == 3) e3x2 = R(2) * (p[0] * p[1] * p[2]);
#pragma unroll
    for (int a = 0; a < NP; ++a) h[a] = p[a] * p[a] * (R(3) - R(2) * p[a]) + e3x2;
}

// Derivatives of h: dh_b/dphi_a = [a == b] d_a + 2 P_a, with d_a = 6 phi_a
// (1 - phi_a) and P_a the product of the other phases' phi (N = 3; for N = 2
// the second term is absent).  So a sum over b of v_b dh_b/dphi_a is
// v_a d_a + 2 P_a sum_b v_b.
template <typename R, int NP>
__device__ __forceinline__ void dh_parts(const R (&p)[NP], R (&d)[NP], R (&P)[NP]) {
#pragma unroll
    for (int a = 0; a < NP; ++a) d[a] = R(6) * (p[a] - p[a] * p[a]);
    if constexpr (NP == 3) {
        P[0] = p[1] * p[2];
        P[1] = p[0] * p[2];
        P[2] = p[0] * p[1];
    } else {
#pragma unroll
        for (int a = 0; a < NP; ++a) P[a] = R(0);
    }
}

// out_a = v_a d_a + 2 P_a sum_b v_b (the h chain rule above), added to out
template <typename R, int NP>
__device__ __forceinline__ void dh_apply(const R (&v)[NP], const R (&d)[NP], const R (&P)[NP], R (&out)[NP]) {
    R s2 = R(0);
    if constexpr (NP == 3) s2 = R(2) * (v[0] + v[1] + v[2]);
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        out[a] = out[a] + v[a] * d[a];
        if constexpr (NP == 3) out[a] = out[a] + s2 * P[a];
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

// Forward face: its share Ehi of the gradient term (times eps) of the lower
// cell L, Elo (subtracted) of the upper cell R, and the unscaled mu flux J.
template <typename R, int NP, int NM>
__device__ __forceinline__ void face_fwd(const R (&pL)[NP], const R (&pR)[NP], const R (&ML)[NM],
                                         const R (&MR)[NM], const R (&uL)[NM], const R (&uR)[NM],
                                         const AdjCoef<R>& c, R (&Ehi)[NP], R (&Elo)[NP], R (&J)[NM]) {
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        Ehi[a] = R(0);
        Elo[a] = R(0);
    }
#pragma unroll
    for (int i = 0; i < NP; ++i)
#pragma unroll
        for (int j = i + 1; j < NP; ++j) {
            const R w = c.c4e[pair_index(i, j)] * (pL[i] * pR[j] - pR[i] * pL[j]);
            Ehi[i] = Ehi[i] - w * pR[j];
            Ehi[j] = Ehi[j] + w * pR[i];
            Elo[i] = Elo[i] - w * pL[j];
            Elo[j] = Elo[j] + w * pL[i];
        }
#pragma unroll
    for (int k = 0; k < NM; ++k) J[k] = (ML[k] + MR[k]) * (uR[k] - uL[k]);
}

// A DPP move of a double (both halves, the same pattern), for the quad sums
// of the parameter terms; the fixed pattern keeps the rounding independent of
// timing.
template <unsigned CTRL, unsigned ROWS>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Block-wide sums of the parameter terms (each scaled by its factor), added
// to this block's accumulator row: wave sums, then the wave sums in wave
// order; B's slots (0..8) first, then A's (0, 1, 2, 9).  rowq: slot q of the
// row, read by lane q of the block's first wave at the kernel's start (no
// other block touches the row).
template <int WPB, bool DOB, bool DOA>
__device__ __forceinline__ void adj_block_add(const double (&pb)[ADJ_NPAR], const double (&pa)[ADJ_NPAR],
                                              const double (&scB)[ADJ_NPAR], const double (&scA)[ADJ_NPAR],
                                              double rowq, double* __restrict__ acc) {
    constexpr int NB = DOB ? 9 : 0, NA = DOA ? 4 : 0;
    constexpr int SA[4] = {0, 1, 2, 9};
    constexpr int NQ = NB + NA;
    __shared__ double red[WPB][NQ];
    const int t = threadIdx.x;
    // Wave sums through an LDS transpose: every lane stores its NQ terms, lane
    // 4q + j adds terms j, j + 4, ..., j + 60 of value q in that order, and a
    // quad sum completes value q in lane 4q.  Only the wave itself reads its
    // slice (rows padded to 65 to spread the banks).
    __shared__ double tr[WPB][NQ][65];
    const int lane = t & 63, wv = t >> 6;
#pragma unroll
    for (int q = 0; q < NB; ++q) tr[wv][q][lane] = pb[q] * scB[q];
#pragma unroll
    for (int q = 0; q < NA; ++q) tr[wv][NB + q][lane] = pa[SA[q]] * scA[SA[q]];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int qq = lane >> 2, j = lane & 3;
    double sq = 0.0;
    if (qq < NQ) {
        sq = tr[wv][qq][j];
#pragma unroll
        for (int i = 1; i < 16; ++i) sq = sq + tr[wv][qq][j + 4 * i];
    }
    sq = sq + dpp_f64<0xB1, 0xF>(sq);  // quad_perm [1,0,3,2]
    sq = sq + dpp_f64<0x4E, 0xF>(sq);  // quad_perm [2,3,0,1]
    if (j == 0 && qq < NQ) red[wv][qq] = sq;
    __syncthreads();
    if (t < ADJ_NPAR) {
        double r = rowq;
        if (DOB && t < 9) {
            double sum = red[0][t];
#pragma unroll
            for (int k = 1; k < WPB; ++k) sum = sum + red[k][t];
            r = r + sum;
        }
        if (DOA && (t < 3 || t == 9)) {
            const int ja = NB + (t < 3 ? t : 3);
            double sum = red[0][ja];
#pragma unroll
            for (int k = 1; k < WPB; ++k) sum = sum + red[k][ja];
            r = r + sum;
        }
        if ((DOB && t < 9) || (DOA && (t < 3 || t == 9))) acc[(size_t)blockIdx.x * ADJ_NPAR + t] = r;
    }
}


struct AdjGeom {
    int nx, ny;
    bool perx, pery;
    int64_t fs;
    // wave plan: ntx strips of ADJ_W columns, each cut into pw segments of len
    // or len + 1 rows (nlong of them long), one wave per segment
    int ntx, pw, len, nlong;
};

// Plans the strips for `slots` waves resident at once (the chip's SIMDs times
// the waves each holds): as many segments per strip as fill the slots once,
// so that every wave starts together and the work per SIMD differs by at
// most one row (the long segments go to different SIMDs, see adj_segment).
inline void adj_plan(AdjGeom& g, int slots) {
    g.ntx = (g.nx + ADJ_W - 1) / ADJ_W;
    int pw = slots / g.ntx;
    pw = pw < 1 ? 1 : (pw > g.ny ? g.ny : pw);
    g.pw = pw;
    g.len = g.ny / pw;
    g.nlong = g.ny % pw;
}

template <int WPB>
inline int adj_blocks(const AdjGeom& g) {
    return (int)(((long long)g.ntx * g.pw + WPB - 1) / WPB);
}

// Waves 0..7 of a block of 8 share SIMDs in pairs, either (w, w+4) or
// (2i, 2i+1) depending on how the waves are dealt; the "a" waves {0, 2, 5, 7}
// meet one "b" wave in both pairings.  a waves below x:
__host__ __device__ inline int adj_count_a(int x) {
    return 4 * (x >> 3) + ((0x33222110 >> (4 * (x & 7))) & 0xF);
}

// Rows [m0, m1) and strip tx of wave gw (tx >= ntx: idle).  The long segments
// of a strip take its "a" waves first (with one wave per SIMD, WPB = 4, every
// wave counts as "a"), so that no SIMD holds two of them while short ones
// remain.
template <int WPB>
__host__ __device__ inline void adj_segment(const AdjGeom& g, int gw, int& tx, int& m0, int& m1) {
    tx = gw / g.pw;
    const int r = gw - tx * g.pw;
    const int base = tx * g.pw;
    int kA = r, nA = g.pw;
    bool isA = true;
    if constexpr (WPB == 8) {
        const int cb = adj_count_a(base);
        kA = adj_count_a(base + r) - cb;
        nA = adj_count_a(base + g.pw) - cb;
        isA = ((0xA5 >> (gw & 7)) & 1) != 0;
    }
    const int kB = r - kA;
    const int eB = g.nlong > nA ? g.nlong - nA : 0;  // long segments left for "b" waves
    const int before = (kA < g.nlong ? kA : g.nlong) + (kB < eB ? kB : eB);
    const bool lng = isA ? kA < g.nlong : kB < eB;
    m0 = g.len * r + before;
    m1 = m0 + g.len + (lng ? 1 : 0);
}

// One face's backward, L the lower cell, R the upper.  XL, XR: the cells'
// cotangents of the gradient term (times eps, NP) and of the unscaled flux
// divergence (NM).  lpL / lpR receive the face's share of lambda_phi at L / R;
// lu the share of lambda_mu at R (-lu at L); lM the share of the mobility
// cotangent (both cells); gp the unscaled gamma terms K T by pair.
template <typename R, int NP, int NM>
__device__ __forceinline__ void face_bwd(const R (&pL)[NP], const R (&pR)[NP], const R (&uL)[NM],
                                         const R (&uR)[NM], const R (&ML)[NM], const R (&MR)[NM],
                                         const R (&XL)[NP + NM], const R (&XR)[NP + NM], const AdjCoef<R>& c,
                                         R (&lpL)[NP], R (&lpR)[NP], R (&lu)[NM], R (&lM)[NM], R (&gp)[3]) {
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        lpL[a] = R(0);
        lpR[a] = R(0);
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) gp[q] = R(0);
    // the pair's term is c4e K T with T = XL_j pR_i - XL_i pR_j + XR_i pL_j - XR_j pL_i
#pragma unroll
    for (int i = 0; i < NP; ++i)
#pragma unroll
        for (int j = i + 1; j < NP; ++j) {
            const int pi = pair_index(i, j);
            const R K = pL[i] * pR[j] - pR[i] * pL[j];
            const R T = (XL[j] * pR[i] - XL[i] * pR[j]) + (XR[i] * pL[j] - XR[j] * pL[i]);
            gp[pi] = K * T;
            const R t = c.c4e[pi] * T, kk = c.c4e[pi] * K;
            lpL[i] = lpL[i] + (pR[j] * t - XR[j] * kk);
            lpL[j] = lpL[j] + (XR[i] * kk - pR[i] * t);
            lpR[i] = lpR[i] + (XL[j] * kk - pL[j] * t);
            lpR[j] = lpR[j] + (pL[i] * t - XL[i] * kk);
        }
#pragma unroll
    for (int k = 0; k < NM; ++k) {
        const R xd = XL[NP + k] - XR[NP + k];
        lu[k] = xd * (ML[k] + MR[k]);
        lM[k] = xd * (uR[k] - uL[k]);
    }
}

// Part A at one cell: the forward cell update of Sec. 2.1 from (phi, mu, h(phi))
// and the cell's gradient term gradE (times eps) and unscaled flux divergence
// divJ, then its backward.  l1in = lambda^{n+1} at the cell.  Xo receives the
// cotangents of gradE (NP) and divJ (NM), lo the cell-local part of
// lambda^n; parA collects the unscaled potential gamma terms and the tau term.
template <typename R, int NP, int NM>
__device__ __forceinline__ void adj_cell_back(const R (&phi)[NP], const R (&mu)[NM], const R (&h0)[NP],
                                              const R (&gradE)[NP], const R (&divJ)[NM], const AdjCoef<R>& c, R tt,
                                              const R (&l1in)[NP + NM], R (&Xo)[NP + NM], R (&lo)[NP + NM],
                                              double (&parA)[ADJ_NPAR], bool own) {
    // ---- forward --------------------------------------------------------
    R dmu[NP][NM], cab[NP][NM], psi[NP];
#pragma unroll
    for (int b = 0; b < NP; ++b) {
        R v = c.C[b] + c.s[b] * tt;
#pragma unroll
        for (int k = 0; k < NM; ++k) {
            dmu[b][k] = mu[k] - c.B[b][k];
            cab[b][k] = c.chi[b][k] * dmu[b][k];
            v = v - R(0.5) * cab[b][k] * dmu[b][k];
        }
        psi[b] = v;
    }
    R d0[NP], P0[NP];
    dh_parts<R, NP>(phi, d0, P0);
    R psum = R(0);
    if constexpr (NP == 3) psum = psi[0] + psi[1] + psi[2];
    R sq[NP];  // phi_b^2
#pragma unroll
    for (int a = 0; a < NP; ++a) sq[a] = phi[a] * phi[a];
    double lam = 0.0;
    R Rr[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        R dw = R(0);
#pragma unroll
        for (int b = 0; b < NP; ++b)
            if (b != a) dw = dw + c.w18e[pair_index(a < b ? a : b, a < b ? b : a)] * sq[b];
        dw = dw * phi[a];
        R dps = psi[a] * d0[a];
        if constexpr (NP == 3) {
            dw = dw + c.g3e * P0[a];
            dps = dps + R(2) * P0[a] * psum;
        }
        Rr[a] = gradE[a] - dw - dps;
        lam = lam + (double)Rr[a];
    }
    lam = lam * (1.0 / NP);  // the Lagrange multiplier in FP64
    R dR[NP], phin[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        dR[a] = (R)((double)Rr[a] - lam);
        phin[a] = phi[a] + c.kphi * dR[a];
    }
    R h1[NP], d1[NP], P1[NP];
    h_of<R, NP>(phin, h1);
    dh_parts<R, NP>(phin, d1, P1);
    R dh[NP];
#pragma unroll
    for (int b = 0; b < NP; ++b) dh[b] = h1[b] - h0[b];

    // ---- mu update: mu + (ktj divJ - sum_b cab_b (h1_b - h0_b)) / sum_b chi_b h1_b
    R lmu[NM], lh1[NP], lh0[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        lh1[a] = R(0);
        lh0[a] = R(0);
    }
#pragma unroll
    for (int k = 0; k < NM; ++k) {
        R src = R(0), chik = R(0), cdh = R(0);
#pragma unroll
        for (int b = 0; b < NP; ++b) {
            src = src + cab[b][k] * dh[b];
            chik = chik + c.chi[b][k] * h1[b];
            cdh = cdh + c.chi[b][k] * dh[b];
        }
        const R r = fast_rcp(chik);
        const R dq = (c.ktj * divJ[k] - src) * r;  // the mu increment
        const R lQ = l1in[NP + k] * r;
        Xo[NP + k] = c.ktj * lQ;
#pragma unroll
        for (int b = 0; b < NP; ++b) {
            const R a = lQ * c.chi[b][k];
            lh0[b] = lh0[b] + a * dmu[b][k];
            lh1[b] = lh1[b] - a * (dmu[b][k] + dq);
        }
        lmu[k] = l1in[NP + k] - lQ * cdh;
    }

    // ---- phi update ------------------------------------------------------
    R lphin[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) lphin[a] = l1in[a];
    dh_apply<R, NP>(lh1, d1, P1, lphin);
    R lsum = R(0), tdot = R(0);
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        lsum = lsum + lphin[a];
        tdot = tdot + lphin[a] * dR[a];
    }
    const R lmean = lsum * (R(1) / R(NP));
    R lR[NP], lphi[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        lR[a] = c.kphi * (lphin[a] - lmean);
        lphi[a] = lphin[a];
        Xo[a] = lR[a];
    }
    dh_apply<R, NP>(lh0, d0, P0, lphi);
    // potential: dw_a = phi_a sum_b w18e_ab phi_b^2 + g3e P_a, by pair (i, j)
    R gpot[3] = {R(0), R(0), R(0)};
#pragma unroll
    for (int i = 0; i < NP; ++i)
#pragma unroll
        for (int j = i + 1; j < NP; ++j) {
            const int pi = pair_index(i, j);
            const R u = lR[i] * phi[j], v = lR[j] * phi[i];
            const R w = c.w18e[pi];
            lphi[i] = lphi[i] - (w * phi[j]) * (u + R(2) * v);
            lphi[j] = lphi[j] - (w * phi[i]) * (v + R(2) * u);
            gpot[pi] = (phi[i] * phi[j]) * (u + v);
        }
    if constexpr (NP == 3) {
        // d(g3e P_a)/dphi_b (b != a) = g3e times the third phase's phi
        lphi[0] = lphi[0] - c.g3e * (lR[1] * phi[2] + lR[2] * phi[1]);
        lphi[1] = lphi[1] - c.g3e * (lR[0] * phi[2] + lR[2] * phi[0]);
        lphi[2] = lphi[2] - c.g3e * (lR[0] * phi[1] + lR[1] * phi[0]);
    }
    // driving force dps_a = psi_a d_a + 2 P_a psum, differentiated in phi and psi
    R sLP = R(0);  // 2 sum_a lR_a P_a
    if constexpr (NP == 3) {
        sLP = R(2) * (lR[0] * P0[0] + lR[1] * P0[1] + lR[2] * P0[2]);
        const R p2 = R(2) * psum;
        lphi[0] = lphi[0] - p2 * (lR[1] * phi[2] + lR[2] * phi[1]);
        lphi[1] = lphi[1] - p2 * (lR[0] * phi[2] + lR[2] * phi[0]);
        lphi[2] = lphi[2] - p2 * (lR[0] * phi[1] + lR[1] * phi[0]);
    }
#pragma unroll
    for (int a = 0; a < NP; ++a) lphi[a] = lphi[a] - lR[a] * psi[a] * (R(6) - R(12) * phi[a]);
#pragma unroll
    for (int b = 0; b < NP; ++b) {
        const R lps = lR[b] * d0[b] + sLP;  // minus the cotangent of psi_b
#pragma unroll
        for (int k = 0; k < NM; ++k) lmu[k] = lmu[k] + lps * cab[b][k];
    }
#pragma unroll
    for (int a = 0; a < NP; ++a) lo[a] = lphi[a];
#pragma unroll
    for (int k = 0; k < NM; ++k) lo[NP + k] = lmu[k];
    if (own) {
#pragma unroll
        for (int q = 0; q < 3; ++q)
            if (q < (NP == 3 ? 3 : 1)) parA[q] += (double)gpot[q];
        parA[9] += (double)tdot;
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

// Adjoint strip kernel.  DOB: part B of step n (sB = s^n, XB = part A's
// cotangents of step n); DOA: part A at sA (step n-1 when fused, else the
// step itself), writing its cotangents to XA.  lam: lambda, updated in place
// at each owned cell (A alone: lambda^{n+1} in, the cell-local part out; B
// alone: that part in, lambda^n out; both: lambda^{n+1} in, step n-1's
// cell-local part out).  The two parts' parameter sums are added B first, as
// separate launches add them.
template <typename R, int NP, int NM, bool DOA, bool DOB>
__global__ void __launch_bounds__(64 * adj_wpb<R>()) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 2 : 1)))
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
    constexpr int WPB = adj_wpb<R>();
    const int lane = threadIdx.x & 63;
    // wave-uniform by construction
    const int wid = __builtin_amdgcn_readfirstlane(blockIdx.x * WPB + (int)(threadIdx.x >> 6));
    int tx, m0, m1;
    adj_segment<WPB>(G, wid, tx, m0, m1);
    if (tx < G.ntx) {
        const int nx = G.nx, ny = G.ny;
        const int64_t fs = G.fs;
        const int cs = tx * ADJ_W - 1 + lane;  // this lane's column
        // loaded column: wrapped, or (zero-flux) the ghost columns -1 and nx as
        // copies of 0 and nx-1; farther out clamped (never owned)
        const int col = G.perx ? wrap(cs, nx) : (cs < 0 ? 0 : (cs >= nx ? nx - 1 : cs));
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
        // carries from the face (m-1, m): B's shares for the upper cell (phi,
        // mu, mobility), A's forward Elo and J
        R cpB[NP], cuB[NM], cMB[NM], cE[NP], cJ[NM];
        {
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
                R lpL[NP], gp[3];
                face_bwd<R, NP, NM>(bl.phi, b0.phi, bl.mu, b0.mu, bl.M, b0.M, xl, x0, c, lpL, cpB, cuB, cMB, gp);
            }
            if constexpr (DOA) {
                adj_finish<R, NP, NM>(c, al);
                adj_finish<R, NP, NM>(c, a0);
                adj_finish<R, NP, NM>(c, a1);
                R Ehi[NP];
                face_fwd<R, NP, NM>(al.phi, a0.phi, al.M, a0.M, al.mu, a0.mu, c, Ehi, cE, cJ);
            }
        }

        // Row m with rows m, m+1 in (b0, b1), (x0, x1), (a0, a1); row m+2 is
        // then loaded into the row-m slots, so that consecutive rows swap the
        // roles of the two slots instead of copying records.  A face between a
        // cell and its own copy (a zero-flux ghost) is evaluated like any
        // other: its terms vanish up to rounding.
        auto row = [&](int m, Cell& b0, Cell& b1, R (&x0)[NF], R (&x1)[NF], Cell& a0, Cell& a1) {
            const int64_t o = (int64_t)m * nx + cs;  // the owned cell (own lanes only)
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
                R lpx[NP], lpxR[NP], lux[NM], lMx[NM], gpx[3];
                face_bwd<R, NP, NM>(b0.phi, pR, b0.mu, uR, b0.M, MR, x0, XR, c, lpx, lpxR, lux, lMx, gpx);
                // y face (m, m+1)
                R lpy[NP], lpyU[NP], luy[NM], lMy[NM], gpy[3];
                face_bwd<R, NP, NM>(b0.phi, b1.phi, b0.mu, b1.mu, b0.M, b1.M, x0, x1, c, lpy, lpyU, luy, lMy, gpy);
                // the cell's four faces: x-hi (own), x-lo (from the previous
                // lane), y-hi (own), y-lo (carried)
                R lphi[NP], lmu[NM], lM[NM];
#pragma unroll
                for (int a = 0; a < NP; ++a) lphi[a] = (lpx[a] + lane_prev(lpxR[a])) + (lpy[a] + cpB[a]);
#pragma unroll
                for (int k = 0; k < NM; ++k) {
                    lmu[k] = (lane_prev(lux[k]) - lux[k]) + (cuB[k] - luy[k]);
                    lM[k] = (lMx[k] + lane_prev(lMx[k])) + (lMy[k] + cMB[k]);
                }
                // mobility M_k = sum_b D_bk chi_bk h_b(phi)
                R mb[NP], d[NP], P[NP];
#pragma unroll
                for (int b = 0; b < NP; ++b) {
                    R v = R(0);
#pragma unroll
                    for (int k = 0; k < NM; ++k) v = v + lM[k] * c.Dchi[b][k];
                    mb[b] = v;
                }
                dh_parts<R, NP>(b0.phi, d, P);
                dh_apply<R, NP>(mb, d, P, lphi);
                if (own) {
#pragma unroll
                    for (int q = 0; q < (NP == 3 ? 3 : 1); ++q) parB[q] += (double)(gpx[q] + gpy[q]);
#pragma unroll
                    for (int k = 0; k < NM; ++k)
#pragma unroll
                        for (int b = 0; b < NP; ++b) parB[3 + 2 * b + k] += (double)(lM[k] * b0.h[b]);
                }
#pragma unroll
                for (int a = 0; a < NP; ++a) {
                    lf[a] = lphi[a];
                    cpB[a] = lpyU[a];
                }
#pragma unroll
                for (int k = 0; k < NM; ++k) {
                    lf[NP + k] = lmu[k];
                    cuB[k] = luy[k];
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
                R Ex[NP], Elx[NP], Jx[NM], Ey[NP], Ely[NP], Jy[NM];
                face_fwd<R, NP, NM>(a0.phi, pR, a0.M, MR, a0.mu, uR, c, Ex, Elx, Jx);
                face_fwd<R, NP, NM>(a0.phi, a1.phi, a0.M, a1.M, a0.mu, a1.mu, c, Ey, Ely, Jy);
                R gradE[NP], divJ[NM];
#pragma unroll
                for (int a = 0; a < NP; ++a) {
                    gradE[a] = (Ex[a] - lane_prev(Elx[a])) + (Ey[a] - cE[a]);
                    cE[a] = Ely[a];
                }
#pragma unroll
                for (int k = 0; k < NM; ++k) {
                    divJ[k] = (Jx[k] - lane_prev(Jx[k])) + (Jy[k] - cJ[k]);
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
                adj_cell_back<R, NP, NM>(ph, mu, hA, gradE, divJ, c, (R)(tt_row0 + tt_slope * (double)m), l1, Xo,
                                         lo, parA, own);
                if (own) {
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
    adj_block_add<WPB, DOB, DOA>(parB, parA, c.scB, c.scA, rowq, acc);
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
    const int nb = adj_blocks<adj_wpb<R>()>(L.g);
    const dim3 grid(nb), block(64 * adj_wpb<R>());
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
