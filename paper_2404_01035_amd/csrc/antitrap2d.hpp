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
// One thread per cell; the 3 x 3 neighbourhood is read through the caches.
#pragma once

#include "mp_internal.hpp"

namespace mp {

__device__ inline int at_wrap(int i, int n, int bc) {
    if (i < 0) return bc == MP_BC_PERIODIC ? n - 1 : 0;
    if (i >= n) return bc == MP_BC_PERIODIC ? 0 : n - 1;
    return i;
}

template <typename R>
__device__ inline R at_prefactor(R f, const AtCoef<R>& c) {
    if (!c.obstacle) return c.prefw;
    if (!(f > R(0) && f < R(1))) return R(0);
    const R h1 = f * f * (R(3) - R(2) * f);
    return c.prefo * f * (R(1) - h1) / sqrt(f * (R(1) - f));
}

// Current on one face.  pL/pR: phi^n of the two cells, tL/tR: their central
// differences along the tangential axis (already / (2 dx)), qL/qR: phi^{n+1},
// uL/uR: mu^n.  Adds the face's j_k to j.
template <typename R, int NP, int NM>
__device__ inline void at_face(const R* pL, const R* pR, const R* tL, const R* tR, const R* qL, const R* qR,
                               const R* uL, const R* uR, const AtCoef<R>& c, R* j) {
    constexpr int LIQ = NP - 1;
    R un[NP], ut[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        const R gn = (pR[a] - pL[a]) * c.rdx;
        const R gt = R(0.5) * (tL[a] + tR[a]);
        const R n2 = gn * gn + gt * gt;
        const R inv = n2 > R(1e-30) ? R(1) / sqrt(n2) : R(0);
        un[a] = gn * inv;
        ut[a] = gt * inv;
    }
    R cl[NM];
#pragma unroll
    for (int k = 0; k < NM; ++k)
        cl[k] = R(0.5) * (c.chi[LIQ][k] * (uL[k] - c.B[LIQ][k]) + c.chi[LIQ][k] * (uR[k] - c.B[LIQ][k]));
#pragma unroll
    for (int a = 0; a < NP - 1; ++a) {
        const R weight = -(un[a] * un[LIQ] + ut[a] * ut[LIQ]);
        const R rate = (R(0.5) * (qL[a] + qR[a]) - R(0.5) * (pL[a] + pR[a])) * c.rdt;
        const R common = at_prefactor(R(0.5) * (pL[a] + pR[a]), c) * rate * un[a] * weight;
#pragma unroll
        for (int k = 0; k < NM; ++k) {
            const R ca = R(0.5) * (c.chi[a][k] * (uL[k] - c.B[a][k]) + c.chi[a][k] * (uR[k] - c.B[a][k]));
            j[k] += common * (ca - cl[k]);
        }
    }
}

template <typename R, int NP, int NM>
__global__ void __launch_bounds__(256) k_antitrap2d(const R* __restrict__ prev, R* __restrict__ next, Geom g,
                                                     AtCoef<R> c) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const int jrow = (int)(blockIdx.y * blockDim.y + threadIdx.y);
    if (i >= g.nx || jrow >= g.ny) return;
    const int64_t fs = g.fstride;
    const int xs[3] = {at_wrap(i - 1, g.nx, g.bcx), i, at_wrap(i + 1, g.nx, g.bcx)};
    const int ys[3] = {at_wrap(jrow - 1, g.ny, g.bcy), jrow, at_wrap(jrow + 1, g.ny, g.bcy)};
    // phi^n on the 3 x 3 neighbourhood, phi^{n+1} and mu^n on the cell and its 4 neighbours
    R P[3][3][NP];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx)
#pragma unroll
            for (int a = 0; a < NP; ++a) P[dy][dx][a] = prev[a * fs + (int64_t)ys[dy] * g.nx + xs[dx]];
    // (a corner ghost is the per-axis maps composed, as on the ghost-padded grid)
    R Q[5][NP], U[5][NM];  // centre, x-, x+, y-, y+
    const int qx[5] = {xs[1], xs[0], xs[2], xs[1], xs[1]};
    const int qy[5] = {ys[1], ys[1], ys[1], ys[0], ys[2]};
#pragma unroll
    for (int s = 0; s < 5; ++s) {
        const int64_t o = (int64_t)qy[s] * g.nx + qx[s];
#pragma unroll
        for (int a = 0; a < NP; ++a) Q[s][a] = next[a * fs + o];
#pragma unroll
        for (int k = 0; k < NM; ++k) U[s][k] = prev[(NP + k) * fs + o];
    }
    // central differences / (2 dx): along y for the cells of row jrow (x faces),
    // along x for the cells of column i (y faces)
    const R h2 = R(0.5) * c.rdx;
    R ty[3][NP], tx[3][NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            ty[d][a] = (P[2][d][a] - P[0][d][a]) * h2;  // cell (xs[d], jrow)
            tx[d][a] = (P[d][2][a] - P[d][0][a]) * h2;  // cell (i, ys[d])
        }
    }
    R jxl[NM] = {}, jxh[NM] = {}, jyl[NM] = {}, jyh[NM] = {};
    at_face<R, NP, NM>(P[1][0], P[1][1], ty[0], ty[1], Q[1], Q[0], U[1], U[0], c, jxl);
    at_face<R, NP, NM>(P[1][1], P[1][2], ty[1], ty[2], Q[0], Q[2], U[0], U[2], c, jxh);
    at_face<R, NP, NM>(P[0][1], P[1][1], tx[0], tx[1], Q[3], Q[0], U[3], U[0], c, jyl);
    at_face<R, NP, NM>(P[1][1], P[2][1], tx[1], tx[2], Q[0], Q[4], U[0], U[4], c, jyh);
    // chi_k(phi^{n+1}) = sum_b h_b chi^b_k, h of Eq. hphi
    R hb[NP];
#pragma unroll
    for (int b = 0; b < NP; ++b) {
        const R f = Q[0][b];
        R cross = R(0);
        if constexpr (NP == 3) cross = Q[0][(b + 1) % 3] * Q[0][(b + 2) % 3];
        hb[b] = R(3) * f * f - R(2) * f * f * f + R(2) * f * cross;
    }
    const int64_t oc = (int64_t)jrow * g.nx + i;
#pragma unroll
    for (int k = 0; k < NM; ++k) {
        R chik = R(0);
#pragma unroll
        for (int b = 0; b < NP; ++b) chik += hb[b] * c.chi[b][k];
        const R div = (jxh[k] - jxl[k]) * c.rdx + (jyh[k] - jyl[k]) * c.rdx;
        R* m = next + (NP + k) * fs + oc;
        *m = *m - c.dt * div / chik;
    }
}

template <typename R>
int at_launch(const AtLaunch& L, const AtCoef<R>& c, hipStream_t s) {
    if (L.g.nz != 1 || L.g.nx < 1 || L.g.ny < 1 || (L.g.ny + 3) / 4 > 65535) return MP_E_PARAM;
    dim3 block(64, 4);
    dim3 grid((unsigned)((L.g.nx + 63) / 64), (unsigned)((L.g.ny + 3) / 4));
    const R* prev = (const R*)L.prev;
    R* next = (R*)L.next;
    if (L.nphases == 2 && L.nmu == 1)
        hipLaunchKernelGGL((k_antitrap2d<R, 2, 1>), grid, block, 0, s, prev, next, L.g, c);
    else if (L.nphases == 2 && L.nmu == 2)
        hipLaunchKernelGGL((k_antitrap2d<R, 2, 2>), grid, block, 0, s, prev, next, L.g, c);
    else if (L.nphases == 3 && L.nmu == 1)
        hipLaunchKernelGGL((k_antitrap2d<R, 3, 1>), grid, block, 0, s, prev, next, L.g, c);
    else if (L.nphases == 3 && L.nmu == 2)
        hipLaunchKernelGGL((k_antitrap2d<R, 3, 2>), grid, block, 0, s, prev, next, L.g, c);
    else
        return MP_E_PARAM;
    return hipGetLastError() == hipSuccess ? MP_OK : MP_E_HIP;
}

}  // namespace mp
