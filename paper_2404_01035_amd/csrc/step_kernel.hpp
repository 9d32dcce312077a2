// Fused phi + mu forward-Euler step of the grand-potential model (MICROSIM,
// arXiv 2404.01035, Sec. 2.1) as one HIP kernel for gfx950.
//
// Work decomposition.  A block owns a tile of BX (x) by BY (y, 3D only) cells
// and walks a segment of `seg` planes along the slowest axis (y in 2D, z in
// 3D).  Planes are staged in a 4-slot LDS ring: while plane m is computed from
// slots m-1, m, m+1, the loads of plane m+2 are already in flight into
// registers and land in slot m+2 (= m-2 mod 4) afterwards, so one barrier per
// plane suffices.  Each plane entry also stores the cell mobility
// M_k = sum_a D^a_k chi^a_k h_a(phi) so faces never recompute h of a neighbour.
// The face between planes m and m+1 is kept in registers and reused as the
// lower face of plane m+1; in-plane faces are recomputed by both cells (same
// code and inputs, so both see the same value).
//
// Every HBM byte of the state is read once per segment plus a two-plane
// overlap and the tile's one-cell rim, which the XCD-aware block order keeps
// inside one L2.
#pragma once

#include "mp_internal.hpp"

namespace mp {

// Ghost index map: -1 and n are the ghosts (wrap or mirror), indices further
// out only occur in the unused rim of a ragged tile and are clamped.
__device__ __forceinline__ int gmap(int i, int n, bool periodic) {
    if (i < 0) return periodic ? n - 1 : 0;
    if (i >= n) return (i == n && periodic) ? 0 : n - 1;
    return i;
}

// Normal component of d(a_c^2 |q|^2)/dq for the four-fold a_c, with the
// isotropic limit below |q|^2 = 1e-30 (direction undefined there).
template <typename R, int NTG>
__device__ __forceinline__ R g_aniso(R qn, const R (&qt)[NTG], R d) {
    R Q2 = qn * qn;
#pragma unroll
    for (int t = 0; t < NTG; ++t) Q2 = Q2 + qt[t] * qt[t];
    if (Q2 <= R(1e-30)) {
        R a0 = R(1) - R(3) * d;
        return R(2) * a0 * a0 * qn;
    }
    R rq = sqrt(Q2);
    R mn = qn / rq;
    R S4 = mn * mn * mn * mn;
#pragma unroll
    for (int t = 0; t < NTG; ++t) {
        R mt = qt[t] / rq;
        S4 = S4 + mt * mt * mt * mt;
    }
    R ac = R(1) - d * (R(3) - R(4) * S4);
    return R(2) * ac * ac * qn + R(32) * d * ac * rq * (mn * mn * mn - mn * S4);
}

// LDS address of a cell: ring slot and in-plane position.
struct Addr {
    int slot;
    int p;
};

// Face between cells L and R (R = L + e_n): gradient-term flux F_a and source
// s_a (for each pair a<b: q_n = pbar_a g_b - pbar_b g_a, G_n = d(a_c^2|q|^2)/dq_n,
// F_a -= gamma G_n pbar_b, F_b += gamma G_n pbar_a, s_a += gamma G_n g_b,
// s_b -= gamma G_n g_a) and the mu flux J_k = (M_L + M_R)/2 (mu_R - mu_L)/dx.
// Tangential gradients (anisotropy only) are the mean of the two cells'
// central differences; Tp/Tm hold the +/- neighbours along each tangential axis.
template <typename R, int NP, int NM, int NF, int PP, bool ANISO, int NTG>
__device__ __forceinline__ void eval_face(const R (*sv)[NF][PP], const R (*sm)[NM][PP],
                                          const Coef<R>& c, Addr L, Addr Rc,
                                          const Addr (&LTp)[NTG], const Addr (&LTm)[NTG],
                                          const Addr (&RTp)[NTG], const Addr (&RTm)[NTG],
                                          R (&F)[NP], R (&S)[NP], R (&J)[NM]) {
    R pb[NP], gg[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        R l = sv[L.slot][a][L.p];
        R r = sv[Rc.slot][a][Rc.p];
        pb[a] = R(0.5) * (l + r);
        gg[a] = (r - l) * c.inv_dx;
        F[a] = R(0);
        S[a] = R(0);
    }
    R tb[NTG > 0 ? NTG : 1][NP];
    if constexpr (ANISO) {
#pragma unroll
        for (int t = 0; t < NTG; ++t) {
#pragma unroll
            for (int a = 0; a < NP; ++a) {
                R tl = (sv[LTp[t].slot][a][LTp[t].p] - sv[LTm[t].slot][a][LTm[t].p]) * c.half_inv_dx;
                R tr = (sv[RTp[t].slot][a][RTp[t].p] - sv[RTm[t].slot][a][RTm[t].p]) * c.half_inv_dx;
                tb[t][a] = R(0.5) * (tl + tr);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < NP; ++i) {
#pragma unroll
        for (int j = i + 1; j < NP; ++j) {
            R qn = pb[i] * gg[j] - pb[j] * gg[i];
            R Gn;
            if constexpr (ANISO) {
                R d = c.delta[i][j];
                if (d != R(0)) {
                    R qt[NTG];
#pragma unroll
                    for (int t = 0; t < NTG; ++t) qt[t] = pb[i] * tb[t][j] - pb[j] * tb[t][i];
                    Gn = g_aniso<R, NTG>(qn, qt, d);
                } else {
                    Gn = R(2) * qn;
                }
            } else {
                Gn = R(2) * qn;
            }
            R gG = c.gam[i][j] * Gn;
            F[i] = F[i] - gG * pb[j];
            F[j] = F[j] + gG * pb[i];
            S[i] = S[i] + gG * gg[j];
            S[j] = S[j] - gG * gg[i];
        }
    }
#pragma unroll
    for (int k = 0; k < NM; ++k) {
        R ml = sm[L.slot][k][L.p];
        R mr = sm[Rc.slot][k][Rc.p];
        R ul = sv[L.slot][NP + k][L.p];
        R ur = sv[Rc.slot][NP + k][Rc.p];
        J[k] = R(0.5) * (ml + mr) * (ur - ul) * c.inv_dx;
    }
}

// Interpolation function h_a of Eq. hphi.
template <typename R, int NP>
__device__ __forceinline__ void interp_h(const R (&phi)[NP], R (&h)[NP]) {
    if constexpr (NP == 2) {
        h[0] = R(3) * phi[0] * phi[0] - R(2) * phi[0] * phi[0] * phi[0];
        h[1] = R(3) * phi[1] * phi[1] - R(2) * phi[1] * phi[1] * phi[1];
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            int b = (a + 1) % 3, g = (a + 2) % 3;
            R o = b < g ? phi[b] * phi[g] : phi[g] * phi[b];
            h[a] = R(3) * phi[a] * phi[a] - R(2) * phi[a] * phi[a] * phi[a] + R(2) * phi[a] * o;
        }
    }
}

template <typename R, int NP, int NM, bool D3, bool ANISO, bool OBST, int BX, int BY>
__global__ void __launch_bounds__(BX * BY)
k_step(const R* __restrict__ in, R* __restrict__ out, Geom g, Coef<R> c, double tbase,
       double tslope, int seg, int ntx, int nty) {
    constexpr int NF = NP + NM;
    constexpr int PW = BX + 2;
    constexpr int PH = D3 ? BY + 2 : 1;
    constexpr int PP = PW * PH;
    constexpr int NT = BX * BY;
    constexpr int NPOS = (PP + NT - 1) / NT;
    constexpr int NS = 4;
    constexpr int NTG = D3 ? 2 : 1;  // tangential axes of a face
    typedef R (*VRow)[NF][PP];
    typedef R (*MRow)[NM][PP];
    __shared__ R sv[NS][NF][PP];
    __shared__ R sm[NS][NM][PP];

    // XCD-aware block order: blocks are dealt round-robin to the 8 XCDs, so
    // give each XCD a contiguous run of tiles (shared rims stay in its L2).
    const int nb = gridDim.x;
    const int q8 = nb / 8;
    const int b = blockIdx.x;
    const int tile = (b < 8 * q8) ? (b % 8) * q8 + b / 8 : b;
    const int tx_i = tile % ntx;
    const int rest = tile / ntx;
    const int ty_i = rest % nty;
    const int sg_i = rest / nty;

    const int x0 = tx_i * BX;
    const int y0 = D3 ? ty_i * BY : 0;
    const int nmarch = D3 ? g.nz : g.ny;
    const int m0 = sg_i * seg;
    const int m1 = min(m0 + seg, nmarch);
    const bool perx = g.bcx == MP_BC_PERIODIC;
    const bool pery = g.bcy == MP_BC_PERIODIC;
    const bool perm = D3 ? (g.bcz == MP_BC_PERIODIC) : pery;
    const int64_t sy = g.nx;
    const int64_t smarch = D3 ? (int64_t)g.nx * g.ny : (int64_t)g.nx;
    const int64_t fs = g.fstride;

    const int tid = threadIdx.x;
    const int lx = tid % BX;
    const int ly = tid / BX;

    // global in-plane offsets of the positions this thread stages
    int64_t poff[NPOS];
#pragma unroll
    for (int k = 0; k < NPOS; ++k) {
        int p = tid + k * NT;
        if (p >= PP) p = PP - 1;
        int ix = p % PW, iy = p / PW;
        int gx = gmap(x0 - 1 + ix, g.nx, perx);
        int gyy = D3 ? gmap(y0 - 1 + iy, g.ny, pery) : 0;
        poff[k] = gx + gyy * sy;
    }

    R reg[NPOS][NF];
    auto fetch = [&](int m) {
        const int64_t mo = (int64_t)gmap(m, nmarch, perm) * smarch;
#pragma unroll
        for (int k = 0; k < NPOS; ++k) {
            if (tid + k * NT < PP) {
#pragma unroll
                for (int f = 0; f < NF; ++f) reg[k][f] = in[f * fs + mo + poff[k]];
            }
        }
    };
    auto stage = [&](int m) {
        const int sl = (m + NS) & (NS - 1);
#pragma unroll
        for (int k = 0; k < NPOS; ++k) {
            const int p = tid + k * NT;
            if (p < PP) {
                R ph[NP], hh[NP];
#pragma unroll
                for (int f = 0; f < NF; ++f) sv[sl][f][p] = reg[k][f];
#pragma unroll
                for (int a = 0; a < NP; ++a) ph[a] = reg[k][a];
                interp_h<R, NP>(ph, hh);
#pragma unroll
                for (int kk = 0; kk < NM; ++kk) {
                    R M = R(0);
#pragma unroll
                    for (int a = 0; a < NP; ++a) M = M + c.Dchi[a][kk] * hh[a];
                    sm[sl][kk][p] = M;
                }
            }
        }
    };

    // prologue: planes m0-1, m0, m0+1
    fetch(m0 - 1);
    stage(m0 - 1);
    fetch(m0);
    stage(m0);
    fetch(m0 + 1);
    stage(m0 + 1);
    __syncthreads();

    const int pc = D3 ? (ly + 1) * PW + (lx + 1) : (lx + 1);
    const int gx = x0 + lx;
    const int gy = D3 ? y0 + ly : 0;
    const bool valid = gx < g.nx && (!D3 || gy < g.ny);

    R Flo[NP], Slo[NP], Jlo[NM];  // face between planes m-1 and m

    for (int m = m0; m < m1; ++m) {
        if (m + 2 <= m1) fetch(m + 2);

        const int s0 = (m + NS) & (NS - 1);
        const int sm1 = (m - 1 + NS) & (NS - 1);
        const int sp1 = (m + 1) & (NS - 1);
        const Addr C0{s0, pc};

        R grad[NP], divj[NM];
#pragma unroll
        for (int a = 0; a < NP; ++a) grad[a] = R(0);
#pragma unroll
        for (int k = 0; k < NM; ++k) divj[k] = R(0);

        auto accumulate = [&](const R (&Fl)[NP], const R (&Sl)[NP], const R (&Jl)[NM],
                              const R (&Fh)[NP], const R (&Sh)[NP], const R (&Jh)[NM]) {
#pragma unroll
            for (int a = 0; a < NP; ++a)
                grad[a] = grad[a] + (Fh[a] - Fl[a]) * c.inv_dx - R(0.5) * (Sh[a] + Sl[a]);
#pragma unroll
            for (int k = 0; k < NM; ++k) divj[k] = divj[k] + (Jh[k] - Jl[k]) * c.inv_dx;
        };

        // ---- x faces (tangential: y in 3D, then the march axis) ----
        {
            R Fl[NP], Sl[NP], Jl[NM], Fh[NP], Sh[NP], Jh[NM];
            Addr Lm{s0, pc - 1};
            Addr Rp{s0, pc + 1};
            if constexpr (D3) {
                Addr lTp[2] = {{s0, pc - 1 + PW}, {sp1, pc - 1}};
                Addr lTm[2] = {{s0, pc - 1 - PW}, {sm1, pc - 1}};
                Addr cTp[2] = {{s0, pc + PW}, {sp1, pc}};
                Addr cTm[2] = {{s0, pc - PW}, {sm1, pc}};
                Addr rTp[2] = {{s0, pc + 1 + PW}, {sp1, pc + 1}};
                Addr rTm[2] = {{s0, pc + 1 - PW}, {sm1, pc + 1}};
                eval_face<R, NP, NM, NF, PP, ANISO, 2>((VRow)sv, (MRow)sm, c, Lm, C0, lTp, lTm, cTp,
                                                       cTm, Fl, Sl, Jl);
                eval_face<R, NP, NM, NF, PP, ANISO, 2>((VRow)sv, (MRow)sm, c, C0, Rp, cTp, cTm, rTp,
                                                       rTm, Fh, Sh, Jh);
            } else {
                Addr lTp[1] = {{sp1, pc - 1}};
                Addr lTm[1] = {{sm1, pc - 1}};
                Addr cTp[1] = {{sp1, pc}};
                Addr cTm[1] = {{sm1, pc}};
                Addr rTp[1] = {{sp1, pc + 1}};
                Addr rTm[1] = {{sm1, pc + 1}};
                eval_face<R, NP, NM, NF, PP, ANISO, 1>((VRow)sv, (MRow)sm, c, Lm, C0, lTp, lTm, cTp,
                                                       cTm, Fl, Sl, Jl);
                eval_face<R, NP, NM, NF, PP, ANISO, 1>((VRow)sv, (MRow)sm, c, C0, Rp, cTp, cTm, rTp,
                                                       rTm, Fh, Sh, Jh);
            }
            accumulate(Fl, Sl, Jl, Fh, Sh, Jh);
        }
        // ---- y faces in 3D (in-plane; tangential: x, then the march axis) ----
        if constexpr (D3) {
            R Fl[NP], Sl[NP], Jl[NM], Fh[NP], Sh[NP], Jh[NM];
            Addr Lm{s0, pc - PW};
            Addr Rp{s0, pc + PW};
            Addr lTp[2] = {{s0, pc - PW + 1}, {sp1, pc - PW}};
            Addr lTm[2] = {{s0, pc - PW - 1}, {sm1, pc - PW}};
            Addr cTp[2] = {{s0, pc + 1}, {sp1, pc}};
            Addr cTm[2] = {{s0, pc - 1}, {sm1, pc}};
            Addr rTp[2] = {{s0, pc + PW + 1}, {sp1, pc + PW}};
            Addr rTm[2] = {{s0, pc + PW - 1}, {sm1, pc + PW}};
            eval_face<R, NP, NM, NF, PP, ANISO, 2>((VRow)sv, (MRow)sm, c, Lm, C0, lTp, lTm, cTp, cTm,
                                                   Fl, Sl, Jl);
            eval_face<R, NP, NM, NF, PP, ANISO, 2>((VRow)sv, (MRow)sm, c, C0, Rp, cTp, cTm, rTp, rTm,
                                                   Fh, Sh, Jh);
            accumulate(Fl, Sl, Jl, Fh, Sh, Jh);
        }
        // ---- march-axis faces (tangential: x, then y in 3D) ----
        {
            R Fh[NP], Sh[NP], Jh[NM];
            const int sp2 = (m + 2) & (NS - 1);
            (void)sp2;
            if (m == m0) {
                // lower face of the segment's first plane: between m-1 and m
                Addr Lm{sm1, pc};
                if constexpr (D3) {
                    Addr lTp[2] = {{sm1, pc + 1}, {sm1, pc + PW}};
                    Addr lTm[2] = {{sm1, pc - 1}, {sm1, pc - PW}};
                    Addr cTp[2] = {{s0, pc + 1}, {s0, pc + PW}};
                    Addr cTm[2] = {{s0, pc - 1}, {s0, pc - PW}};
                    eval_face<R, NP, NM, NF, PP, ANISO, 2>((VRow)sv, (MRow)sm, c, Lm, C0, lTp, lTm,
                                                           cTp, cTm, Flo, Slo, Jlo);
                } else {
                    Addr lTp[1] = {{sm1, pc + 1}};
                    Addr lTm[1] = {{sm1, pc - 1}};
                    Addr cTp[1] = {{s0, pc + 1}};
                    Addr cTm[1] = {{s0, pc - 1}};
                    eval_face<R, NP, NM, NF, PP, ANISO, 1>((VRow)sv, (MRow)sm, c, Lm, C0, lTp, lTm,
                                                           cTp, cTm, Flo, Slo, Jlo);
                }
            }
            Addr Rp{sp1, pc};
            if constexpr (D3) {
                Addr cTp[2] = {{s0, pc + 1}, {s0, pc + PW}};
                Addr cTm[2] = {{s0, pc - 1}, {s0, pc - PW}};
                Addr rTp[2] = {{sp1, pc + 1}, {sp1, pc + PW}};
                Addr rTm[2] = {{sp1, pc - 1}, {sp1, pc - PW}};
                eval_face<R, NP, NM, NF, PP, ANISO, 2>((VRow)sv, (MRow)sm, c, C0, Rp, cTp, cTm, rTp,
                                                       rTm, Fh, Sh, Jh);
            } else {
                Addr cTp[1] = {{s0, pc + 1}};
                Addr cTm[1] = {{s0, pc - 1}};
                Addr rTp[1] = {{sp1, pc + 1}};
                Addr rTm[1] = {{sp1, pc - 1}};
                eval_face<R, NP, NM, NF, PP, ANISO, 1>((VRow)sv, (MRow)sm, c, C0, Rp, cTp, cTm, rTp,
                                                       rTm, Fh, Sh, Jh);
            }
            accumulate(Flo, Slo, Jlo, Fh, Sh, Jh);
#pragma unroll
            for (int a = 0; a < NP; ++a) {
                Flo[a] = Fh[a];
                Slo[a] = Sh[a];
            }
#pragma unroll
            for (int k = 0; k < NM; ++k) Jlo[k] = Jh[k];
        }

        // ---- cell update ----
        R phi[NP], mu[NM];
#pragma unroll
        for (int a = 0; a < NP; ++a) phi[a] = sv[s0][a][pc];
#pragma unroll
        for (int k = 0; k < NM; ++k) mu[k] = sv[s0][NP + k][pc];

        const int yrow = D3 ? gy : m;
        const R tt = (R)(tbase + tslope * (double)yrow);  // T - Te

        // grand potentials psi^b = -sum_k (mu_k - B^b_k)^2 / (4 A^b_k) + C^b + s^b (T - Te)
        R psi[NP];
#pragma unroll
        for (int b2 = 0; b2 < NP; ++b2) {
            R v = R(0);
#pragma unroll
            for (int k = 0; k < NM; ++k) {
                R d = mu[k] - c.B[b2][k];
                v = v - c.halfchi[b2][k] * d * d;
            }
            psi[b2] = v + c.C[b2] + c.s[b2] * tt;
        }

        // dh_b/dphi_a and dw/dphi_a
        R Rr[NP];
#pragma unroll
        for (int a = 0; a < NP; ++a) {
            R dwa = R(0);
#pragma unroll
            for (int b2 = 0; b2 < NP; ++b2) {
                if (b2 == a) continue;
                if constexpr (OBST)
                    dwa = dwa + c.wcoef[a][b2] * phi[b2];
                else
                    dwa = dwa + c.wcoef[a][b2] * phi[a] * phi[b2] * phi[b2];
            }
            if constexpr (NP == 3) {
                const int b2 = (a + 1) % 3, g2 = (a + 2) % 3;
                dwa = dwa + c.gamma3 * (b2 < g2 ? phi[b2] * phi[g2] : phi[g2] * phi[b2]);
            }
            R dps = R(0);
#pragma unroll
            for (int b2 = 0; b2 < NP; ++b2) {
                R dhba;
                if (b2 == a) {
                    R cross = R(0);
                    if constexpr (NP == 3) {
                        const int u = (a + 1) % 3, v = (a + 2) % 3;
                        cross = u < v ? phi[u] * phi[v] : phi[v] * phi[u];
                    }
                    dhba = R(6) * phi[a] - R(6) * phi[a] * phi[a] + R(2) * cross;
                } else {
                    R restv = R(0);
                    if constexpr (NP == 3) restv = phi[3 - a - b2];
                    dhba = R(2) * phi[b2] * restv;
                }
                dps = dps + psi[b2] * dhba;
            }
            Rr[a] = c.eps * grad[a] - dwa * c.inv_eps - dps;
        }

        // Lagrange multiplier in FP64 in both precisions
        double lam = 0.0;
#pragma unroll
        for (int a = 0; a < NP; ++a) lam = lam + (double)Rr[a];
        lam = lam / (double)NP;
        R phin[NP];
#pragma unroll
        for (int a = 0; a < NP; ++a) phin[a] = phi[a] + c.kphi * (R)((double)Rr[a] - lam);
        if constexpr (OBST) {
            R sum = R(0);
#pragma unroll
            for (int a = 0; a < NP; ++a) {
                phin[a] = fmin(fmax(phin[a], R(0)), R(1));
                sum = sum + phin[a];
            }
#pragma unroll
            for (int a = 0; a < NP; ++a) phin[a] = phin[a] / sum;
        }

        R h0[NP], h1[NP];
        interp_h<R, NP>(phi, h0);
        interp_h<R, NP>(phin, h1);
        R mun[NM];
#pragma unroll
        for (int k = 0; k < NM; ++k) {
            R src = R(0), chik = R(0);
#pragma unroll
            for (int a = 0; a < NP; ++a) {
                R ca = (mu[k] - c.B[a][k]) * c.chi[a][k];
                src = src + ca * (h1[a] - h0[a]);
                chik = chik + h1[a] * c.chi[a][k];
            }
            mun[k] = mu[k] + (c.dt * divj[k] - src) / chik;
        }

        if (valid) {
            const int64_t o = (int64_t)gx + (int64_t)gy * sy + (int64_t)m * smarch;
#pragma unroll
            for (int a = 0; a < NP; ++a) out[a * fs + o] = phin[a];
#pragma unroll
            for (int k = 0; k < NM; ++k) out[(NP + k) * fs + o] = mun[k];
        }

        if (m + 2 <= m1) stage(m + 2);
        __syncthreads();
    }
}

// Dispatch one step to the kernel instance for (N, K-1, dim, anisotropy, potential, tile).
template <typename R, bool D3>
int launch_step_dim(const StepLaunch& L, const Coef<R>& c, hipStream_t s);

template <typename R, int NP, int NM, bool D3, bool ANISO, bool OBST, int BX, int BY>
int launch_instance(const StepLaunch& L, const Coef<R>& c, hipStream_t s) {
    const int ntx = (L.g.nx + BX - 1) / BX;
    const int nty = D3 ? (L.g.ny + BY - 1) / BY : 1;
    const int nmarch = D3 ? L.g.nz : L.g.ny;
    const int nseg = (nmarch + L.seg - 1) / L.seg;
    const long long nblocks = (long long)ntx * nty * nseg;
    if (nblocks <= 0 || nblocks > 0x7fffffffLL) return MP_E_PARAM;
    hipLaunchKernelGGL((k_step<R, NP, NM, D3, ANISO, OBST, BX, BY>), dim3((unsigned)nblocks),
                       dim3(BX * BY), 0, s, (const R*)L.in, (R*)L.out, L.g, c, L.tbase, L.tslope,
                       L.seg, ntx, nty);
    return MP_OK;
}

template <typename R, int NP, int NM, bool D3, bool ANISO, bool OBST>
int launch_tile(const StepLaunch& L, const Coef<R>& c, hipStream_t s) {
    if constexpr (D3) {
        return launch_instance<R, NP, NM, true, ANISO, OBST, 64, 4>(L, c, s);
    } else {
        switch (L.bx) {
            case 64: return launch_instance<R, NP, NM, false, ANISO, OBST, 64, 1>(L, c, s);
            case 128: return launch_instance<R, NP, NM, false, ANISO, OBST, 128, 1>(L, c, s);
            default: return launch_instance<R, NP, NM, false, ANISO, OBST, 256, 1>(L, c, s);
        }
    }
}

template <typename R, int NP, int NM, bool D3>
int launch_flags(const StepLaunch& L, const Coef<R>& c, hipStream_t s) {
    const bool obst = L.potential == MP_OBSTACLE;
    if (L.aniso) {
        return obst ? launch_tile<R, NP, NM, D3, true, true>(L, c, s)
                    : launch_tile<R, NP, NM, D3, true, false>(L, c, s);
    }
    return obst ? launch_tile<R, NP, NM, D3, false, true>(L, c, s)
                : launch_tile<R, NP, NM, D3, false, false>(L, c, s);
}

template <typename R, bool D3>
int launch_step_dim(const StepLaunch& L, const Coef<R>& c, hipStream_t s) {
    if (L.nphases == 2 && L.nmu == 1) return launch_flags<R, 2, 1, D3>(L, c, s);
    if (L.nphases == 2 && L.nmu == 2) return launch_flags<R, 2, 2, D3>(L, c, s);
    if (L.nphases == 3 && L.nmu == 1) return launch_flags<R, 3, 1, D3>(L, c, s);
    if (L.nphases == 3 && L.nmu == 2) return launch_flags<R, 3, 2, D3>(L, c, s);
    return MP_E_PARAM;
}

}  // namespace mp
