// Device arithmetic of one grand-potential step (MICROSIM, arXiv 2404.01035,
// Sec. 2.1), shared by the 2D and 3D step kernels.
//
// Faces.  On a face normal to axis n between cells L and R, with
// sigma_a = phi_L,a + phi_R,a and delta_a = phi_R,a - phi_L,a, the pair term of
// Eq. Eqn_a has q_n = (sigma_a delta_b - sigma_b delta_a) / (2 dx).  The
// gradient term of Eq. phi_eqn at a cell is
//   eps [ sum_axes (F_hi - F_lo)/dx - (s_hi + s_lo)/2 ],
// F_a = d(a)/d(d_n phi_a), s_a = the face's share of d(a)/d(phi_a).  Writing
// U = 2F - dx s (what the face contributes to the cell below it) and
// W = 2F + dx s (to the cell above it) this is eps/(2 dx) sum_axes (U_hi - W_lo),
// and for each pair, with g = 2 gamma G_n (G_n = d(a_c^2|q|^2)/dq_n):
//   U_a -= g phi_R,b,  U_b += g phi_R,a,  W_a -= g phi_L,b,  W_b += g phi_L,a.
// a_c depends only on the direction of q and G_n is homogeneous of degree one,
// so the anisotropic G_n is evaluated on the rescaled q~ = 2 dx q (the guard
// |q|^2 <= 1e-30 is rescaled with it).  The mu flux uses
// M~ = dt/(2 dx^2) M, so that dt div(M grad mu) = sum_axes (J_hi - J_lo) with
// J = (M~_L + M~_R)(mu_R - mu_L).
//
// Cells.  psi^b = C^b + s^b (T - Te) - sum_k (mu_k - B^b_k)^2 / (4 A^b_k);
// with P_a = phi_b phi_c (N = 3) the driving force of Eq. phi_eqn is
// sum_b psi^b dh_b/dphi_a = 6 psi_a phi_a (1 - phi_a) + 2 P_a sum_b psi_b, and
// h_a = phi_a^2 (3 - 2 phi_a) + 2 phi_a P_a (Eq. hphi).  lambda is the mean of
// the N right-hand sides, accumulated in FP64 in both precisions.
#pragma once

#include "mp_internal.hpp"

namespace mp {

// Ghost index map: -1 and n are the ghosts (wrap or mirror); indices further
// out only occur in the unused rim of a ragged tile and are clamped.
__device__ __forceinline__ int gmap(int i, int n, bool periodic) {
    if (i < 0) return periodic ? n - 1 : 0;
    if (i >= n) return (i == n && periodic) ? 0 : n - 1;
    return i;
}

// Index i mod n for any integer i (n >= 1).
__device__ __forceinline__ int wrap(int i, int n) {
    const int r = i % n;
    return r < 0 ? r + n : r;
}

__device__ __forceinline__ int pair_index(int i, int j) { return i + j - 1; }  // (0,1)->0 (0,2)->1 (1,2)->2

// 1/sqrt(x), x > 0 and normal: hardware estimate (about 1 ulp in FP32), two
// Newton steps in FP64.
__device__ __forceinline__ float rsqrt_ok(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_ok(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    y = y * fma(-hx * y, y, 1.5);
    return y * fma(-hx * y, y, 1.5);
}

// Normal component of d(a_c^2 |q|^2)/dq for the four-fold a_c, on the rescaled
// q.  m = q/|q| comes from one reciprocal square root; the |q|^2 <= guard
// limit is selected at the end, so lanes do not diverge.
template <typename R, int NTG>
__device__ __forceinline__ R g_aniso(R qn, const R (&qt)[NTG], R d, R guard) {
    R Q2 = qn * qn;
#pragma unroll
    for (int t = 0; t < NTG; ++t) Q2 = Q2 + qt[t] * qt[t];
    const bool small = Q2 <= guard;
    const R Q2s = small ? R(1) : Q2;
    const R inv = rsqrt_ok(Q2s);
    const R rq = Q2s * inv;
    const R mn = qn * inv;
    const R mn2 = mn * mn;
    R S4 = mn2 * mn2;
#pragma unroll
    for (int t = 0; t < NTG; ++t) {
        const R mt = qt[t] * inv;
        const R mt2 = mt * mt;
        S4 = S4 + mt2 * mt2;
    }
    const R ac = R(1) - d * (R(3) - R(4) * S4);
    const R gen = R(2) * ac * ac * qn + R(32) * d * ac * rq * (mn2 * mn - mn * S4);
    const R a0 = R(1) - R(3) * d;
    return small ? R(2) * a0 * a0 * qn : gen;
}

// Entries of a cell's scaled mobility record: NM (diagonal M) or, in the
// general kernels, the NM x NM matrix row by row.
template <int NM, bool GEN>
constexpr int mob_n() {
    return GEN ? NM * NM : NM;
}

// One face: U, W (gradient term) and J (mu flux).  tau[t][a] is the unscaled
// sum of the two cells' central differences along tangential axis t
// (= 4 dx times the face's tangential gradient); unused when !ANISO.  GEN:
// mL, mR are mobility matrices and J = (M~_L + M~_R) (mu_R - mu_L).
template <typename R, int NP, int NM, bool ANISO, int NTG, bool GEN = false>
__device__ __forceinline__ void face_core(const R (&pL)[NP], const R (&pR)[NP],
                                          const R (&tau)[NTG > 0 ? NTG : 1][NP],
                                          const R (&mL)[mob_n<NM, GEN>()], const R (&mR)[mob_n<NM, GEN>()],
                                          const R (&uL)[NM], const R (&uR)[NM], const Coef<R>& c,
                                          R (&U)[NP], R (&W)[NP], R (&J)[NM]) {
    R sg[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        if constexpr (ANISO) sg[a] = pL[a] + pR[a];
        U[a] = R(0);
        W[a] = R(0);
    }
#pragma unroll
    for (int i = 0; i < NP; ++i) {
#pragma unroll
        for (int j = i + 1; j < NP; ++j) {
            const int pi = pair_index(i, j);
            // sigma_i delta_j - sigma_j delta_i = 2 (phi_L,i phi_R,j - phi_L,j phi_R,i)
            const R qh = pL[i] * pR[j] - pL[j] * pR[i];
            R gh;
            if constexpr (ANISO) {
                R d = c.del[pi];
                if (d != R(0)) {
                    R qt[NTG];
#pragma unroll
                    for (int t = 0; t < NTG; ++t)
                        qt[t] = R(0.25) * (sg[i] * tau[t][j] - sg[j] * tau[t][i]);
                    gh = c.gd[pi] * g_aniso<R, NTG>(R(2) * qh, qt, d, c.qguard);
                } else {
                    gh = c.g4d[pi] * qh;
                }
            } else {
                gh = c.g4d[pi] * qh;
            }
            U[i] = U[i] - gh * pR[j];
            U[j] = U[j] + gh * pR[i];
            W[i] = W[i] - gh * pL[j];
            W[j] = W[j] + gh * pL[i];
        }
    }
    if constexpr (GEN && NM == 2) {
        const R d0 = uR[0] - uL[0], d1 = uR[1] - uL[1];
        J[0] = (mL[0] + mR[0]) * d0 + (mL[1] + mR[1]) * d1;
        J[1] = (mL[2] + mR[2]) * d0 + (mL[3] + mR[3]) * d1;
    } else {
#pragma unroll
        for (int k = 0; k < NM; ++k) J[k] = (mL[k] + mR[k]) * (uR[k] - uL[k]);
    }
}

// Interpolation functions h_a of Eq. hphi.  For N = 3 the coupling term
// 2 phi_a phi_b phi_c is the same triple product for every phase.
template <typename R, int NP>
__device__ __forceinline__ void interp_h(const R (&phi)[NP], R (&h)[NP]) {
    R e3x2 = R(0);
    if constexpr (NP == 3) e3x2 = R(2) * (phi[0] * phi[1] * phi[2]);
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        const R sq = phi[a] * phi[a];
        if constexpr (NP == 3)
            h[a] = sq * (R(3) - R(2) * phi[a]) + e3x2;
        else
            h[a] = sq * (R(3) - R(2) * phi[a]);
    }
}

// Scaled cell mobility M~_k = sum_a (D^a_k chi^a_k dt / (2 dx^2)) h_a.
template <typename R, int NP, int NM>
__device__ __forceinline__ void mobility(const R (&h)[NP], const Coef<R>& c, R (&Mt)[NM]) {
#pragma unroll
    for (int k = 0; k < NM; ++k) {
        R m = R(0);
#pragma unroll
        for (int a = 0; a < NP; ++a) m = m + c.Dt[a][k] * h[a];
        Mt[k] = m;
    }
}

// The general kernels' mobility matrix M~_kj = sum_a (D^a chi^a)_kj dt / (2 dx^2) h_a,
// row by row.
template <typename R, int NP, int NM>
__device__ __forceinline__ void mobility_gen(const R (&h)[NP], const CoefX<R>& x, R (&Mt)[NM * NM]) {
#pragma unroll
    for (int k = 0; k < NM; ++k)
#pragma unroll
        for (int j = 0; j < NM; ++j) {
            R m = R(0);
#pragma unroll
            for (int a = 0; a < NP; ++a) m = m + x.Dx[a][k][j] * h[a];
            Mt[k * NM + j] = m;
        }
}

// Either mobility record, by the kernel's model.
template <typename R, int NP, int NM, bool GEN>
__device__ __forceinline__ void mobility_any(const R (&h)[NP], const Coef<R>& c, const CoefX<R>* x,
                                             R (&Mt)[mob_n<NM, GEN>()]) {
    if constexpr (GEN)
        mobility_gen<R, NP, NM>(h, *x, Mt);
    else
        mobility<R, NP, NM>(h, c, Mt);
}

// Reciprocal to within a few ulp: hardware estimate plus Newton steps.
__device__ __forceinline__ double fast_rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float fast_rcp(float x) {
    float r = __builtin_amdgcn_rcpf(x);
    float e = fmaf(-x, r, 1.0f);
    return fmaf(r, e, r);
}

// 2 (C^b + s^b (T - Te)) for every phase: constant along a row of fixed y.
template <typename R, int NP>
__device__ __forceinline__ void psi_const(R tt, const Coef<R>& c, R (&Cs)[NP]) {
#pragma unroll
    for (int b = 0; b < NP; ++b) Cs[b] = R(2) * (c.C[b] + c.s[b] * tt);
}

// The same with the quadratic term of C^b(T) (general kernels).
template <typename R, int NP, bool GEN>
__device__ __forceinline__ void psi_const_any(R tt, const Coef<R>& c, const CoefX<R>* x, R (&Cs)[NP]) {
    if constexpr (GEN) {
#pragma unroll
        for (int b = 0; b < NP; ++b) Cs[b] = R(2) * (c.C[b] + (c.s[b] + x->Ct[b] * tt) * tt);
    } else {
        psi_const<R, NP>(tt, c, Cs);
    }
}

// Cell update from the face sums Gs_a = sum_axes (U_hi - W_lo) and
// Js_k = sum_axes (J_hi - J_lo); h0 = h(phi^n) of the cell; Cs from psi_const.
// The cell's psi is carried doubled, psi2 = 2 psi = Cs - sum_k chi (mu - B)^2,
// so that chi (mu_k - B^b_k) serves psi and the mu source term alike.  h1
// receives h(phi^{n+1}).
template <typename R, int NP, int NM, bool OBST>
__device__ __forceinline__ void cell_update(const R (&phi)[NP], const R (&mu)[NM],
                                            const R (&h0)[NP], const R (&Gs)[NP],
                                            const R (&Js)[NM], const R (&Cs)[NP], const Coef<R>& c,
                                            R (&phin)[NP], R (&mun)[NM], R (&h1)[NP]) {
    R dmu[NP][NM], cdm[NP][NM];
    R psi2[NP];
#pragma unroll
    for (int b = 0; b < NP; ++b) {
        R v = Cs[b];
#pragma unroll
        for (int k = 0; k < NM; ++k) {
            dmu[b][k] = mu[k] - c.B[b][k];
            cdm[b][k] = c.chi[b][k] * dmu[b][k];
            v = v - cdm[b][k] * dmu[b][k];
        }
        psi2[b] = v;
    }
    R sq[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) sq[a] = phi[a] * phi[a];
    R P[NP];
    if constexpr (NP == 3) {
        P[0] = phi[1] * phi[2];
        P[1] = phi[0] * phi[2];
        P[2] = phi[0] * phi[1];
    }
    // the triple-junction well term and the psi sum share the factor P_a
    R Z = R(0);
    if constexpr (NP == 3) Z = c.g3e + ((psi2[0] + psi2[1]) + psi2[2]);

    // Rr_a = cE Gs_a - (dw_a / eps + 3 psi2_a phi_a (1 - phi_a) + P_a Z); the
    // well coefficients carry the 1/eps
    R Rr[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        R dw = R(0);
#pragma unroll
        for (int b = 0; b < NP; ++b) {
            if (b == a) continue;
            const R wc = c.wce[pair_index(a < b ? a : b, a < b ? b : a)];
            if constexpr (OBST)
                dw = dw + wc * phi[b];
            else
                dw = dw + wc * sq[b];
        }
        const R t3 = R(3) - R(3) * phi[a];
        R Y;
        if constexpr (OBST)
            Y = dw + phi[a] * (psi2[a] * t3);
        else
            Y = phi[a] * (dw + psi2[a] * t3);
        if constexpr (NP == 3) Y = Y + P[a] * Z;
        Rr[a] = c.cE * Gs[a] - Y;
    }

    double lam = 0.0;
#pragma unroll
    for (int a = 0; a < NP; ++a) lam = lam + (double)Rr[a];
    lam = lam * (1.0 / NP);
#pragma unroll
    for (int a = 0; a < NP; ++a) phin[a] = phi[a] + c.kphi * (R)((double)Rr[a] - lam);
    if constexpr (OBST) {
        R sum = R(0);
#pragma unroll
        for (int a = 0; a < NP; ++a) {
            phin[a] = fmin(fmax(phin[a], R(0)), R(1));
            sum = sum + phin[a];
        }
        const R inv = R(1) / sum;
#pragma unroll
        for (int a = 0; a < NP; ++a) phin[a] = phin[a] * inv;
    }

    R dh[NP];
    interp_h<R, NP>(phin, h1);
#pragma unroll
    for (int a = 0; a < NP; ++a) dh[a] = h1[a] - h0[a];
#pragma unroll
    for (int k = 0; k < NM; ++k) {
        R src = R(0), chik = R(0);
#pragma unroll
        for (int a = 0; a < NP; ++a) {
            src = src + cdm[a][k] * dh[a];
            chik = chik + h1[a] * c.chi[a][k];
        }
        mun[k] = mu[k] + (Js[k] - src) * fast_rcp(chik);
    }
}

// Nearest point (Euclidean) of the simplex {phi >= 0, sum phi = 1} to y: the
// obstacle step with the Lagrange multiplier over the active phases.  The
// active set starts as all phases; theta = (sum of the active y - 1) / (their
// count) is subtracted from the active phases and a phase that comes out
// negative leaves the set.  NP passes always suffice (a pass that removes
// nothing repeats the previous one), so every lane runs the same NP passes.
template <typename R, int NP>
__device__ __forceinline__ void simplex_project(R (&y)[NP]) {
    bool act[NP];
    R x[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) act[a] = true;
#pragma unroll
    for (int it = 0; it < NP; ++it) {
        R s = R(0);
        int n = 0;
#pragma unroll
        for (int a = 0; a < NP; ++a) {
            s = s + (act[a] ? y[a] : R(0));
            n += act[a] ? 1 : 0;
        }
        const R inv = n == 1 ? R(1) : (n == 2 ? R(0.5) : R(1) / R(3));
        const R th = (s - R(1)) * inv;
#pragma unroll
        for (int a = 0; a < NP; ++a) {
            x[a] = act[a] ? y[a] - th : R(0);
            act[a] = act[a] && !(x[a] < R(0));
        }
    }
#pragma unroll
    for (int a = 0; a < NP; ++a) y[a] = act[a] ? x[a] : R(0);
}

// Cell update of the extended model (general kernels): as cell_update, with
// B^b(T) = B^b + Bt^b tt and C^b(T) (in Cs) at this cell's T - Te = tt, the
// susceptibility and mobility as NM x NM matrices (psi^b = C^b - (mu - B^b)
// chi^b (mu - B^b) / 2, c^b = chi^b (mu - B^b)), the dT/dt term
// Theta_k = sum_a h_a(phi^{n+1}) (dc^a_k/dT) (T^{n+1} - T^n), the update
// mu^{n+1} = mu + [sum_a h_a(phi^{n+1}) chi^a]^-1 (Js - source - Theta) by a
// 2 x 2 solve, tau(phi) = sum tau_ab phi_a phi_b / sum phi_a phi_b from the
// per-pair constants (the single tau in bulk, where the pair sum is <= 1e-30),
// and for the obstacle either projection.
template <typename R, int NP, int NM, bool OBST>
__device__ __forceinline__ void cell_update_gen(const R (&phi)[NP], const R (&mu)[NM], const R (&h0)[NP],
                                                const R (&Gs)[NP], const R (&Js)[NM], const R (&Cs)[NP], R tt,
                                                const Coef<R>& c, const CoefX<R>& x, R (&phin)[NP],
                                                R (&mun)[NM], R (&h1)[NP]) {
    R dmu[NP][NM], cdm[NP][NM];
    R psi2[NP];
#pragma unroll
    for (int b = 0; b < NP; ++b) {
#pragma unroll
        for (int k = 0; k < NM; ++k) dmu[b][k] = mu[k] - (c.B[b][k] + x.Bt[b][k] * tt);
        if constexpr (NM == 2) {
            cdm[b][0] = c.chi[b][0] * dmu[b][0] + x.chx[b] * dmu[b][1];
            cdm[b][1] = x.chx[b] * dmu[b][0] + c.chi[b][1] * dmu[b][1];
        } else {
            cdm[b][0] = c.chi[b][0] * dmu[b][0];
        }
        R v = Cs[b];
#pragma unroll
        for (int k = 0; k < NM; ++k) v = v - cdm[b][k] * dmu[b][k];
        psi2[b] = v;
    }
    R sq[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) sq[a] = phi[a] * phi[a];
    R P[NP];
    if constexpr (NP == 3) {
        P[0] = phi[1] * phi[2];
        P[1] = phi[0] * phi[2];
        P[2] = phi[0] * phi[1];
    }
    R Z = R(0);
    if constexpr (NP == 3) Z = c.g3e + ((psi2[0] + psi2[1]) + psi2[2]);
    R Rr[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        R dw = R(0);
#pragma unroll
        for (int b = 0; b < NP; ++b) {
            if (b == a) continue;
            const R wc = c.wce[pair_index(a < b ? a : b, a < b ? b : a)];
            if constexpr (OBST)
                dw = dw + wc * phi[b];
            else
                dw = dw + wc * sq[b];
        }
        const R t3 = R(3) - R(3) * phi[a];
        R Y;
        if constexpr (OBST)
            Y = dw + phi[a] * (psi2[a] * t3);
        else
            Y = phi[a] * (dw + psi2[a] * t3);
        if constexpr (NP == 3) Y = Y + P[a] * Z;
        Rr[a] = c.cE * Gs[a] - Y;
    }
    if constexpr (!OBST) {
        // Eq. Well1 (KKS): dg/dphi_a = phi_a [sum_b 2 Theta_ab phi_b^2 (in wce)
        // + 2 Theta_a (1 - phi_a)(1 - 2 phi_a) + 2 Theta_abd phi_b^2 phi_d^2]; one
        // uniform branch around all phases, so that the other states skip it
        if (x.well1) {
#pragma unroll
            for (int a = 0; a < NP; ++a) {
                R e = x.th1[a] * ((R(1) - phi[a]) * (R(1) - R(2) * phi[a]));
                if constexpr (NP == 3) e = e + x.th3 * (sq[(a + 1) % 3] * sq[(a + 2) % 3]);
                Rr[a] = Rr[a] - phi[a] * e;
            }
        }
    }
    double lam = 0.0;
#pragma unroll
    for (int a = 0; a < NP; ++a) lam = lam + (double)Rr[a];
    lam = lam * (1.0 / NP);
    R kp = c.kphi;
    if (x.tpair) {
        R num, den;
        if constexpr (NP == 3) {
            num = (x.tab[0] * P[2] + x.tab[1] * P[1]) + x.tab[2] * P[0];
            den = (P[2] + P[1]) + P[0];
        } else {
            den = phi[0] * phi[1];
            num = x.tab[0] * den;
        }
        kp = den > R(1e-30) ? x.ktau * (den * fast_rcp(num)) : c.kphi;
    }
#pragma unroll
    for (int a = 0; a < NP; ++a) phin[a] = phi[a] + kp * (R)((double)Rr[a] - lam);
    if constexpr (OBST) {
        if (x.proj) {
            simplex_project<R, NP>(phin);
        } else {
            R sum = R(0);
#pragma unroll
            for (int a = 0; a < NP; ++a) {
                phin[a] = fmin(fmax(phin[a], R(0)), R(1));
                sum = sum + phin[a];
            }
            const R inv = R(1) / sum;
#pragma unroll
            for (int a = 0; a < NP; ++a) phin[a] = phin[a] * inv;
        }
    }
    R dh[NP];
    interp_h<R, NP>(phin, h1);
#pragma unroll
    for (int a = 0; a < NP; ++a) dh[a] = h1[a] - h0[a];
    R rhs[NM];
#pragma unroll
    for (int k = 0; k < NM; ++k) {
        R src = R(0), th = R(0);
#pragma unroll
        for (int a = 0; a < NP; ++a) {
            src = src + cdm[a][k] * dh[a];
            th = th + h1[a] * x.th[a][k];
        }
        rhs[k] = (Js[k] - src) - th;
    }
    R c00 = R(0);
#pragma unroll
    for (int a = 0; a < NP; ++a) c00 = c00 + h1[a] * c.chi[a][0];
    if constexpr (NM == 2) {
        R c11 = R(0), c01 = R(0);
#pragma unroll
        for (int a = 0; a < NP; ++a) {
            c11 = c11 + h1[a] * c.chi[a][1];
            c01 = c01 + h1[a] * x.chx[a];
        }
        const R inv = fast_rcp(c00 * c11 - c01 * c01);
        mun[0] = mu[0] + (c11 * rhs[0] - c01 * rhs[1]) * inv;
        mun[1] = mu[1] + (c00 * rhs[1] - c01 * rhs[0]) * inv;
    } else {
        mun[0] = mu[0] + rhs[0] * fast_rcp(c00);
    }
}

// Either cell update, by the kernel's model.
template <typename R, int NP, int NM, bool OBST, bool GEN>
__device__ __forceinline__ void cell_update_any(const R (&phi)[NP], const R (&mu)[NM], const R (&h0)[NP],
                                                const R (&Gs)[NP], const R (&Js)[NM], const R (&Cs)[NP], R tt,
                                                const Coef<R>& c, const CoefX<R>* x, R (&phin)[NP],
                                                R (&mun)[NM], R (&h1)[NP]) {
    if constexpr (GEN)
        cell_update_gen<R, NP, NM, OBST>(phi, mu, h0, Gs, Js, Cs, tt, c, *x, phin, mun, h1);
    else
        cell_update<R, NP, NM, OBST>(phi, mu, h0, Gs, Js, Cs, c, phin, mun, h1);
}

// Value of the next / previous lane of the wave (lane 63's next is lane 0 and
// lane 0's previous is lane 63).  FP32 goes through the LDS crossbar
// (ds_bpermute), which leaves the vector ALU -- the FP32 step's limit -- to the
// arithmetic; FP64 uses DPP wave rotates, two per value, which avoid the LDS
// round trip (for FP32 the rotates measured slower: each needs wait states
// after the instruction that wrote its source).
__device__ __forceinline__ float lane_next(float v) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute((((int)threadIdx.x + 1) & 63) << 2, __float_as_int(v)));
}
__device__ __forceinline__ float lane_prev(float v) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute((((int)threadIdx.x + 63) & 63) << 2, __float_as_int(v)));
}
// wave_rol:1 / wave_ror:1 have a source lane for every lane, so the DPP move
// needs no "old" value (bound_ctrl set, no zeroing move before it)
__device__ __forceinline__ int rot_next(int v) { return __builtin_amdgcn_mov_dpp(v, 0x134, 0xF, 0xF, true); }
__device__ __forceinline__ int rot_prev(int v) { return __builtin_amdgcn_mov_dpp(v, 0x13C, 0xF, 0xF, true); }
__device__ __forceinline__ double lane_next(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = rot_next((int)(b & 0xffffffffLL));
    const int hi = rot_next((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane_prev(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = rot_prev((int)(b & 0xffffffffLL));
    const int hi = rot_prev((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

}  // namespace mp
