// Per-cell diagnostics and their FP64 accumulators, shared by the separate
// diagnostics pass and the step kernels that form the partial sums of the
// state they store (the global checks of Sec. 2.1: the sum of the phase
// fields, the solute of the composition constraint c = sum_a h_a c^a(mu),
// phase volumes, the susceptibility and non-finite values).
#pragma once

#include "mp_internal.hpp"

namespace mp {

// Neumaier-compensated sum.
struct Neu {
    double s, c;
};

__device__ __forceinline__ void neu_add(Neu& a, double x) {
    double t = a.s + x;
    if (fabs(a.s) >= fabs(x))
        a.c += (a.s - t) + x;
    else
        a.c += (x - t) + a.s;
    a.s = t;
}

__device__ __forceinline__ void neu_merge(Neu& a, const Neu& b) {
    neu_add(a, b.s);
    a.c += b.c;
}

// h_a of Eq. hphi in FP64 (the coupling term 2 phi_a phi_b phi_c for N = 3).
template <int NP>
__device__ __forceinline__ void h_fp64(const double (&p)[NP], double (&h)[NP]) {
    for (int a = 0; a < NP; ++a) {
        double o = 0.0;
        if (NP == 3) {
            int b = (a + 1) % 3, g = (a + 2) % 3;
            o = p[b] * p[g];
        }
        h[a] = 3.0 * p[a] * p[a] - 2.0 * p[a] * p[a] * p[a] + 2.0 * p[a] * o;
    }
}

// Per-thread (per-lane) accumulators: plain FP64 sums over the few dozen
// cells one thread visits; compensation starts at the merges (DiagRec).
// Sums are of phi_a and c_k per cell; the cell volume dx^d multiplies the
// final sums on the host.
struct DiagAcc {
    double mass[2];
    double vol[3];
    double maxdev;
    double minchi[2];
    int nonfin;
};

__device__ __forceinline__ void acc_init(DiagAcc& A) {
    for (int k = 0; k < 2; ++k) A.mass[k] = 0.0;
    for (int a = 0; a < 3; ++a) A.vol[a] = 0.0;
    A.maxdev = 0.0;
    A.minchi[0] = A.minchi[1] = INFINITY;
    A.nonfin = 0;
}

// A partial record: Neumaier sums, merged in a fixed order.
struct DiagRec {
    Neu mass[2];
    Neu vol[3];
    double maxdev;
    double minchi[2];
    double nonfin;
};

__device__ __forceinline__ void rec_init(DiagRec& R) {
    for (int k = 0; k < 2; ++k) R.mass[k] = {0.0, 0.0};
    for (int a = 0; a < 3; ++a) R.vol[a] = {0.0, 0.0};
    R.maxdev = 0.0;
    R.minchi[0] = R.minchi[1] = INFINITY;
    R.nonfin = 0.0;
}

__device__ __forceinline__ void rec_from(DiagRec& R, const DiagAcc& A) {
    for (int k = 0; k < 2; ++k) R.mass[k] = {A.mass[k], 0.0};
    for (int a = 0; a < 3; ++a) R.vol[a] = {A.vol[a], 0.0};
    R.maxdev = A.maxdev;
    R.minchi[0] = A.minchi[0];
    R.minchi[1] = A.minchi[1];
    R.nonfin = (double)A.nonfin;
}

__device__ __forceinline__ void rec_merge(DiagRec& A, const DiagRec& B) {
    for (int k = 0; k < 2; ++k) neu_merge(A.mass[k], B.mass[k]);
    for (int a = 0; a < 3; ++a) neu_merge(A.vol[a], B.vol[a]);
    A.maxdev = fmax(A.maxdev, B.maxdev);
    A.minchi[0] = fmin(A.minchi[0], B.minchi[0]);
    A.minchi[1] = fmin(A.minchi[1], B.minchi[1]);
    A.nonfin += B.nonfin;
}

__device__ __forceinline__ void rec_store(double* r, const DiagRec& A) {
    for (int k = 0; k < 2; ++k) {
        r[DV_MASS + 2 * k] = A.mass[k].s;
        r[DV_MASS + 2 * k + 1] = A.mass[k].c;
    }
    for (int a = 0; a < 3; ++a) {
        r[DV_VOL + 2 * a] = A.vol[a].s;
        r[DV_VOL + 2 * a + 1] = A.vol[a].c;
    }
    r[DV_MAXDEV] = A.maxdev;
    r[DV_MINCHI] = A.minchi[0];
    r[DV_MINCHI + 1] = A.minchi[1];
    r[DV_NONFIN] = A.nonfin;
}

__device__ __forceinline__ void rec_load(DiagRec& A, const double* r) {
    for (int k = 0; k < 2; ++k) A.mass[k] = {r[DV_MASS + 2 * k], r[DV_MASS + 2 * k + 1]};
    for (int a = 0; a < 3; ++a) A.vol[a] = {r[DV_VOL + 2 * a], r[DV_VOL + 2 * a + 1]};
    A.maxdev = r[DV_MAXDEV];
    A.minchi[0] = r[DV_MINCHI];
    A.minchi[1] = r[DV_MINCHI + 1];
    A.nonfin = r[DV_NONFIN];
}

// One cell's contribution: phi and mu as stored (widened to FP64), tt = T - Te
// of the cell's row at the state's time level (used when TDEP: the extended
// model's B^a(T)).  c_k = sum_a h_a c^a_k = mu_k sum_a h_a chi^a_kk
// + mu_{1-k} sum_a h_a chi^a_01 - sum_a h_a (cb + cbt tt)^a_k.
template <int NP, int NM, bool TDEP>
__device__ __forceinline__ void diag_cell(const double (&p)[NP], const double (&mu)[NM], double tt,
                                          const DiagCoef& dc, DiagAcc& A) {
    bool fin = true;
    double sum = 0.0;
    for (int a = 0; a < NP; ++a) {
        fin = fin && isfinite(p[a]);
        sum += p[a];
    }
    for (int k = 0; k < NM; ++k) fin = fin && isfinite(mu[k]);
    if (!fin) A.nonfin += 1;
    double h[NP];
    h_fp64<NP>(p, h);
    A.maxdev = fmax(A.maxdev, fabs(sum - 1.0));
    for (int a = 0; a < NP; ++a) A.vol[a] += p[a];
    double xs = 0.0;
    if (NM == 2)
        for (int a = 0; a < NP; ++a) xs += h[a] * dc.chx[a];
    for (int k = 0; k < NM; ++k) {
        double chi = 0.0, cb = 0.0;
        for (int a = 0; a < NP; ++a) {
            chi += h[a] * dc.chi[a][k];
            cb += h[a] * (TDEP ? dc.cb[a][k] + dc.cbt[a][k] * tt : dc.cb[a][k]);
        }
        double cc = mu[k] * chi - cb;
        if (NM == 2) cc += mu[1 - k] * xs;
        A.mass[k] += cc;
        A.minchi[k] = fmin(A.minchi[k], chi);
    }
}

// Order-preserving map of doubles to unsigned 64-bit keys (non-NaN values:
// x < y exactly when key(x) < key(y)), so that LDS integer min / max atomics
// take minima and maxima of doubles.
__device__ __forceinline__ unsigned long long ord_key(double x) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double ord_val(unsigned long long k) {
    const unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double((long long)b);
}

// The fused diagnostics' per-lane accumulators of a 2D strip, kept in LDS and
// updated with LDS atomics that return nothing, so that no registers are held
// across the strip's row loop.  Each lane owns its slots (slot j of the lane
// at base[j * 256]), so its additions happen in its program order.  The
// solute sum is kept as sums of h_a, h_a mu_k and (TDEP) h_a (T - Te), which
// the coefficients of c^a(mu) combine once per lane at the end:
// sum c_k = sum_a chi_kk S_mu[a][k] + chi_01 S_mu[a][1-k] - cb_k S_h[a] - cbt_k S_t[a].
template <int NP, int NM, bool TDEP>
struct DiagStrip {
    // sums: phi_a, h_a, h_a mu_k, (TDEP) h_a tt, the non-finite count; then the keys
    static constexpr int NS = 2 * NP + NP * NM + (TDEP ? NP : 0) + 1;
    static constexpr int NONFIN = NS - 1;
    static constexpr int NK = 1 + NM;  // max dev, min chi_k
    static constexpr int STRIDE = 256;
    static constexpr int WORDS = (NS + NK) * STRIDE;  // doubles of LDS per block
    double* s;  // this lane's first slot; slot j at s[j * STRIDE], key j at slot NS + j

    __device__ __forceinline__ unsigned long long* key(int j) const {
        return (unsigned long long*)(s + (NS + j) * STRIDE);
    }
    __device__ __forceinline__ void init(double* lds, int lane) {
        s = lds + lane;
        for (int j = 0; j < NS; ++j) s[j * STRIDE] = 0.0;
        *key(0) = ord_key(0.0);
        for (int k = 0; k < NM; ++k) *key(1 + k) = ord_key(INFINITY);
    }
    __device__ __forceinline__ void add(int j, double v) const {
        __hip_atomic_fetch_add(s + j * STRIDE, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    }
    // one stored cell: the same per-cell values as diag_cell
    __device__ __forceinline__ void cell(const double (&p)[NP], const double (&mu)[NM], double tt,
                                         const DiagCoef& dc) const {
        bool fin = true;
        double sum = 0.0;
        for (int a = 0; a < NP; ++a) {
            fin = fin && isfinite(p[a]);
            sum += p[a];
        }
        for (int k = 0; k < NM; ++k) fin = fin && isfinite(mu[k]);
        if (!fin) add(NONFIN, 1.0);
        double h[NP];
        h_fp64<NP>(p, h);
        const double dev = fabs(sum - 1.0);
        // a NaN leaves the maximum and minima as fmax / fmin would
        __hip_atomic_fetch_max(key(0), ord_key(dev == dev ? dev : 0.0), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WAVEFRONT);
        for (int a = 0; a < NP; ++a) {
            add(a, p[a]);
            add(NP + a, h[a]);
            for (int k = 0; k < NM; ++k) add(2 * NP + a * NM + k, h[a] * mu[k]);
            if constexpr (TDEP) add(2 * NP + NP * NM + a, h[a] * tt);
        }
        for (int k = 0; k < NM; ++k) {
            double chi = 0.0;
            for (int a = 0; a < NP; ++a) chi += h[a] * dc.chi[a][k];
            __hip_atomic_fetch_min(key(1 + k), ord_key(chi == chi ? chi : INFINITY), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WAVEFRONT);
        }
    }
    // this lane's partial record
    __device__ __forceinline__ void record(const DiagCoef& dc, DiagRec& R) const {
        double S[NS];
        for (int j = 0; j < NS; ++j) S[j] = s[j * STRIDE];
        for (int a = 0; a < 3; ++a) R.vol[a] = {a < NP ? S[a] : 0.0, 0.0};
        for (int k = 0; k < 2; ++k) {
            double m = 0.0;
            if (k < NM) {
                for (int a = 0; a < NP; ++a) {
                    m += dc.chi[a][k] * S[2 * NP + a * NM + k] - dc.cb[a][k] * S[NP + a];
                    if constexpr (NM == 2) m += dc.chx[a] * S[2 * NP + a * NM + 1 - k];
                    if constexpr (TDEP) m -= dc.cbt[a][k] * S[2 * NP + NP * NM + a];
                }
            }
            R.mass[k] = {m, 0.0};
        }
        R.maxdev = ord_val(*key(0));
        R.minchi[0] = R.minchi[1] = INFINITY;
        for (int k = 0; k < NM; ++k) R.minchi[k] = ord_val(*key(1 + k));
        R.nonfin = S[NONFIN];
    }
};

// Fold the 64 lanes' records into lane 0 (a fixed tree: lane i takes lane
// i + w for w = 32, 16, ..., 1).  Every lane of the wave must call it.
__device__ __forceinline__ void rec_wave_reduce(DiagRec& A) {
    for (int w = 32; w > 0; w >>= 1) {
        DiagRec B;
        for (int k = 0; k < 2; ++k) {
            B.mass[k].s = __shfl_down(A.mass[k].s, w);
            B.mass[k].c = __shfl_down(A.mass[k].c, w);
            B.minchi[k] = __shfl_down(A.minchi[k], w);
        }
        for (int a = 0; a < 3; ++a) {
            B.vol[a].s = __shfl_down(A.vol[a].s, w);
            B.vol[a].c = __shfl_down(A.vol[a].c, w);
        }
        B.maxdev = __shfl_down(A.maxdev, w);
        B.nonfin = __shfl_down(A.nonfin, w);
        rec_merge(A, B);
    }
}

// A lane's accumulators folded over the wave; lane 0 stores the record.
__device__ __forceinline__ void diag_wave_store(const DiagAcc& A, double* rec) {
    DiagRec R;
    rec_from(R, A);
    rec_wave_reduce(R);
    if ((threadIdx.x & 63) == 0) rec_store(rec, R);
}

}  // namespace mp
