// 3D fused phi + mu step: xy tiles staged in an LDS ring of z planes.
//
// A block owns a 64 (x) by BY (y, 4 or 8) tile and walks a segment of z planes.  A
// 4-slot LDS ring holds planes m-1, m, m+1 (plus the slot being filled): the
// loads of plane m+2 are issued into registers before plane m is computed and
// land in the free slot afterwards, so one barrier per plane suffices.  Each
// staged cell also stores its scaled mobility M~ so that faces never recompute
// h of a neighbour.  The z face between planes m and m+1 stays in registers
// (its W, J) and becomes the lower face of plane m+1; in-plane faces are
// evaluated by both of their cells with identical code and inputs.  Blocks are
// dealt XCD-aware so that a band of tiles shares one XCD's L2.
#pragma once

#include "diag_cell.hpp"
#include "gp_device.hpp"

namespace mp {

// The step of one block (GEN: the extended model's arithmetic, x its terms).
template <typename R, int NP, int NM, bool ANISO, bool OBST, int BX, int BY, bool GEN, bool DIAG = false>
__device__ __forceinline__ void step3d_block(const R* __restrict__ in, R* __restrict__ out, const Geom& g,
                                             const Coef<R>& c, const int64_t* __restrict__ stepctr, int kstep,
                                             double tb0, double tdn, double tslope, int seg, int ntx, int nty,
                                             const CoefX<R>* x, DiagAcc* da = nullptr,
                                             const DiagCoef* dc = nullptr) {
    constexpr int NF = NP + NM;
    constexpr int NMM = mob_n<NM, GEN>();
    constexpr int PW = BX + 2;
    constexpr int PH = BY + 2;
    constexpr int PP = PW * PH;
    constexpr int NT = BX * BY;
    constexpr int NPOS = (PP + NT - 1) / NT;
    constexpr int NS = 4;
    __shared__ R sv[NS][NF][PP];
    __shared__ R sm[NS][NMM][PP];

    const int nb = gridDim.x;
    const int q8 = nb / 8;
    const int b = blockIdx.x;
    const int tile = (b < 8 * q8) ? (b % 8) * q8 + b / 8 : b;
    const int tx_i = tile % ntx;
    const int rest = tile / ntx;
    const int ty_i = rest % nty;
    const int sg_i = rest / nty;

    const int x0 = tx_i * BX;
    const int y0 = ty_i * BY;
    const int m0 = sg_i * seg;
    const int m1 = min(m0 + seg, g.nz);
    const bool perx = g.bcx == MP_BC_PERIODIC;
    const bool pery = g.bcy == MP_BC_PERIODIC;
    const bool perz = g.bcz == MP_BC_PERIODIC;
    const int64_t sy = g.nx;
    const int64_t sz = (int64_t)g.nx * g.ny;
    const int64_t fs = g.fstride;

    const int tid = threadIdx.x;
    const int lx = tid % BX;
    const int ly = tid / BX;

    // Tile positions as loaded: the first (BY + 2) * BX are the halo rows'
    // interior columns, one aligned BX-wide row segment per wave; the last
    // 2 (BY + 2) are the rows' two halo columns.  ppos[k] is the LDS position
    // (row * PW + column) of this thread's k-th load.
    constexpr int NCORE = (BY + 2) * BX;
    int64_t poff[NPOS];
    int ppos[NPOS];
#pragma unroll
    for (int k = 0; k < NPOS; ++k) {
        int q = tid + k * NT;
        if (q >= PP) q = PP - 1;
        int ix, iy;
        if (q < NCORE) {
            iy = q / BX;
            ix = 1 + q % BX;
        } else {
            iy = (q - NCORE) >> 1;
            ix = ((q - NCORE) & 1) * (PW - 1);
        }
        ppos[k] = iy * PW + ix;
        poff[k] = gmap(x0 - 1 + ix, g.nx, perx) + gmap(y0 - 1 + iy, g.ny, pery) * sy;
    }

    R reg[NPOS][NF];
    auto fetch = [&](int m) {
        const int64_t mo = (int64_t)gmap(m, g.nz, perz) * sz;
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
            const int p = ppos[k];
            if (tid + k * NT < PP) {
                R ph[NP], hh[NP], Mt[NMM];
#pragma unroll
                for (int f = 0; f < NF; ++f) sv[sl][f][p] = reg[k][f];
#pragma unroll
                for (int a = 0; a < NP; ++a) ph[a] = reg[k][a];
                interp_h<R, NP>(ph, hh);
                mobility_any<R, NP, NM, GEN>(hh, c, x, Mt);
#pragma unroll
                for (int kk = 0; kk < NMM; ++kk) sm[sl][kk][p] = Mt[kk];
            }
        }
    };

    // Face between (sL, pL) and (sR, pR); tangential axes given as (slot, offset)
    // steps: dS*[t] is the slot step, dP*[t] the in-plane position step.
    auto face = [&](int sL, int pL, int sR, int pR, const int (&tS)[2], const int (&tP)[2],
                    R (&U)[NP], R (&Wf)[NP], R (&J)[NM]) {
        R phL[NP], phR[NP], uL[NM], uR[NM], mL[NMM], mR[NMM];
#pragma unroll
        for (int a = 0; a < NP; ++a) {
            phL[a] = sv[sL][a][pL];
            phR[a] = sv[sR][a][pR];
        }
#pragma unroll
        for (int k = 0; k < NM; ++k) {
            uL[k] = sv[sL][NP + k][pL];
            uR[k] = sv[sR][NP + k][pR];
        }
#pragma unroll
        for (int k = 0; k < NMM; ++k) {
            mL[k] = sm[sL][k][pL];
            mR[k] = sm[sR][k][pR];
        }
        R tau[2][NP];
        if constexpr (ANISO) {
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int sLp = (sL + tS[t] + NS) & (NS - 1), sLm = (sL - tS[t] + NS) & (NS - 1);
                const int sRp = (sR + tS[t] + NS) & (NS - 1), sRm = (sR - tS[t] + NS) & (NS - 1);
#pragma unroll
                for (int a = 0; a < NP; ++a)
                    tau[t][a] = (sv[sLp][a][pL + tP[t]] - sv[sLm][a][pL - tP[t]]) +
                                (sv[sRp][a][pR + tP[t]] - sv[sRm][a][pR - tP[t]]);
            }
        }
        face_core<R, NP, NM, ANISO, 2, GEN>(phL, phR, tau, mL, mR, uL, uR, c, U, Wf, J);
    };

    fetch(m0 - 1);
    stage(m0 - 1);
    fetch(m0);
    stage(m0);
    fetch(m0 + 1);
    stage(m0 + 1);
    __syncthreads();

    const int pc = (ly + 1) * PW + (lx + 1);
    const int gx = x0 + lx;
    const int gy = y0 + ly;
    const bool valid = gx < g.nx && gy < g.ny;
    const double tbase = tb0 + tdn * (double)(*stepctr + kstep);
    R Cs[NP];  // T - Te depends on y only
    const R tt = (R)(tbase + tslope * (double)gy);
    psi_const_any<R, NP, GEN>(tt, c, x, Cs);

    // tangential steps: x faces see (y, z), y faces see (x, z), z faces see (x, y)
    const int tSx[2] = {0, 1}, tPx[2] = {PW, 0};
    const int tSy[2] = {0, 1}, tPy[2] = {1, 0};
    const int tSz[2] = {0, 0}, tPz[2] = {1, PW};

    R Wlo[NP], Jlo[NM];  // z face between planes m-1 and m
    {
        R Ud[NP];
        const int s0 = (m0 + NS) & (NS - 1), sm1 = (m0 - 1 + NS) & (NS - 1);
        face(sm1, pc, s0, pc, tSz, tPz, Ud, Wlo, Jlo);
    }

    for (int m = m0; m < m1; ++m) {
        if (m + 2 <= m1) fetch(m + 2);
        const int s0 = (m + NS) & (NS - 1);
        const int sp1 = (m + 1) & (NS - 1);

        R Gs[NP], Js[NM];
        {
            R Ul[NP], Wl[NP], Jl[NM], Uh[NP], Wh[NP], Jh[NM];
            face(s0, pc - 1, s0, pc, tSx, tPx, Ul, Wl, Jl);
            face(s0, pc, s0, pc + 1, tSx, tPx, Uh, Wh, Jh);
#pragma unroll
            for (int a = 0; a < NP; ++a) Gs[a] = Uh[a] - Wl[a];
#pragma unroll
            for (int k = 0; k < NM; ++k) Js[k] = Jh[k] - Jl[k];
        }
        {
            R Ul[NP], Wl[NP], Jl[NM], Uh[NP], Wh[NP], Jh[NM];
            face(s0, pc - PW, s0, pc, tSy, tPy, Ul, Wl, Jl);
            face(s0, pc, s0, pc + PW, tSy, tPy, Uh, Wh, Jh);
#pragma unroll
            for (int a = 0; a < NP; ++a) Gs[a] = Gs[a] + (Uh[a] - Wl[a]);
#pragma unroll
            for (int k = 0; k < NM; ++k) Js[k] = Js[k] + (Jh[k] - Jl[k]);
        }
        {
            R Uh[NP], Wh[NP], Jh[NM];
            face(s0, pc, sp1, pc, tSz, tPz, Uh, Wh, Jh);
#pragma unroll
            for (int a = 0; a < NP; ++a) {
                Gs[a] = Gs[a] + (Uh[a] - Wlo[a]);
                Wlo[a] = Wh[a];
            }
#pragma unroll
            for (int k = 0; k < NM; ++k) {
                Js[k] = Js[k] + (Jh[k] - Jlo[k]);
                Jlo[k] = Jh[k];
            }
        }

        R phi[NP], mu[NM], h0[NP];
#pragma unroll
        for (int a = 0; a < NP; ++a) phi[a] = sv[s0][a][pc];
#pragma unroll
        for (int k = 0; k < NM; ++k) mu[k] = sv[s0][NP + k][pc];
        interp_h<R, NP>(phi, h0);
        R phin[NP], mun[NM];
        R h1[NP];
        cell_update_any<R, NP, NM, OBST, GEN>(phi, mu, h0, Gs, Js, Cs, tt, c, x, phin, mun, h1);

        if (valid) {
            const int64_t o = (int64_t)gx + (int64_t)gy * sy + (int64_t)m * sz;
#pragma unroll
            for (int a = 0; a < NP; ++a) out[a * fs + o] = phin[a];
#pragma unroll
            for (int k = 0; k < NM; ++k) out[(NP + k) * fs + o] = mun[k];
            if constexpr (DIAG) {
                double p[NP], u[NM];
#pragma unroll
                for (int a = 0; a < NP; ++a) p[a] = (double)phin[a];
#pragma unroll
                for (int k = 0; k < NM; ++k) u[k] = (double)mun[k];
                diag_cell<NP, NM, GEN>(p, u, dc->tt0 + dc->tslope * (double)gy, *dc, *da);
            }
        }

        if (m + 2 <= m1) stage(m + 2);
        __syncthreads();
    }
}

template <typename R, int NP, int NM, bool ANISO, bool OBST, int BX, int BY>
__global__ void __launch_bounds__(BX * BY)
k_step3d(const R* __restrict__ in, R* __restrict__ out, Geom g, Coef<R> c,
         const int64_t* __restrict__ stepctr, int kstep, double tb0, double tdn, double tslope,
         int seg, int ntx, int nty) {
    step3d_block<R, NP, NM, ANISO, OBST, BX, BY, false>(in, out, g, c, stepctr, kstep, tb0, tdn, tslope, seg,
                                                        ntx, nty, nullptr);
}

// The extended model's 3D kernel (64 x 4 tiles).
template <typename R, int NP, int NM, bool ANISO, bool OBST>
__global__ void __launch_bounds__(256)
k_step3d_gen(const R* __restrict__ in, R* __restrict__ out, Geom g, Coef<R> c,
             const int64_t* __restrict__ stepctr, int kstep, double tb0, double tdn, double tslope,
             int seg, int ntx, int nty, CoefX<R> x) {
    step3d_block<R, NP, NM, ANISO, OBST, 64, 4, true>(in, out, g, c, stepctr, kstep, tb0, tdn, tslope, seg,
                                                      ntx, nty, &x);
}

// The same tiles writing, beside the state, one partial diagnostics record
// per block (block b's at d.part + b * DIAG_VALS): the diagnostics of the
// state they store.
template <typename R, int NP, int NM, bool ANISO, bool OBST, int BX, int BY, bool GEN>
__global__ void __launch_bounds__(BX * BY)
k_step3d_diag(const R* __restrict__ in, R* __restrict__ out, Geom g, Coef<R> c,
              const int64_t* __restrict__ stepctr, int kstep, double tb0, double tdn, double tslope,
              int seg, int ntx, int nty, CoefX<R> x, DiagOut d) {
    constexpr int NW = BX * BY / 64;
    __shared__ double drec[NW][DIAG_VALS];
    DiagAcc A;
    acc_init(A);
    step3d_block<R, NP, NM, ANISO, OBST, BX, BY, GEN, true>(in, out, g, c, stepctr, kstep, tb0, tdn, tslope, seg,
                                                            ntx, nty, GEN ? &x : nullptr, &A, &d.dc);
    diag_wave_store(A, drec[threadIdx.x >> 6]);
    __syncthreads();
    if (threadIdx.x == 0) {
        DiagRec T;
        rec_load(T, drec[0]);
        for (int w = 1; w < NW; ++w) {
            DiagRec B;
            rec_load(B, drec[w]);
            rec_merge(T, B);
        }
        rec_store(d.part + (int64_t)blockIdx.x * DIAG_VALS, T);
    }
}

template <typename R, int NP, int NM, bool ANISO, bool OBST, int BY, bool GEN>
int call_3d_diag(const StepLaunch& L, const Coef<R>& c, const CoefX<R>& x, KernelCall& k) {
    constexpr int BX = 64;
    const int ntx = (L.g.nx + BX - 1) / BX;
    const int nty = (L.g.ny + BY - 1) / BY;
    const int nseg = (L.g.nz + L.seg - 1) / L.seg;
    const long long nblocks = (long long)ntx * nty * nseg;
    if (nblocks <= 0 || nblocks > 0x7fffffffLL || !L.diag) return MP_E_PARAM;
    k.func = (const void*)&k_step3d_diag<R, NP, NM, ANISO, OBST, BX, BY, GEN>;
    k.grid = dim3((unsigned)nblocks);
    k.block = dim3(BX * BY);
    k.nrec = nblocks;
    k.arg((const R*)L.in);
    k.arg((R*)L.out);
    k.arg(L.g);
    k.arg(c);
    k.arg(L.stepctr);
    k.arg(L.kstep);
    k.arg(L.tb0);
    k.arg(L.tdn);
    k.arg(L.tslope);
    k.arg(L.seg);
    k.arg(ntx);
    k.arg(nty);
    k.arg(x);
    k.arg(*L.diag);
    return MP_OK;
}

template <typename R, int NP, int NM, bool ANISO, bool OBST, bool DIAG = false>
int call_3d_gen(const StepLaunch& L, const Coef<R>& c, const CoefX<R>& x, KernelCall& k) {
    if constexpr (DIAG) return call_3d_diag<R, NP, NM, ANISO, OBST, 4, true>(L, c, x, k);
    const int ntx = (L.g.nx + 63) / 64;
    const int nty = (L.g.ny + 3) / 4;
    const int nseg = (L.g.nz + L.seg - 1) / L.seg;
    const long long nblocks = (long long)ntx * nty * nseg;
    if (nblocks <= 0 || nblocks > 0x7fffffffLL) return MP_E_PARAM;
    k.func = (const void*)&k_step3d_gen<R, NP, NM, ANISO, OBST>;
    k.grid = dim3((unsigned)nblocks);
    k.block = dim3(256);
    k.arg((const R*)L.in);
    k.arg((R*)L.out);
    k.arg(L.g);
    k.arg(c);
    k.arg(L.stepctr);
    k.arg(L.kstep);
    k.arg(L.tb0);
    k.arg(L.tdn);
    k.arg(L.tslope);
    k.arg(L.seg);
    k.arg(ntx);
    k.arg(nty);
    k.arg(x);
    return MP_OK;
}

template <typename R, int NP, int NM, bool ANISO, bool OBST, int BY>
int call_3d_by(const StepLaunch& L, const Coef<R>& c, KernelCall& k) {
    constexpr int BX = 64;
    const int ntx = (L.g.nx + BX - 1) / BX;
    const int nty = (L.g.ny + BY - 1) / BY;
    const int nseg = (L.g.nz + L.seg - 1) / L.seg;
    const long long nblocks = (long long)ntx * nty * nseg;
    if (nblocks <= 0 || nblocks > 0x7fffffffLL) return MP_E_PARAM;
    k.func = (const void*)&k_step3d<R, NP, NM, ANISO, OBST, BX, BY>;
    k.grid = dim3((unsigned)nblocks);
    k.block = dim3(BX * BY);
    k.arg((const R*)L.in);
    k.arg((R*)L.out);
    k.arg(L.g);
    k.arg(c);
    k.arg(L.stepctr);
    k.arg(L.kstep);
    k.arg(L.tb0);
    k.arg(L.tdn);
    k.arg(L.tslope);
    k.arg(L.seg);
    k.arg(ntx);
    k.arg(nty);
    return MP_OK;
}

// LDS bytes of a 64 x BY tile ring (4 planes of the fields and M~, with halo).
template <typename R, int NP, int NM, int BY>
constexpr int lds3d_bytes() {
    return 4 * (NP + 2 * NM) * 66 * (BY + 2) * (int)sizeof(R);
}

// bx = threads per block: 256 (64 x 4 tiles) or 512 (64 x 8 tiles, taller, so
// fewer y-halo rows are loaded per cell; only where the LDS ring stays small).
template <typename R, int NP, int NM, bool ANISO, bool OBST, bool DIAG = false>
int call_3d(const StepLaunch& L, const Coef<R>& c, KernelCall& k) {
    if constexpr (DIAG) {
        const CoefX<R> none{};
        if (L.bx == 512) {
            if constexpr (lds3d_bytes<R, NP, NM, 8>() <= 64 * 1024)
                return call_3d_diag<R, NP, NM, ANISO, OBST, 8, false>(L, c, none, k);
            return MP_E_PARAM;
        }
        return call_3d_diag<R, NP, NM, ANISO, OBST, 4, false>(L, c, none, k);
    } else {
        if (L.bx == 512) {
            if constexpr (lds3d_bytes<R, NP, NM, 8>() <= 64 * 1024)
                return call_3d_by<R, NP, NM, ANISO, OBST, 8>(L, c, k);
            return MP_E_PARAM;
        }
        return call_3d_by<R, NP, NM, ANISO, OBST, 4>(L, c, k);
    }
}

}  // namespace mp
