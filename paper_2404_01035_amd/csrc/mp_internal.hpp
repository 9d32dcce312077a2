// Internal declarations shared by the host API (api.cpp) and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/mp.h"

namespace mp {

// Grid geometry as the kernels see it.  In 2D nz = 1 and the march axis
// (the slowest one, walked by each block) is y; in 3D it is z.
struct Geom {
    int32_t nx, ny, nz;
    int32_t bcx, bcy, bcz;  // MP_BC_PERIODIC (0) or MP_BC_NOFLUX (1)
    int64_t fstride;        // elements per field = nx * ny * nz
};

// Model coefficients in the run precision R, derived once on the host in
// FP64 and folded for the face/cell arithmetic of gp_device.hpp.
// Pair index: (0,1) -> 0, (0,2) -> 1, (1,2) -> 2.
template <typename R>
struct Coef {
    R cE;          // eps / (2 dx)
    R kphi;        // dt / (tau eps)
    R qguard;      // (2 dx)^2 * 1e-30, the |q|^2 guard on the rescaled q
    R g4d[3];      // 4 gamma_ab / dx (isotropic pair factor on phi_L,i phi_R,j - phi_L,j phi_R,i)
    R gd[3];       // gamma_ab / dx (anisotropic pair factor)
    R del[3];      // delta_ab
    R wce[3];      // 18 gamma_ab / eps (multi-well) or 16/pi^2 gamma_ab / eps (obstacle)
    R g3e;         // gamma_abd / eps
    R chi[3][2];   // 1 / (2 A)
    R B[3][2];
    R C[3];
    R s[3];
    R Dt[3][2];    // D chi dt / (2 dx^2)
};

// Terms of the extended model, read only by the general (GEN) kernels:
// temperature-dependent B and C (Sec. 3), the dT/dt term of Eq.
// Mu_explicit_temperature, off-diagonal susceptibility and mobility (Eq.
// free_energy_density with the i < j term, Eq. Mass_conservation with a full
// D), per-pair relaxation constants and the active-set obstacle projection.
template <typename R>
struct CoefX {
    R Bt[3][2];     // B^a_k(T) = B^a_k + Bt^a_k (T - Te)
    R Ct[3];        // C^a(T) = C^a + s^a (T - Te) + Ct^a (T - Te)^2
    R chx[3];       // off-diagonal susceptibility (chi^a)_01 (K = 3); the diagonal is Coef::chi
    R Dx[3][2][2];  // scaled mobility (D^a chi^a)_kj dt / (2 dx^2)
    R th[3][2];     // Theta coefficient (dc^a_k/dT) (T^{n+1} - T^n) = -(chi^a Bt^a)_k (T^{n+1} - T^n)
    R tab[3];       // per-pair relaxation constants tau_ab (pair index)
    R ktau;         // dt / eps
    int32_t tpair;  // 1: tau(phi) from tab; 0: the single tau (Coef::kphi)
    int32_t proj;   // obstacle projection: 0 clip and renormalise, 1 onto the simplex (active set)
    int32_t well1;  // 1: the KKS potential of Eq. Well1 (its pair terms sit in Coef::wce)
    R th1[3];       // 2 Theta_a
    R th3;          // 2 Theta_abd
};

// Coefficients the FP64 diagnostics reduction needs.
// c^a(mu) = chi^a (mu - B^a - Bt^a (T - Te)), so
// c^a_k = chi_kk mu_k + chi_01 mu_{1-k} - cb_k - cbt_k (T - Te).
struct DiagCoef {
    double chi[3][2];  // chi^a_kk
    double chx[3];     // chi^a_01 (K = 3)
    double cb[3][2];   // (chi^a B^a)_k
    double cbt[3][2];  // (chi^a Bt^a)_k (the extended model's B^a(T))
    double tt0;        // T - Te at row 0 of the reduced state's time level
    double tslope;   // T - Te per row
    int32_t nx, ny;  // rows: cell i lies in row (i / nx) mod ny
};

// Where a step kernel leaves the diagnostics of the state it stores: one
// partial record of DIAG_VALS doubles per wave (2D strips) or per block (3D
// tiles), reduced afterwards by the diagnostics' final kernel.
struct DiagOut {
    double* part;
    DiagCoef dc;
};

// One launch of the fused step kernel.  The time level of the launch is
// *stepctr + kstep (the counter lives in device memory so that a replayed
// graph of launches stays correct); T - Te at row j is
// tb0 + tdn * n + tslope * j.
struct StepLaunch {
    const void* in;
    void* out;
    void* out1 = nullptr;  // two steps per launch: also receives the state after the first
    Geom g;
    int nphases, nmu, dim, potential, aniso;
    int bx, seg, vec;
    int fuse;  // steps per launch: 1, or 2 (2D single grid)
    const int64_t* stepctr;
    int kstep;
    double tb0, tdn, tslope;
    const DiagOut* diag = nullptr;  // the diagnostics kernels: partial records of the stored state
};

// A kernel launch described as data: launched directly or added to a graph.
struct KernelCall {
    const void* func = nullptr;
    dim3 grid, block;
    alignas(16) unsigned char store[1024];
    size_t used = 0;
    void* args[16];
    int nargs = 0;
    bool bad = false;      // an argument did not fit: the call must not be launched
    long long nrec = 0;    // partial diagnostics records the launch writes
    template <typename T>
    void arg(const T& v) {
        const size_t at = (used + alignof(T) - 1) / alignof(T) * alignof(T);
        if (bad || nargs >= 16 || at + sizeof(T) > sizeof store) {
            bad = true;
            return;
        }
        __builtin_memcpy(store + at, &v, sizeof(T));
        args[nargs++] = store + at;
        used = at + sizeof(T);
    }
};

// One instance of a batch, as the batched kernel reads it from device memory.
template <typename R>
struct InstDesc {
    Geom g;
    int32_t np, nm;
    int32_t ntx, nseg, seg;         // work items: ntx strips by nseg row segments of seg rows
    int32_t vec;                    // cells per lane of the strip kernel (vec2d_width)
    int64_t off;                    // element offset of the instance's state
    double tb0, tdn, tslope;        // T - Te = tb0 + tdn * n + tslope * j
    Coef<R> c;
};

// First work item of each XCD's slice of a batch's work list, and its end.
struct BatchCuts {
    int32_t c[9];
};

// One launch of the batched 2D kernel.
struct BatchLaunch {
    const void* in;
    void* out;
    const void* table;  // InstDesc<R>[ninst] in device memory
    const int* items;   // work list in device memory: (instance, local item) pairs
    BatchCuts cuts;     // XCD x takes items cuts.c[x] .. cuts.c[x+1]-1
    int potential, aniso;
    int vmax;  // widest cells-per-lane among the items (1 or 2)
    int fuse;  // steps per launch (1 or 2)
    int nblocks;
    const int64_t* stepctr;
    int kstep;
};

constexpr int DIAG_BLOCKS_MAX = 1024;
constexpr int DIAG_VALS = 16;  // per-block partial record, doubles
// record layout: mass (sum, comp) x2, volume (sum, comp) x3, max_dev, min_chi x2, nonfinite
constexpr int DV_MASS = 0, DV_VOL = 4, DV_MAXDEV = 10, DV_MINCHI = 11, DV_NONFIN = 13;

int call_step_f64(const StepLaunch& L, const Coef<double>& c, KernelCall& k);
int call_step_f32(const StepLaunch& L, const Coef<float>& c, KernelCall& k);
// DIAG: the instances that also write the partial diagnostics records of the
// state they store (StepLaunch::diag), one per 2D strip wave or 3D tile.
template <typename R, bool D3, bool DIAG = false>
int call_step_dim(const StepLaunch& L, const Coef<R>& c, KernelCall& k);
// The general kernels of the extended model (one cell per lane in 2D, 64 x 4
// tiles in 3D).
template <typename R, bool D3, bool DIAG = false>
int call_step_gen(const StepLaunch& L, const Coef<R>& c, const CoefX<R>& x, KernelCall& k);
template <typename R>
int call_batch(const BatchLaunch& L, KernelCall& k);
void call_advance(int64_t* ctr, int64_t by, KernelCall& k);

// Adjoint (adjoint2d.hpp): plain coefficients and one reverse step.
template <typename R>
struct AdjCoef;
struct AdjLaunch;
template <typename R>
int adj_launch(const AdjLaunch& L, const AdjCoef<R>& c, hipStream_t s);
void adj_fill(double* p, int64_t n, double v, hipStream_t s);
void adj_reduce(const double* acc, int nrows, double* out, hipStream_t s);

// Cells per lane of the 2D strip kernel: the widest power of two up to
// min(16 / elem, cap) (cap <= 0: no cap) that divides the row length, so that
// each lane's cells form one aligned vector.  A strip wave writes
// W2D_LANES_OUT_HOST lanes' worth of columns.
__host__ __device__ inline int vec2d_width(int64_t nx, int elem, int cap) {
    int v = 16 / elem;
    while (cap > 0 && v > cap) v /= 2;
    for (; v > 1; v /= 2)
        if (nx % v == 0) return v;
    return 1;
}

// Written lanes per 2D strip wave (lanes 1..62; 0 and 63 hold the halo),
// waves per block of the batched kernel.
constexpr int W2D_LANES_OUT_HOST = 62;
constexpr int W2X_LANES_OUT_HOST = 60;  // the two-step strip keeps two halo lanes per side
constexpr int BATCH_WPB_HOST = 4;
inline int batch_waves_per_block_host() { return BATCH_WPB_HOST; }

// Anti-trapping current of Eq. jatr, applied to the mu^{n+1} of a finished 2D
// single-grid step (antitrap2d.hpp).
template <typename R>
struct AtCoef {
    R prefw;       // multi-well prefactor eps / (2 sqrt 2)
    R prefo;       // obstacle prefactor scale pi eps / 4
    int obstacle;  // 1: obstacle prefactor, 0: multi-well
    R rdx, rdt, dt;
    R chi[3][2];   // 1 / (2 A^a_k)
    R B[3][2];
};

struct AtLaunch {
    const void* prev;  // state n: phi^n, mu^n
    void* next;        // state n+1: phi^{n+1} read, mu^{n+1} corrected in place
    Geom g;
    int nphases, nmu;
};

template <typename R>
int at_launch(const AtLaunch& L, const AtCoef<R>& c, hipStream_t s);

int launch_diag(const void* state, int precision, const Geom& g, int nphases, int nmu,
                const DiagCoef& dc, double* partials, double* result, hipStream_t s);
int diag_blocks(int64_t ncells);
// The final reduction alone, over nrec partial records (fixed order).
int launch_diag_final(const double* partials, int64_t nrec, double* result, hipStream_t s);
// Most partial records one fused step launch may write (8 MiB of records).
constexpr int64_t FUSED_REC_MAX = 65536;

// Moving frame (frame.hip): the front row (partials: front_blocks ints) and
// the shift of a state by whole rows along y with melt appended.
int front_blocks(int64_t ncells);
int launch_front(const void* state, int precision, const Geom& g, int nphases, int* partials, int64_t* result,
                 hipStream_t s);
int launch_shift(const void* in, void* out, int precision, const Geom& g, int nphases, int nmu, int rows,
                 const double* mu_melt, hipStream_t s);

}  // namespace mp
