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
    R inv_eps;     // 1 / eps
    R kphi;        // dt / (tau eps)
    R qguard;      // (2 dx)^2 * 1e-30, the |q|^2 guard on the rescaled q
    R g2d[3];      // 2 gamma_ab / dx (isotropic pair factor)
    R gd[3];       // gamma_ab / dx (anisotropic pair factor)
    R del[3];      // delta_ab
    R wc[3];       // 18 gamma_ab (multi-well) or 16/pi^2 gamma_ab (obstacle)
    R gamma3;      // gamma_abd
    R chi[3][2];   // 1 / (2 A)
    R halfchi[3][2];  // 1 / (4 A)
    R B[3][2];
    R C[3];
    R s[3];
    R Dt[3][2];    // D chi dt / (2 dx^2)
};

// Coefficients the FP64 diagnostics reduction needs.
struct DiagCoef {
    double chi[3][2];
    double B[3][2];
    double vol;      // dx^d
};

// One launch of the fused step kernel.
struct StepLaunch {
    const void* in;
    void* out;
    Geom g;
    int nphases, nmu, dim, potential, aniso;
    int bx, seg;
    double tbase, tslope;  // T(y) - Te = tbase + tslope * j for row j at this step
};

constexpr int DIAG_BLOCKS_MAX = 1024;
constexpr int DIAG_VALS = 16;  // per-block partial record, doubles
// record layout: mass (sum, comp) x2, volume (sum, comp) x3, max_dev, min_chi x2, nonfinite
constexpr int DV_MASS = 0, DV_VOL = 4, DV_MAXDEV = 10, DV_MINCHI = 11, DV_NONFIN = 13;

int launch_step_f64(const StepLaunch& L, const Coef<double>& c, hipStream_t s);
int launch_step_f32(const StepLaunch& L, const Coef<float>& c, hipStream_t s);
template <typename R, bool D3>
int launch_step_dim(const StepLaunch& L, const Coef<R>& c, hipStream_t s);

int launch_diag(const void* state, int precision, const Geom& g, int nphases, int nmu,
                const DiagCoef& dc, double* ws, hipStream_t s);
int diag_blocks(int64_t ncells);

}  // namespace mp
