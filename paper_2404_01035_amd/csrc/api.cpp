// Host side of the C ABI declared in include/mp.h: validation, coefficient
// derivation, buffer bookkeeping and kernel dispatch.  mp_dt_limit,
// mp_create, mp_state_bytes, mp_workspace_bytes, mp_set_tile/mp_get_tile,
// mp_current/mp_set_step, mp_destroy and mp_last_error make no HIP call, so
// they work on a machine without a GPU.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "mp_internal.hpp"

struct mp_state {
    mp_grid grid;
    int N, K;  // phases, components (K - 1 diffusion potentials)
    mp_params prm;
    double dt_lim;
    void* buf[2];
    void* ws;
    bool bound;
    int cur;
    int64_t step;
    int bx, seg;
    bool aniso;
};

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char msg[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(msg, sizeof msg, fmt, ap);
    va_end(ap);
    g_err = msg;
    return code;
}

int ok() {
    g_err.clear();
    return MP_OK;
}

bool finite(double x) { return std::isfinite(x); }

int nmu_of(const mp_state* st) { return st->K - 1; }
int nfields_of(const mp_state* st) { return st->N + st->K - 1; }

int64_t ncells_of(const mp_grid& g) { return g.n[0] * g.n[1] * g.n[2]; }

int check_grid(const mp_grid* g) {
    if (!g) return fail(MP_E_NULLPTR, "grid is NULL");
    if (g->dim != 2 && g->dim != 3) return fail(MP_E_PARAM, "dim must be 2 or 3 (got %d)", g->dim);
    for (int i = 0; i < 3; ++i) {
        if (g->n[i] < 1 || g->n[i] > (int64_t)1 << 30)
            return fail(MP_E_PARAM, "n[%d] = %lld out of range [1, 2^30]", i, (long long)g->n[i]);
        if (g->bc[i] != MP_BC_PERIODIC && g->bc[i] != MP_BC_NOFLUX)
            return fail(MP_E_PARAM, "bc[%d] = %d is not MP_BC_PERIODIC or MP_BC_NOFLUX", i, g->bc[i]);
    }
    if (g->dim == 2 && g->n[2] != 1) return fail(MP_E_PARAM, "2D grid needs n[2] = 1");
    if (!(g->dx > 0.0) || !finite(g->dx)) return fail(MP_E_PARAM, "dx must be positive and finite");
    return MP_OK;
}

int check_params(int N, int K, const mp_params* p) {
    if (!p) return fail(MP_E_NULLPTR, "params is NULL");
    if (N != 2 && N != 3) return fail(MP_E_PARAM, "nphases must be 2 or 3 (got %d)", N);
    if (K != 2 && K != 3) return fail(MP_E_PARAM, "ncomp must be 2 or 3 (got %d)", K);
    if (p->precision != MP_FP64 && p->precision != MP_FP32)
        return fail(MP_E_PARAM, "precision must be MP_FP64 or MP_FP32");
    if (p->potential != MP_WELL && p->potential != MP_OBSTACLE)
        return fail(MP_E_PARAM, "potential must be MP_WELL or MP_OBSTACLE");
    if (!(p->eps > 0) || !finite(p->eps)) return fail(MP_E_PARAM, "eps must be positive and finite");
    if (!(p->tau > 0)) return fail(MP_E_PARAM, "tau must be positive");
    if (!(p->dt > 0) || !finite(p->dt)) return fail(MP_E_PARAM, "dt must be positive and finite");
    for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b) {
            if (a == b) continue;
            if (!(p->gamma[a][b] > 0) || !finite(p->gamma[a][b]))
                return fail(MP_E_PARAM, "gamma[%d][%d] must be positive and finite", a, b);
            if (p->gamma[a][b] != p->gamma[b][a])
                return fail(MP_E_PARAM, "gamma must be symmetric (gamma[%d][%d])", a, b);
            if (!(p->delta[a][b] >= 0.0) || !(p->delta[a][b] < 1.0 / 3.0))
                return fail(MP_E_PARAM, "delta[%d][%d] must lie in [0, 1/3)", a, b);
            if (p->delta[a][b] != p->delta[b][a])
                return fail(MP_E_PARAM, "delta must be symmetric (delta[%d][%d])", a, b);
        }
    if (!finite(p->gamma3)) return fail(MP_E_PARAM, "gamma3 must be finite");
    for (int a = 0; a < N; ++a) {
        if (!finite(p->C[a]) || !finite(p->s[a])) return fail(MP_E_PARAM, "C/s must be finite");
        for (int k = 0; k < K - 1; ++k) {
            if (!(p->A[a][k] > 0) || !finite(p->A[a][k]))
                return fail(MP_E_PARAM, "A[%d][%d] must be positive and finite", a, k);
            if (!finite(p->B[a][k])) return fail(MP_E_PARAM, "B[%d][%d] must be finite", a, k);
            if (!(p->D[a][k] >= 0) || !finite(p->D[a][k]))
                return fail(MP_E_PARAM, "D[%d][%d] must be >= 0 and finite", a, k);
        }
    }
    if (!finite(p->Te) || !finite(p->T0) || !finite(p->G) || !finite(p->V) || !finite(p->y0))
        return fail(MP_E_PARAM, "temperature parameters must be finite");
    return MP_OK;
}

double dt_limit_of(const mp_grid* g, int N, int K, const mp_params* p) {
    double gmax = 0.0, dmax = 0.0;
    for (int a = 0; a < N; ++a)
        for (int b = a + 1; b < N; ++b) {
            gmax = std::fmax(gmax, p->gamma[a][b]);
            dmax = std::fmax(dmax, std::fabs(p->delta[a][b]));
        }
    const double base = g->dx * g->dx / (2.0 * g->dim);
    double lim = INFINITY;
    if (gmax > 0) lim = base * p->tau / (2.0 * gmax * (N - 1) / N * (1.0 + 20.0 * dmax));
    for (int k = 0; k < K - 1; ++k) {
        double top = 0.0, cmin = INFINITY;
        for (int a = 0; a < N; ++a) {
            const double chi = 1.0 / (2.0 * p->A[a][k]);
            top = std::fmax(top, p->D[a][k] * chi);
            cmin = std::fmin(cmin, chi);
        }
        if (top > 0) lim = std::fmin(lim, base * cmin / top);
    }
    return lim;
}

template <typename R>
mp::Coef<R> make_coef(const mp_state* st) {
    const mp_params& p = st->prm;
    const double dx = st->grid.dx;
    mp::Coef<R> c;
    std::memset(&c, 0, sizeof c);
    c.cE = (R)(p.eps / (2.0 * dx));
    c.inv_eps = (R)(1.0 / p.eps);
    c.kphi = (R)(p.dt / (p.tau * p.eps));
    c.qguard = (R)(4.0 * dx * dx * 1e-30);
    const double wfac = p.potential == MP_OBSTACLE ? 16.0 / (M_PI * M_PI) : 18.0;
    const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
    for (int q = 0; q < 3; ++q) {
        const double g = p.gamma[pa[q]][pb[q]];
        c.g2d[q] = (R)(2.0 * g / dx);
        c.gd[q] = (R)(g / dx);
        c.del[q] = (R)p.delta[pa[q]][pb[q]];
        c.wc[q] = (R)(wfac * g);
    }
    c.gamma3 = (R)p.gamma3;
    const double dtf = p.dt / (2.0 * dx * dx);
    for (int a = 0; a < st->N; ++a) {
        c.C[a] = (R)p.C[a];
        c.s[a] = (R)p.s[a];
        for (int k = 0; k < st->K - 1; ++k) {
            const double chi = 1.0 / (2.0 * p.A[a][k]);
            c.chi[a][k] = (R)chi;
            c.halfchi[a][k] = (R)(0.5 * chi);
            c.B[a][k] = (R)p.B[a][k];
            c.Dt[a][k] = (R)(p.D[a][k] * chi * dtf);
        }
    }
    return c;
}

mp::Geom make_geom(const mp_state* st) {
    mp::Geom g;
    g.nx = (int32_t)st->grid.n[0];
    g.ny = (int32_t)st->grid.n[1];
    g.nz = (int32_t)st->grid.n[2];
    g.bcx = st->grid.bc[0];
    g.bcy = st->grid.bc[1];
    g.bcz = st->grid.bc[2];
    g.fstride = ncells_of(st->grid);
    return g;
}

int hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) return fail(MP_E_HIP, "%s: %s", what, hipGetErrorString(e));
    return MP_OK;
}

}  // namespace

namespace mp {
int launch_step_f64(const StepLaunch& L, const Coef<double>& c, hipStream_t s) {
    return L.dim == 3 ? launch_step_dim<double, true>(L, c, s) : launch_step_dim<double, false>(L, c, s);
}
int launch_step_f32(const StepLaunch& L, const Coef<float>& c, hipStream_t s) {
    return L.dim == 3 ? launch_step_dim<float, true>(L, c, s) : launch_step_dim<float, false>(L, c, s);
}
}  // namespace mp

extern "C" {

double mp_dt_limit(const mp_grid* grid, int nphases, int ncomp, const mp_params* params) {
    if (check_grid(grid) != MP_OK) return -1.0;
    if (check_params(nphases, ncomp, params) != MP_OK) return -1.0;
    ok();
    return dt_limit_of(grid, nphases, ncomp, params);
}

int mp_create(const mp_grid* grid, int nphases, int ncomp, const mp_params* params, mp_state** out) {
    if (!out) return fail(MP_E_NULLPTR, "out is NULL");
    *out = nullptr;
    int rc = check_grid(grid);
    if (rc) return rc;
    rc = check_params(nphases, ncomp, params);
    if (rc) return rc;
    const double lim = dt_limit_of(grid, nphases, ncomp, params);
    if (params->dt > lim * (1.0 + 1e-12))
        return fail(MP_E_UNSTABLE, "dt = %.17g exceeds the explicit stability limit %.17g",
                    params->dt, lim);
    const int64_t nc = ncells_of(*grid);
    if (nc * (nphases + ncomp - 1) > ((int64_t)1 << 40))
        return fail(MP_E_PARAM, "grid too large");
    mp_state* st = new (std::nothrow) mp_state();
    if (!st) return fail(MP_E_PARAM, "out of host memory");
    st->grid = *grid;
    st->N = nphases;
    st->K = ncomp;
    st->prm = *params;
    st->dt_lim = lim;
    st->buf[0] = st->buf[1] = nullptr;
    st->ws = nullptr;
    st->bound = false;
    st->cur = 0;
    st->step = 0;
    st->aniso = false;
    for (int a = 0; a < nphases; ++a)
        for (int b = a + 1; b < nphases; ++b)
            if (params->delta[a][b] != 0.0) st->aniso = true;
    if (grid->dim == 3) {
        st->bx = 64;
        st->seg = 16;
    } else {
        // measured best on 4096^2 (both precisions): short segments keep enough
        // waves in flight to cover HBM latency
        st->bx = 256;
        st->seg = 16;
    }
    *out = st;
    return ok();
}

size_t mp_state_bytes(const mp_state* st) {
    if (!st) return 0;
    const size_t el = st->prm.precision == MP_FP64 ? sizeof(double) : sizeof(float);
    return (size_t)ncells_of(st->grid) * (size_t)nfields_of(st) * el;
}

size_t mp_workspace_bytes(const mp_state* st) {
    if (!st) return 0;
    return (size_t)(mp::DIAG_BLOCKS_MAX + 1) * mp::DIAG_VALS * sizeof(double);
}

int mp_bind(mp_state* st, void* buf0, void* buf1, void* workspace) {
    if (!st) return fail(MP_E_NULLPTR, "state is NULL");
    if (!buf0 || !buf1 || !workspace) return fail(MP_E_NULLPTR, "buffer pointer is NULL");
    if (buf0 == buf1) return fail(MP_E_PARAM, "buf0 and buf1 must differ");
    if (((uintptr_t)buf0 | (uintptr_t)buf1 | (uintptr_t)workspace) & 255u)
        return fail(MP_E_PARAM, "buffers must be 256-byte aligned");
    st->buf[0] = buf0;
    st->buf[1] = buf1;
    st->ws = workspace;
    st->bound = true;
    st->cur = 0;
    st->step = 0;
    return ok();
}

int mp_step(mp_state* st, int64_t nsteps, void* stream) {
    if (!st) return fail(MP_E_NULLPTR, "state is NULL");
    if (!st->bound) return fail(MP_E_UNBOUND, "mp_step before mp_bind");
    if (nsteps < 0) return fail(MP_E_PARAM, "nsteps must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    mp::StepLaunch L;
    L.g = make_geom(st);
    L.nphases = st->N;
    L.nmu = nmu_of(st);
    L.dim = st->grid.dim;
    L.potential = st->prm.potential;
    L.aniso = st->aniso ? 1 : 0;
    L.bx = st->bx;
    L.seg = st->seg;
    const mp_params& p = st->prm;
    const bool f64 = p.precision == MP_FP64;
    mp::Coef<double> cd;
    mp::Coef<float> cf;
    if (f64)
        cd = make_coef<double>(st);
    else
        cf = make_coef<float>(st);
    for (int64_t i = 0; i < nsteps; ++i) {
        const double t = (double)(st->step) * p.dt;
        // T(y) - Te = T0 + G (j dx - y0 - V t) - Te
        L.tbase = p.T0 - p.Te - p.G * (p.y0 + p.V * t);
        L.tslope = p.G * st->grid.dx;
        L.in = st->buf[st->cur];
        L.out = st->buf[1 - st->cur];
        const int rc = f64 ? mp::launch_step_f64(L, cd, s) : mp::launch_step_f32(L, cf, s);
        if (rc) return fail(rc, "no kernel instance for this configuration");
        const int hr = hip_check(hipGetLastError(), "step kernel launch");
        if (hr) return hr;
        st->cur = 1 - st->cur;
        st->step += 1;
    }
    return ok();
}

int mp_current(const mp_state* st, int* which_buf, int64_t* step) {
    if (!st) return fail(MP_E_NULLPTR, "state is NULL");
    if (which_buf) *which_buf = st->cur;
    if (step) *step = st->step;
    return ok();
}

int mp_set_step(mp_state* st, int64_t step, int which_buf) {
    if (!st) return fail(MP_E_NULLPTR, "state is NULL");
    if (which_buf != 0 && which_buf != 1) return fail(MP_E_PARAM, "which_buf must be 0 or 1");
    if (step < 0) return fail(MP_E_PARAM, "step must be >= 0");
    st->step = step;
    st->cur = which_buf;
    return ok();
}

int mp_diagnostics(mp_state* st, mp_diag* out, void* stream) {
    if (!st || !out) return fail(MP_E_NULLPTR, "state or out is NULL");
    if (!st->bound) return fail(MP_E_UNBOUND, "mp_diagnostics before mp_bind");
    hipStream_t s = (hipStream_t)stream;
    mp::DiagCoef dc;
    std::memset(&dc, 0, sizeof dc);
    for (int a = 0; a < st->N; ++a)
        for (int k = 0; k < st->K - 1; ++k) {
            dc.chi[a][k] = 1.0 / (2.0 * st->prm.A[a][k]);
            dc.B[a][k] = st->prm.B[a][k];
        }
    dc.vol = std::pow(st->grid.dx, st->grid.dim);
    mp::Geom g = make_geom(st);
    double* ws = (double*)st->ws;
    int rc = mp::launch_diag(st->buf[st->cur], st->prm.precision, g, st->N, nmu_of(st), dc, ws, s);
    if (rc) return fail(rc, "no diagnostics instance");
    rc = hip_check(hipGetLastError(), "diagnostics launch");
    if (rc) return rc;
    double r[mp::DIAG_VALS];
    rc = hip_check(hipMemcpyAsync(r, ws + (size_t)mp::DIAG_BLOCKS_MAX * mp::DIAG_VALS, sizeof r,
                                  hipMemcpyDeviceToHost, s),
                   "diagnostics copy");
    if (rc) return rc;
    rc = hip_check(hipStreamSynchronize(s), "diagnostics sync");
    if (rc) return rc;
    std::memset(out, 0, sizeof *out);
    out->step = st->step;
    for (int k = 0; k < nmu_of(st); ++k) {
        out->mass[k] = r[mp::DV_MASS + 2 * k] + r[mp::DV_MASS + 2 * k + 1];
        out->min_chi[k] = r[mp::DV_MINCHI + k];
    }
    for (int a = 0; a < st->N; ++a) out->volume[a] = r[mp::DV_VOL + 2 * a] + r[mp::DV_VOL + 2 * a + 1];
    out->max_sum_dev = r[mp::DV_MAXDEV];
    out->nonfinite = (int64_t)r[mp::DV_NONFIN];
    if (out->nonfinite > 0)
        return fail(MP_E_NONFINITE, "%lld cells hold NaN or Inf", (long long)out->nonfinite);
    return ok();
}

int mp_set_tile(mp_state* st, int bx, int seg) {
    if (!st) return fail(MP_E_NULLPTR, "state is NULL");
    if (bx) {
        const bool okbx = st->grid.dim == 3 ? bx == 64 : (bx == 64 || bx == 128 || bx == 256);
        if (!okbx) return fail(MP_E_PARAM, "unsupported tile width %d", bx);
        st->bx = bx;
    }
    if (seg) {
        if (seg < 1) return fail(MP_E_PARAM, "seg must be >= 1");
        st->seg = seg;
    }
    return ok();
}

int mp_get_tile(const mp_state* st, int* bx, int* seg) {
    if (!st) return fail(MP_E_NULLPTR, "state is NULL");
    if (bx) *bx = st->bx;
    if (seg) *seg = st->seg;
    return ok();
}

void mp_destroy(mp_state* st) { delete st; }

const char* mp_last_error(void) { return g_err.c_str(); }

}  // extern "C"
