// Host side of the C ABI declared in include/mp.h: validation, coefficient
// derivation, buffer bookkeeping, kernel dispatch, graph replay and batching.
// mp_dt_limit, mp_create, mp_create_batch, mp_state_bytes,
// mp_workspace_bytes, mp_get_tile, mp_set_graph, mp_current,
// mp_instance_count/offset and mp_last_error make no HIP call, so they work
// on a machine without a GPU, and neither does mp_destroy unless mp_adjoint
// created its second stream; mp_set_step and mp_set_tile touch the device only
// once the state is bound.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "adjoint2d.hpp"
#include "diag_static.hpp"
#include "mp_internal.hpp"

namespace mp {
// step_at.hip: the 2D step with the anti-trapping current folded in; batch_at.hip: the same for a batch
template <typename R>
int call_step_at(const StepLaunch& L, const Coef<R>& c, const AtCoef<R>& ac, KernelCall& k);
template <typename R>
int call_step_at_gen(const StepLaunch& L, const Coef<R>& c, const AtCoef<R>& ac, const CoefX<R>& x, KernelCall& k);
// antitrap_gen.hip: the correction kernels for the extended model
template <typename R>
int at_launch_gen(const AtLaunch& L, const AtCoef<R>& c, const CoefX<R>& x, const int64_t* stepctr, int kstep,
                  double tb0, double tdn, double tslope, hipStream_t s);
template <typename R>
int call_batch_at(const BatchLaunch& L, const void* atab, KernelCall& k);
// batch_gen.hip: the batch of the extended model, plain and with the current
template <typename R>
int call_batch_gen(const BatchLaunch& L, const void* xtab, KernelCall& k);
template <typename R>
int call_batch_at_gen(const BatchLaunch& L, const void* atab, const void* xtab, KernelCall& k);
}  // namespace mp

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Inst {
    mp_grid grid;
    int N, K;
    mp_params prm;
    bool aniso;
    bool ext;                 // uses the extended model: the general kernels
    int64_t yshift;           // frame offset in rows (mp_shift)
    size_t off_bytes, bytes;  // within each state buffer
};

}  // namespace

struct mp_state {
    bool batch;
    std::vector<Inst> inst;
    int precision, potential;
    bool aniso;
    void* buf[2];
    void* ws;
    bool bound;
    int cur;
    int64_t step;
    int bx, seg, vec;  // vec: cap on cells per lane of the 2D strips (-1: none)
    int fuse;  // steps per launch of the step kernel: 1, or 2 (2D single grid)
    int antitrap;  // anti-trapping current: 0 off, 1 on (folded into the 2D step), 2 on (separate correction)
    int graph_chunk;
    hipGraphExec_t gexec[2];  // by starting buffer
    int gend[2];              // buffer current after a replay, by starting buffer
    std::vector<mp::KernelCall> gcalls[2];  // argument records of each graph's nodes, kept alive
    std::vector<int> items;  // batch work list (host copy): (instance, local item) pairs
    int nitems;
    mp::BatchCuts cuts;      // first item of each XCD's slice of the list, and the end
    int batch_blocks;
    // adjoint: a second stream (default priority) that recomputes the next
    // segment while the current one is swept, and the events ordering them
    hipStream_t aux;
    hipEvent_t ev[5];  // start, recomputed[2], swept[2]
};

namespace {

thread_local std::string g_err;

// MP_LOG set to anything but "0" or "": every failure message also goes to stderr.
bool log_enabled() {
    static const bool on = [] {
        const char* v = std::getenv("MP_LOG");
        return v && *v && std::strcmp(v, "0") != 0;
    }();
    return on;
}

int fail(int code, const char* fmt, ...) {
    char msg[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(msg, sizeof msg, fmt, ap);
    va_end(ap);
    g_err = msg;
    if (log_enabled()) fprintf(stderr, "[mpstep] error %d: %s\n", code, msg);
    return code;
}

int ok() {
    g_err.clear();
    return MP_OK;
}

bool finite(double x) { return std::isfinite(x); }

int64_t ncells_of(const mp_grid& g) { return g.n[0] * g.n[1] * g.n[2]; }

size_t elem_of(int precision) { return precision == MP_FP64 ? sizeof(double) : sizeof(float); }

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
    if (p->model != MP_GP && p->model != MP_KKS) return fail(MP_E_PARAM, "model must be MP_GP or MP_KKS");
    if (p->model == MP_GP && p->potential != MP_WELL && p->potential != MP_OBSTACLE &&
        p->potential != MP_OBSTACLE_ACTIVE)
        return fail(MP_E_PARAM, "potential must be MP_WELL, MP_OBSTACLE or MP_OBSTACLE_ACTIVE");
    if (p->model == MP_KKS && p->potential != MP_WELL && p->potential != MP_THETA)
        return fail(MP_E_PARAM, "the KKS variant takes MP_WELL (Eq. Well) or MP_THETA (Eq. Well1)");
    if (!(p->eps > 0) || !finite(p->eps)) return fail(MP_E_PARAM, "eps must be positive and finite");
    if (p->model == MP_GP && !(p->tau > 0)) return fail(MP_E_PARAM, "tau must be positive");
    if (p->model == MP_KKS) {
        if (!(p->Mphi > 0) || !finite(p->Mphi)) return fail(MP_E_PARAM, "Mphi must be positive and finite");
        if (!(p->theta3 >= 0) || !finite(p->theta3)) return fail(MP_E_PARAM, "theta3 must be >= 0 and finite");
        for (int a = 0; a < N; ++a) {
            if (!(p->theta[a] >= 0) || !finite(p->theta[a]))
                return fail(MP_E_PARAM, "theta[%d] must be >= 0 and finite", a);
            for (int b = 0; b < N; ++b) {
                if (a == b) continue;
                if (!(p->theta_ab[a][b] >= 0) || !finite(p->theta_ab[a][b]))
                    return fail(MP_E_PARAM, "theta_ab[%d][%d] must be >= 0 and finite", a, b);
                if (p->theta_ab[a][b] != p->theta_ab[b][a])
                    return fail(MP_E_PARAM, "theta_ab must be symmetric (theta_ab[%d][%d])", a, b);
                if (p->tau_ab[a][b] != 0.0)
                    return fail(MP_E_PARAM, "the KKS variant relaxes with Mphi: tau_ab must be 0");
            }
        }
    }
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
    // extended model
    bool anypair = false, allpair = true;
    for (int a = 0; a < N; ++a)
        for (int b = a + 1; b < N; ++b) {
            const double t = p->tau_ab[a][b];
            if (!finite(t) || t < 0.0) return fail(MP_E_PARAM, "tau_ab[%d][%d] must be >= 0 and finite", a, b);
            if (t != p->tau_ab[b][a]) return fail(MP_E_PARAM, "tau_ab must be symmetric (tau_ab[%d][%d])", a, b);
            anypair = anypair || t > 0.0;
            allpair = allpair && t > 0.0;
        }
    if (anypair && !allpair) return fail(MP_E_PARAM, "tau_ab: every pair > 0, or all 0");
    for (int a = 0; a < N; ++a) {
        if (!finite(p->Ct[a])) return fail(MP_E_PARAM, "Ct[%d] must be finite", a);
        for (int k = 0; k < K - 1; ++k)
            if (!finite(p->Bt[a][k])) return fail(MP_E_PARAM, "Bt[%d][%d] must be finite", a, k);
        if (K == 3) {
            if (!finite(p->A01[a]) || !finite(p->D01[a])) return fail(MP_E_PARAM, "A01/D01[%d] must be finite", a);
            if (!(4.0 * p->A[a][0] * p->A[a][1] - p->A01[a] * p->A01[a] > 0.0))
                return fail(MP_E_PARAM, "phase %d: the curvature matrix [[2A0, A01], [A01, 2A1]] must be positive definite", a);
            if (!(p->D[a][0] * p->D[a][1] - p->D01[a] * p->D01[a] >= 0.0))
                return fail(MP_E_PARAM, "phase %d: the diffusivity matrix [[D0, D01], [D01, D1]] must be positive semidefinite", a);
        }
    }
    return MP_OK;
}

// Susceptibility chi^a = (H^a)^-1 of phase a, H^a = [[2 A0, A01], [A01, 2 A1]]
// (K = 3) or 2 A0 (K = 2); the plain 1 / (2 A) where there is no cross term.
void chi_of(const mp_params& p, int a, int K, double chi[2][2]) {
    chi[0][0] = chi[0][1] = chi[1][0] = chi[1][1] = 0.0;
    if (K == 3 && p.A01[a] != 0.0) {
        const double det = 4.0 * p.A[a][0] * p.A[a][1] - p.A01[a] * p.A01[a];
        chi[0][0] = 2.0 * p.A[a][1] / det;
        chi[1][1] = 2.0 * p.A[a][0] / det;
        chi[0][1] = chi[1][0] = -p.A01[a] / det;
        return;
    }
    for (int k = 0; k < K - 1; ++k) chi[k][k] = 1.0 / (2.0 * p.A[a][k]);
}

// Diffusivity matrix D^a (the off-diagonal entry for K = 3).
void diff_of(const mp_params& p, int a, int K, double D[2][2]) {
    D[0][0] = p.D[a][0];
    D[1][1] = K == 3 ? p.D[a][1] : 0.0;
    D[0][1] = D[1][0] = K == 3 ? p.D01[a] : 0.0;
}

// The kernels' potential switch: Eq. Well1 runs in the multi-well kernels
// (general instances, CoefX::well1).
int kernel_potential(int potential) { return potential == MP_THETA ? MP_WELL : potential; }

bool uses_extended(int N, int K, const mp_params& p) {
    if (p.potential == MP_OBSTACLE_ACTIVE || p.potential == MP_THETA) return true;
    for (int a = 0; a < N; ++a) {
        if (p.Ct[a] != 0.0) return true;
        for (int k = 0; k < K - 1; ++k)
            if (p.Bt[a][k] != 0.0) return true;
        if (K == 3 && (p.A01[a] != 0.0 || p.D01[a] != 0.0)) return true;
        for (int b = a + 1; b < N; ++b)
            if (p.tau_ab[a][b] != 0.0) return true;
    }
    return false;
}

double dt_limit_of(const mp_grid* g, int N, int K, const mp_params* p) {
    double gmax = 0.0, dmax = 0.0, tau = p->tau;
    for (int a = 0; a < N; ++a)
        for (int b = a + 1; b < N; ++b) {
            gmax = std::fmax(gmax, p->gamma[a][b]);
            dmax = std::fmax(dmax, std::fabs(p->delta[a][b]));
            if (p->tau_ab[a][b] > 0.0) tau = std::fmin(tau, p->tau_ab[a][b]);
        }
    const double base = g->dx * g->dx / (2.0 * g->dim);
    double lim = INFINITY;
    if (p->model == MP_KKS) {
        // Eq. aceq: the gradient term's coefficient is Mphi eps^2/2 where the
        // grand-potential model has 1/tau; the potential's stiffness
        // max_a d^2 g/dphi_a^2 <= S bounds dt Mphi S <= 1 as well
        tau = 2.0 / (p->Mphi * p->eps * p->eps);
        double S = 0.0;
        for (int a = 0; a < N; ++a) {
            double sa = p->potential == MP_THETA ? 2.0 * p->theta[a] : 0.0;
            for (int b = 0; b < N; ++b)
                if (b != a) sa += p->potential == MP_THETA ? 2.0 * p->theta_ab[a][b] : 18.0 * p->gamma[a][b];
            S = std::fmax(S, sa);
        }
        if (S > 0) lim = 1.0 / (p->Mphi * S);
    }
    if (gmax > 0) lim = std::fmin(lim, base * tau / (2.0 * gmax * (N - 1) / N * (1.0 + 20.0 * dmax)));
    bool cross = false;
    for (int a = 0; a < N && K == 3; ++a) cross = cross || p->A01[a] != 0.0 || p->D01[a] != 0.0;
    if (cross) {
        // eigenvalues of chi^-1 M are at most max_a |D^a chi^a|_2 / min_a lambda_min(chi^a)
        double lmin = INFINITY, top = 0.0;
        for (int a = 0; a < N; ++a) {
            double c[2][2], D[2][2];
            chi_of(*p, a, K, c);
            diff_of(*p, a, K, D);
            lmin = std::fmin(lmin, 0.5 * (c[0][0] + c[1][1]) -
                                       std::sqrt(0.25 * (c[0][0] - c[1][1]) * (c[0][0] - c[1][1]) + c[0][1] * c[0][1]));
            double m[2][2];
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) m[i][j] = D[i][0] * c[0][j] + D[i][1] * c[1][j];
            const double sa = m[0][0] * m[0][0] + m[1][0] * m[1][0];
            const double sb = m[0][0] * m[0][1] + m[1][0] * m[1][1];
            const double sc = m[0][1] * m[0][1] + m[1][1] * m[1][1];
            top = std::fmax(top, std::sqrt(0.5 * (sa + sc) + std::sqrt(0.25 * (sa - sc) * (sa - sc) + sb * sb)));
        }
        if (top > 0) lim = std::fmin(lim, base * lmin / top);
        return lim;
    }
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

// Full validation of one problem, as mp_create does it.
int validate(const mp_grid* grid, int N, int K, const mp_params* p, const char* who) {
    int rc = check_grid(grid);
    if (rc) return rc;
    rc = check_params(N, K, p);
    if (rc) return rc;
    const double lim = dt_limit_of(grid, N, K, p);
    if (p->dt > lim * (1.0 + 1e-12))
        return fail(MP_E_UNSTABLE, "%sdt = %.17g exceeds the explicit stability limit %.17g", who,
                    p->dt, lim);
    if (ncells_of(*grid) * (N + K - 1) > ((int64_t)1 << 40)) return fail(MP_E_PARAM, "grid too large");
    return MP_OK;
}

Inst make_inst(const mp_grid* g, int N, int K, const mp_params* p) {
    Inst I;
    I.grid = *g;
    I.N = N;
    I.K = K;
    I.prm = *p;
    I.aniso = false;
    for (int a = 0; a < N; ++a)
        for (int b = a + 1; b < N; ++b)
            if (p->delta[a][b] != 0.0) I.aniso = true;
    I.ext = uses_extended(N, K, *p);
    I.yshift = 0;
    I.bytes = (size_t)ncells_of(*g) * (size_t)(N + K - 1) * elem_of(p->precision);
    I.off_bytes = 0;
    return I;
}

template <typename R>
mp::Coef<R> make_coef(const Inst& I) {
    const mp_params& p = I.prm;
    const double dx = I.grid.dx;
    mp::Coef<R> c;
    std::memset(&c, 0, sizeof c);
    const bool kks = p.model == MP_KKS;
    // the bracket of Eq. phi_eqn is eps G - w_{,a}/eps - psi_{,a} - lambda with
    // the rate 1/(tau eps); that of Eq. aceq (KKS) is eps^2/2 G - g_{,a} -
    // psi_{,a} - lambda with the rate Mphi
    c.cE = (R)((kks ? 0.5 * p.eps * p.eps : p.eps) / (2.0 * dx));
    c.kphi = (R)(kks ? p.dt * p.Mphi : p.dt / (p.tau * p.eps));
    c.qguard = (R)(4.0 * dx * dx * 1e-30);
    const double wfac = p.potential == MP_OBSTACLE || p.potential == MP_OBSTACLE_ACTIVE ? 16.0 / (M_PI * M_PI)
                                                                                        : 18.0;
    const double weps = kks ? 1.0 : p.eps;
    const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
    for (int q = 0; q < 3; ++q) {
        const double g = p.gamma[pa[q]][pb[q]];
        c.g4d[q] = (R)(4.0 * g / dx);
        c.gd[q] = (R)(g / dx);
        c.del[q] = (R)p.delta[pa[q]][pb[q]];
        // Eq. Well1's pair term Theta_ab phi_a^2 phi_b^2 has the form of Eq. Well's 9 gamma_ab
        c.wce[q] = (R)(p.potential == MP_THETA ? 2.0 * p.theta_ab[pa[q]][pb[q]] : wfac * g / weps);
    }
    c.g3e = (R)(p.potential == MP_THETA ? 0.0 : p.gamma3 / weps);
    const double dtf = p.dt / (2.0 * dx * dx);
    for (int a = 0; a < I.N; ++a) {
        c.C[a] = (R)p.C[a];
        c.s[a] = (R)p.s[a];
        double chi[2][2];
        chi_of(p, a, I.K, chi);
        for (int k = 0; k < I.K - 1; ++k) {
            c.chi[a][k] = (R)chi[k][k];
            c.B[a][k] = (R)p.B[a][k];
            c.Dt[a][k] = (R)(p.D[a][k] * chi[k][k] * dtf);
        }
    }
    return c;
}

// T - Te per step of the temperature law (T0 + G (y - y0 - V t), t = n dt).
double temperature_step(const Inst& I) { return -I.prm.G * I.prm.V * I.prm.dt; }

// The extended model's coefficients for the general kernels.
template <typename R>
mp::CoefX<R> make_coefx(const Inst& I) {
    const mp_params& p = I.prm;
    mp::CoefX<R> x;
    std::memset(&x, 0, sizeof x);
    const double dtf = p.dt / (2.0 * I.grid.dx * I.grid.dx);
    const double dT = temperature_step(I);
    const int K1 = I.K - 1;
    for (int a = 0; a < I.N; ++a) {
        double chi[2][2], D[2][2];
        chi_of(p, a, I.K, chi);
        diff_of(p, a, I.K, D);
        x.Ct[a] = (R)p.Ct[a];
        x.chx[a] = (R)(K1 == 2 ? chi[0][1] : 0.0);
        for (int k = 0; k < K1; ++k) {
            x.Bt[a][k] = (R)p.Bt[a][k];
            double cb = 0.0;
            for (int j = 0; j < K1; ++j) {
                cb += chi[k][j] * p.Bt[a][j];
                double dc = 0.0;
                for (int l = 0; l < K1; ++l) dc += D[k][l] * chi[l][j];
                x.Dx[a][k][j] = (R)(dc * dtf);
            }
            x.th[a][k] = (R)(-cb * dT);
        }
    }
    const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
    for (int q = 0; q < 3; ++q) {
        x.tab[q] = (R)p.tau_ab[pa[q]][pb[q]];
        if (pb[q] < I.N && p.tau_ab[pa[q]][pb[q]] > 0.0) x.tpair = 1;
    }
    x.ktau = (R)(p.dt / p.eps);
    x.proj = p.potential == MP_OBSTACLE_ACTIVE ? 1 : 0;
    // Eq. Well1 beyond its pair terms: 2 Theta_a phi_a (1 - phi_a)(1 - 2 phi_a) and
    // 2 Theta_abd phi_a phi_b^2 phi_d^2 in dg/dphi_a
    x.well1 = p.potential == MP_THETA ? 1 : 0;
    for (int a = 0; a < I.N; ++a) x.th1[a] = (R)(p.potential == MP_THETA ? 2.0 * p.theta[a] : 0.0);
    x.th3 = (R)(p.potential == MP_THETA ? 2.0 * p.theta3 : 0.0);
    return x;
}

template <typename R>
mp::AtCoef<R> make_at_coef(const Inst& I) {
    const mp_params& p = I.prm;
    mp::AtCoef<R> c;
    std::memset(&c, 0, sizeof c);
    c.prefw = (R)(p.eps / (2.0 * std::sqrt(2.0)));
    c.prefo = (R)(M_PI * p.eps / 4.0);
    c.obstacle = p.potential != MP_WELL ? 1 : 0;
    c.rdx = (R)(1.0 / I.grid.dx);
    c.rdt = (R)(1.0 / p.dt);
    c.dt = (R)p.dt;
    for (int a = 0; a < I.N; ++a) {
        double chi[2][2];
        chi_of(p, a, I.K, chi);  // 1 / (2 A) without the off-diagonal curvature
        for (int k = 0; k < I.K - 1; ++k) {
            c.chi[a][k] = (R)chi[k][k];
            c.B[a][k] = (R)p.B[a][k];
        }
    }
    return c;
}

mp::Geom make_geom(const mp_grid& gr) {
    mp::Geom g;
    g.nx = (int32_t)gr.n[0];
    g.ny = (int32_t)gr.n[1];
    g.nz = (int32_t)gr.n[2];
    g.bcx = gr.bc[0];
    g.bcy = gr.bc[1];
    g.bcz = gr.bc[2];
    g.fstride = ncells_of(gr);
    return g;
}

// T - Te at row j and step n: T0 + G ((j + yshift) dx - y0 - V n dt) - Te
// = tb0 + tdn n + tslope j
void temperature_law(const Inst& I, double& tb0, double& tdn, double& tslope) {
    const mp_params& p = I.prm;
    tb0 = p.T0 - p.Te - p.G * p.y0 + p.G * I.grid.dx * (double)I.yshift;
    tdn = temperature_step(I);
    tslope = p.G * I.grid.dx;
}

int hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) return fail(MP_E_HIP, "%s: %s", what, hipGetErrorString(e));
    return MP_OK;
}

// Strip waves across one row of a batched instance (W2X_LANES_OUT written lanes
// of vec_of cells each, for one and two steps per launch alike).
// Cap on cells per lane: the tile's, at most 2 in a batch (the batched kernel
// is built for 1 or 2).
int vec_cap(const mp_state* st) {
    if (!st->batch) return st->vec;
    return st->vec == 1 ? 1 : 2;
}
int vec_of(const mp_state* st, const Inst& I) {
    return mp::vec2d_width(I.grid.n[0], (int)elem_of(I.prm.precision), vec_cap(st));
}
int strips_of(const mp_state* st, const Inst& I) {
    const int64_t w = mp::W2X_LANES_OUT_HOST * vec_of(st, I);
    return (int)((I.grid.n[0] + w - 1) / w);
}

// ---- workspace layout -------------------------------------------------------
// [diag partials + one result record per instance][time level][instance table][work list]
// [anti-trapping coefficient table][extended-model coefficient table]
// [partial diagnostics records of a fused step launch (single grids)]
size_t ws_diag_bytes(const mp_state* st) {
    return align_up((size_t)(mp::DIAG_BLOCKS_MAX + st->inst.size()) * mp::DIAG_VALS * sizeof(double));
}
size_t ws_ctr_off(const mp_state* st) { return ws_diag_bytes(st); }
size_t ws_table_off(const mp_state* st) { return ws_ctr_off(st) + kAlign; }
size_t table_bytes(const mp_state* st) {
    const size_t one =
        st->precision == MP_FP64 ? sizeof(mp::InstDesc<double>) : sizeof(mp::InstDesc<float>);
    return st->batch ? align_up(one * st->inst.size()) : 0;
}
size_t ws_items_off(const mp_state* st) { return ws_table_off(st) + table_bytes(st); }
size_t items_capacity(const mp_state* st) {
    if (!st->batch) return 0;
    size_t n = 0;  // the work list is longest at seg = 1: one item per strip and row
    for (const Inst& I : st->inst) n += (size_t)strips_of(st, I) * (size_t)I.grid.n[1];
    return n;
}

size_t ws_attab_off(const mp_state* st) { return ws_items_off(st) + align_up(2 * sizeof(int) * items_capacity(st)); }
size_t attab_bytes(const mp_state* st) {
    const size_t one = st->precision == MP_FP64 ? sizeof(mp::AtCoef<double>) : sizeof(mp::AtCoef<float>);
    return st->batch ? align_up(one * st->inst.size()) : 0;
}
size_t ws_xtab_off(const mp_state* st) { return ws_attab_off(st) + attab_bytes(st); }
size_t xtab_bytes(const mp_state* st) {
    const size_t one = st->precision == MP_FP64 ? sizeof(mp::CoefX<double>) : sizeof(mp::CoefX<float>);
    return st->batch ? align_up(one * st->inst.size()) : 0;
}
size_t ws_frec_off(const mp_state* st) { return ws_xtab_off(st) + xtab_bytes(st); }
// Records a fused step launch writes: one per 2D strip wave or 3D tile, most
// at seg = 1; capped at FUSED_REC_MAX (a launch over the cap reduces in a
// separate pass instead).
int64_t frec_cap(const mp_state* st) {
    if (st->batch) return 0;
    const mp_grid& g = st->inst[0].grid;
    int64_t n;
    if (g.dim == 3)
        n = ((g.n[0] + 63) / 64) * ((g.n[1] + 3) / 4) * g.n[2];
    else
        n = ((g.n[0] + mp::W2X_LANES_OUT_HOST - 1) / mp::W2X_LANES_OUT_HOST) * g.n[1];
    return n < mp::FUSED_REC_MAX ? n : mp::FUSED_REC_MAX;
}
size_t frec_bytes(const mp_state* st) { return align_up((size_t)frec_cap(st) * mp::DIAG_VALS * sizeof(double)); }
double* dev_frec(mp_state* st) { return (double*)((char*)st->ws + ws_frec_off(st)); }

// A batch with an instance of the extended model steps every instance with the general kernels.
bool batch_gen(const mp_state* st) {
    for (const Inst& I : st->inst)
        if (I.ext) return true;
    return false;
}

int64_t* dev_ctr(mp_state* st) { return (int64_t*)((char*)st->ws + ws_ctr_off(st)); }

void drop_graphs(mp_state* st) {
    for (int p = 0; p < 2; ++p) {
        if (st->gexec[p]) {
            (void)hipGraphExecDestroy(st->gexec[p]);
            st->gexec[p] = nullptr;
        }
        st->gcalls[p].clear();
    }
}

// Work list of a batch: one item per (instance, column strip, row segment),
// as (instance, local index) pairs, in instance order until arrange_items
// deals it out.
void build_items(mp_state* st) {
    st->items.clear();
    for (size_t i = 0; i < st->inst.size(); ++i) {
        const Inst& I = st->inst[i];
        const int nseg = (int)((I.grid.n[1] + st->seg - 1) / st->seg);
        const int n = strips_of(st, I) * nseg;
        for (int l = 0; l < n; ++l) st->items.insert(st->items.end(), {(int)i, l});
    }
    st->nitems = (int)(st->items.size() / 2);
    for (int x = 0; x <= 8; ++x) st->cuts.c[x] = (int)((long long)st->nitems * x / 8);
}

// Estimated cost of one item: its rows (plus the two-step halo rows) times
// the strip's width in cells per lane times the work of a cell for (N, K).
double item_cost(const mp_state* st, const Inst& I, int local) {
    const int ntx = strips_of(st, I);
    const int m0 = (local / ntx) * st->seg;
    const int rows = (int)std::min<int64_t>(st->seg, I.grid.n[1] - m0);
    const int N = I.N, nm = I.K - 1, pairs = N * (N - 1) / 2;
    return (rows + 2.0) * vec_of(st, I) * (30.0 + 40.0 * N + 20.0 * nm + 14.0 * pairs + 6.0 * nm);
}

// Deal the work list to the persistent kernel, whose waves of XCD x take the
// items cuts[x] .. cuts[x+1]-1 with stride wpx (its waves per XCD): whole
// instances go to the XCD slices largest first, each to the slice with the
// least work so far (an instance's strips then share one XCD's L2); inside a
// slice the items are sorted by cost, largest first, and laid out in rounds
// of wpx, every other round reversed, so that the waves' shares come out even.
// Deterministic; the results do not depend on the order.
void arrange_items(mp_state* st, int wpx) {
    const int ninst = (int)st->inst.size();
    std::vector<std::vector<int>> by_inst(ninst);
    std::vector<double> icost(ninst, 0.0);
    for (int it = 0; it < st->nitems; ++it) {
        const int i = st->items[2 * it], l = st->items[2 * it + 1];
        by_inst[i].push_back(l);
        icost[i] += item_cost(st, st->inst[i], l);
    }
    std::vector<int> order(ninst);
    for (int i = 0; i < ninst; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return icost[a] > icost[b]; });
    std::vector<int> slice_of(ninst);
    double load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int i : order) {
        int x = 0;
        for (int y = 1; y < 8; ++y)
            if (load[y] < load[x]) x = y;
        slice_of[i] = x;
        load[x] += icost[i];
    }
    std::vector<int> out;
    out.reserve(st->items.size());
    for (int x = 0; x < 8; ++x) {
        st->cuts.c[x] = (int)(out.size() / 2);
        std::vector<std::pair<double, std::pair<int, int>>> v;
        for (int i = 0; i < ninst; ++i)
            if (slice_of[i] == x)
                for (int l : by_inst[i]) v.push_back({item_cost(st, st->inst[i], l), {i, l}});
        std::stable_sort(v.begin(), v.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
        const int w = wpx < 1 ? 1 : wpx;
        for (size_t r0 = 0; r0 < v.size(); r0 += w) {
            const size_t r1 = std::min(v.size(), r0 + (size_t)w);
            if ((r0 / w) % 2 == 1) std::reverse(v.begin() + r0, v.begin() + r1);
            for (size_t k = r0; k < r1; ++k) out.insert(out.end(), {v[k].second.first, v[k].second.second});
        }
    }
    st->cuts.c[8] = (int)(out.size() / 2);
    st->items.swap(out);
}

template <typename R>
int upload_table(mp_state* st) {
    std::vector<mp::InstDesc<R>> tab(st->inst.size());
    for (size_t i = 0; i < st->inst.size(); ++i) {
        const Inst& I = st->inst[i];
        mp::InstDesc<R>& d = tab[i];
        std::memset(&d, 0, sizeof d);
        d.g = make_geom(I.grid);
        d.np = I.N;
        d.nm = I.K - 1;
        d.ntx = strips_of(st, I);
        d.vec = vec_of(st, I);
        d.seg = st->seg;
        d.nseg = (int)((I.grid.n[1] + st->seg - 1) / st->seg);
        d.off = (int64_t)(I.off_bytes / sizeof(R));
        temperature_law(I, d.tb0, d.tdn, d.tslope);
        d.c = make_coef<R>(I);
    }
    std::vector<mp::AtCoef<R>> atab(st->inst.size());
    for (size_t i = 0; i < st->inst.size(); ++i) atab[i] = make_at_coef<R>(st->inst[i]);
    std::vector<mp::CoefX<R>> xtab(st->inst.size());
    for (size_t i = 0; i < st->inst.size(); ++i) xtab[i] = make_coefx<R>(st->inst[i]);
    char* ws = (char*)st->ws;
    int rc = hip_check(hipMemcpy(ws + ws_table_off(st), tab.data(),
                                 sizeof(mp::InstDesc<R>) * tab.size(), hipMemcpyHostToDevice),
                       "instance table upload");
    if (rc == MP_OK)
        rc = hip_check(hipMemcpy(ws + ws_attab_off(st), atab.data(), sizeof(mp::AtCoef<R>) * atab.size(),
                                 hipMemcpyHostToDevice),
                       "anti-trapping table upload");
    if (rc == MP_OK)
        rc = hip_check(hipMemcpy(ws + ws_xtab_off(st), xtab.data(), sizeof(mp::CoefX<R>) * xtab.size(),
                                 hipMemcpyHostToDevice),
                       "extended-model table upload");
    return rc;
}

int upload_items(mp_state* st) {
    return hip_check(hipMemcpy((char*)st->ws + ws_items_off(st), st->items.data(), sizeof(int) * st->items.size(),
                               hipMemcpyHostToDevice),
                     "work list upload");
}

// The anti-trapping current folded into the step kernel (2D single grids and
// batches): mp_step then runs the ordinary launch path, one step per launch.
bool at_folded(const mp_state* st) { return st->antitrap == 1 && (st->batch || st->inst[0].grid.dim == 2); }

// Steps per launch of the ordinary path.
int launch_fuse(const mp_state* st) { return st->antitrap ? 1 : st->fuse; }

// mp_step_diag forms the diagnostics inside the last step launch for single
// grids without the anti-trapping current, in FP64 2D and in 3D.  The FP32 2D
// strips take the separate pass: their lane shuffles go through the LDS
// pipe, where the accumulators' atomics delay them, and the fused launch
// measured slower than the step plus the separate pass.
bool fused_diag(const mp_state* st) {
    return !st->batch && !st->antitrap && (st->inst[0].grid.dim == 3 || st->precision == MP_FP64);
}

// The batched kernel for L: with the current folded in while it is on.
int batch_call(mp_state* st, const mp::BatchLaunch& L, mp::KernelCall& k) {
    const void* atab = (const char*)st->ws + ws_attab_off(st);
    const void* xtab = (const char*)st->ws + ws_xtab_off(st);
    const bool f64 = st->precision == MP_FP64;
    if (batch_gen(st)) {
        if (st->antitrap)
            return f64 ? mp::call_batch_at_gen<double>(L, atab, xtab, k) : mp::call_batch_at_gen<float>(L, atab, xtab, k);
        return f64 ? mp::call_batch_gen<double>(L, xtab, k) : mp::call_batch_gen<float>(L, xtab, k);
    }
    if (st->antitrap) return f64 ? mp::call_batch_at<double>(L, atab, k) : mp::call_batch_at<float>(L, atab, k);
    return f64 ? mp::call_batch<double>(L, k) : mp::call_batch<float>(L, k);
}

int choose_batch_blocks(mp_state* st) {
    int dev = 0, cus = 0, per = 0;
    int rc = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (rc) return rc;
    rc = hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "CU count");
    if (rc) return rc;
    mp::BatchLaunch L;
    std::memset(&L, 0, sizeof L);
    L.potential = st->potential;
    L.aniso = st->aniso ? 1 : 0;
    L.vmax = vec_cap(st);
    L.fuse = launch_fuse(st);
    L.nblocks = 8;
    mp::KernelCall k;
    rc = batch_call(st, L, k);
    if (rc) return fail(rc, "no batched kernel instance");
    rc = hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k.func, (int)k.block.x, 0),
                   "occupancy query");
    if (rc) return rc;
    if (per < 1) per = 1;
    long long nb = (long long)cus * per;
    const long long need = (st->nitems + mp::BATCH_WPB_HOST - 1) / mp::BATCH_WPB_HOST;
    if (nb > need) nb = need;
    nb = (nb + 7) / 8 * 8;
    if (nb < 8) nb = 8;
    st->batch_blocks = (int)nb;
    build_items(st);
    arrange_items(st, (int)(nb / 8) * mp::BATCH_WPB_HOST);
    return upload_items(st);
}

int sync_batch(mp_state* st) {
    build_items(st);
    if (!st->bound) return MP_OK;
    const int rc = st->precision == MP_FP64 ? upload_table<double>(st) : upload_table<float>(st);
    if (rc) return rc;
    return choose_batch_blocks(st);
}

int make_single_call(mp_state* st, const void* in, void* out, const int64_t* ctr, int kstep,
                     mp::KernelCall& k, int fuse = 1, void* out1 = nullptr, const mp::DiagOut* diag = nullptr);


// One launch of `fuse` steps (1 or 2; a batch always 1); kstep is the
// launch's offset from the device time level.
int make_step_call(mp_state* st, int kstep, int from, mp::KernelCall& k, int fuse = 1) {
    if (st->batch) {
        mp::BatchLaunch L;
        L.in = st->buf[from];
        L.out = st->buf[1 - from];
        L.table = (const char*)st->ws + ws_table_off(st);
        L.items = (const int*)((const char*)st->ws + ws_items_off(st));
        L.cuts = st->cuts;
        L.potential = st->potential;
        L.aniso = st->aniso ? 1 : 0;
        L.vmax = vec_cap(st);
        L.fuse = fuse;
        L.nblocks = st->batch_blocks;
        L.stepctr = dev_ctr(st);
        L.kstep = kstep;
        return batch_call(st, L, k);
    }
    return make_single_call(st, st->buf[from], st->buf[1 - from], dev_ctr(st), kstep, k, fuse);
}

// Single-grid launch of `fuse` steps from ``in`` to ``out`` at time level
// *ctr + kstep.
int make_single_call(mp_state* st, const void* in, void* out, const int64_t* ctr, int kstep,
                     mp::KernelCall& k, int fuse, void* out1, const mp::DiagOut* diag) {
    const Inst& I = st->inst[0];
    mp::StepLaunch L;
    L.in = in;
    L.out = out;
    L.g = make_geom(I.grid);
    L.nphases = I.N;
    L.nmu = I.K - 1;
    L.dim = I.grid.dim;
    L.potential = kernel_potential(I.prm.potential);
    L.aniso = I.aniso ? 1 : 0;
    L.bx = st->bx;
    L.seg = st->seg;
    L.vec = st->vec;
    L.fuse = fuse;
    L.out1 = out1;
    L.stepctr = ctr;
    L.kstep = kstep;
    L.diag = diag;
    temperature_law(I, L.tb0, L.tdn, L.tslope);
    if (diag) {
        // the instances that also write the diagnostics' partial records
        // (fused_diag: FP64 2D strips and 3D tiles)
        if (at_folded(st) || out1 || !fused_diag(st)) return MP_E_PARAM;
        const bool d3 = I.grid.dim == 3;
        if (st->precision == MP_FP64) {
            if (I.ext)
                return d3 ? mp::call_step_gen<double, true, true>(L, make_coef<double>(I), make_coefx<double>(I), k)
                          : mp::call_step_gen<double, false, true>(L, make_coef<double>(I), make_coefx<double>(I), k);
            return d3 ? mp::call_step_dim<double, true, true>(L, make_coef<double>(I), k)
                      : mp::call_step_dim<double, false, true>(L, make_coef<double>(I), k);
        }
        if (I.ext) return mp::call_step_gen<float, true, true>(L, make_coef<float>(I), make_coefx<float>(I), k);
        return mp::call_step_dim<float, true, true>(L, make_coef<float>(I), k);
    }
    if (at_folded(st) && !out1) {
        if (I.ext) {
            if (st->precision == MP_FP64)
                return mp::call_step_at_gen<double>(L, make_coef<double>(I), make_at_coef<double>(I),
                                                    make_coefx<double>(I), k);
            return mp::call_step_at_gen<float>(L, make_coef<float>(I), make_at_coef<float>(I), make_coefx<float>(I),
                                               k);
        }
        if (st->precision == MP_FP64) return mp::call_step_at<double>(L, make_coef<double>(I), make_at_coef<double>(I), k);
        return mp::call_step_at<float>(L, make_coef<float>(I), make_at_coef<float>(I), k);
    }
    if (I.ext) {
        if (st->precision == MP_FP64)
            return I.grid.dim == 3 ? mp::call_step_gen<double, true>(L, make_coef<double>(I), make_coefx<double>(I), k)
                                   : mp::call_step_gen<double, false>(L, make_coef<double>(I), make_coefx<double>(I), k);
        return I.grid.dim == 3 ? mp::call_step_gen<float, true>(L, make_coef<float>(I), make_coefx<float>(I), k)
                               : mp::call_step_gen<float, false>(L, make_coef<float>(I), make_coefx<float>(I), k);
    }
    if (st->precision == MP_FP64) return mp::call_step_f64(L, make_coef<double>(I), k);
    return mp::call_step_f32(L, make_coef<float>(I), k);
}

int launch(const mp::KernelCall& k, hipStream_t s) {
    if (k.bad) return fail(MP_E_PARAM, "kernel arguments exceed the launch record");
    return hip_check(hipLaunchKernel(k.func, k.grid, k.block, (void**)k.args, 0, s), "kernel launch");
}

// Graph of graph_chunk steps starting from buffer `from` (launches of st->fuse
// steps each), then the time-level advance.  Sets gend[from].
int build_graph(mp_state* st, int from, hipGraphExec_t* out) {
    std::vector<mp::KernelCall>& calls = st->gcalls[from];
    const int F = launch_fuse(st);
    const int nl = st->graph_chunk / F;  // graph_chunk is even, F is 1 or 2
    calls.assign((size_t)nl + 1, mp::KernelCall());
    for (int i = 0; i <= nl; ++i) {
        if (i < nl) {
            const int rc = make_step_call(st, i * F, (from + i) & 1, calls[i], F);
            if (rc) return fail(rc, "no kernel instance for this configuration");
        } else {
            mp::call_advance(dev_ctr(st), st->graph_chunk, calls[i]);
        }
    }
    st->gend[from] = (from + nl) & 1;
    hipGraph_t g = nullptr;
    int rc = hip_check(hipGraphCreate(&g, 0), "hipGraphCreate");
    if (rc) return rc;
    hipGraphNode_t prev = nullptr;
    for (size_t i = 0; i < calls.size() && rc == MP_OK; ++i) {
        const mp::KernelCall& k = calls[i];
        hipKernelNodeParams np;
        std::memset(&np, 0, sizeof np);
        np.func = (void*)k.func;
        np.gridDim = k.grid;
        np.blockDim = k.block;
        np.sharedMemBytes = 0;
        np.kernelParams = (void**)k.args;
        np.extra = nullptr;
        hipGraphNode_t node = nullptr;
        rc = hip_check(hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &np),
                       "hipGraphAddKernelNode");
        prev = node;
    }
    if (rc == MP_OK)
        rc = hip_check(hipGraphInstantiate(out, g, nullptr, nullptr, 0), "hipGraphInstantiate");
    (void)hipGraphDestroy(g);
    return rc;
}

// 3D tiles of 64 x 8 exist where their LDS ring fits in 64 KiB.
bool d3_tall_ok(const mp_state* st) {
    const Inst& I = st->inst[0];
    const int elem = (int)elem_of(st->precision);
    return 4 * (I.N + 2 * (I.K - 1)) * 66 * 10 * elem <= 64 * 1024;
}

void init_state(mp_state* st) {
    st->buf[0] = st->buf[1] = nullptr;
    st->ws = nullptr;
    st->bound = false;
    st->cur = 0;
    st->step = 0;
    st->graph_chunk = 0;
    st->fuse = 1;
    st->antitrap = 0;
    st->gexec[0] = st->gexec[1] = nullptr;
    st->gend[0] = 0;
    st->gend[1] = 1;
    st->nitems = 0;
    st->batch_blocks = 0;
    st->aux = nullptr;
    for (hipEvent_t& e : st->ev) e = nullptr;
    st->aniso = false;
    for (const Inst& I : st->inst) st->aniso = st->aniso || I.aniso;
    st->precision = st->inst[0].prm.precision;
    st->vec = -1;
    st->potential = kernel_potential(st->inst[0].prm.potential);
    if (st->inst[0].grid.dim == 3) {
        // measured best on 512^3 FP32: tall tiles, long z segments
        st->bx = d3_tall_ok(st) ? 512 : 256;
        st->seg = 64;
    } else if (st->batch) {
        // measured best on the 256-instance ensemble: two steps per launch,
        // one cell per lane (keeps the batched kernel at 5 waves per SIMD)
        st->fuse = 2;
        st->bx = 64 * mp::BATCH_WPB_HOST;
        st->seg = 32;
        st->vec = 1;
    } else {
        // two steps per launch (the state crosses HBM once per two steps);
        // tiles measured best for it on 4096^2: one cell per lane (FP64 at 3
        // waves per SIMD without spills, FP32 at 5), 31- / 14-row segments
        // (their wave counts come out just under a whole number of the
        // chip's resident wave slots, so the last wave round is nearly full)
        st->fuse = 2;
        st->bx = 256;
        st->seg = st->precision == MP_FP64 ? 31 : 14;
        st->vec = 1;
    }
}

// Diagnostics of instance i of the state held in ``base`` (one state buffer),
// with per-block partials in ``partials`` and the result record in ``result``.
mp::DiagCoef make_diag_coef(const mp_state* st, int i, int64_t step) {
    const Inst& I = st->inst[i];
    mp::DiagCoef dc;
    std::memset(&dc, 0, sizeof dc);
    const int K1 = I.K - 1;
    for (int a = 0; a < I.N; ++a) {
        double chi[2][2];
        chi_of(I.prm, a, I.K, chi);
        dc.chx[a] = K1 == 2 ? chi[0][1] : 0.0;
        for (int k = 0; k < K1; ++k) {
            dc.chi[a][k] = chi[k][k];
            dc.cb[a][k] = chi[k][k] * I.prm.B[a][k];
            dc.cbt[a][k] = chi[k][k] * I.prm.Bt[a][k];
            if (K1 == 2) {
                dc.cb[a][k] += chi[k][1 - k] * I.prm.B[a][1 - k];
                dc.cbt[a][k] += chi[k][1 - k] * I.prm.Bt[a][1 - k];
            }
        }
    }
    double tb0, tdn, tslope;
    temperature_law(I, tb0, tdn, tslope);
    dc.tt0 = tb0 + tdn * (double)step;
    dc.tslope = tslope;
    dc.nx = (int32_t)I.grid.n[0];
    dc.ny = (int32_t)I.grid.n[1];
    return dc;
}

int diag_instance_at(const mp_state* st, int i, const void* base, int64_t step, double* partials, double* result,
                     hipStream_t s) {
    const Inst& I = st->inst[i];
    const mp::DiagCoef dc = make_diag_coef(st, i, step);
    const void* state = (const char*)base + I.off_bytes;
    int rc = mp::launch_diag(state, st->precision, make_geom(I.grid), I.N, I.K - 1, dc, partials, result, s);
    if (rc) return fail(rc, "no diagnostics instance");
    return hip_check(hipGetLastError(), "diagnostics launch");
}

int diag_instance(mp_state* st, int i, hipStream_t s) {
    double* ws = (double*)st->ws;
    return diag_instance_at(st, i, st->buf[st->cur], st->step, ws,
                            ws + (size_t)(mp::DIAG_BLOCKS_MAX + i) * mp::DIAG_VALS, s);
}

void unpack_diag(const mp_state* st, int i, const double* r, int64_t step, mp_diag* out) {
    const Inst& I = st->inst[i];
    std::memset(out, 0, sizeof *out);
    out->step = step;
    // the records hold sums of c_k and phi_a over cells; dx^d once here
    const double vol = std::pow(I.grid.dx, I.grid.dim);
    for (int k = 0; k < I.K - 1; ++k) {
        out->mass[k] = (r[mp::DV_MASS + 2 * k] + r[mp::DV_MASS + 2 * k + 1]) * vol;
        out->min_chi[k] = r[mp::DV_MINCHI + k];
    }
    for (int a = 0; a < I.N; ++a) out->volume[a] = (r[mp::DV_VOL + 2 * a] + r[mp::DV_VOL + 2 * a + 1]) * vol;
    out->max_sum_dev = r[mp::DV_MAXDEV];
    out->nonfinite = (int64_t)r[mp::DV_NONFIN];
}

// Copy the instances' result records to the host and unpack them.
int diag_collect(mp_state* st, mp_diag* out, hipStream_t s) {
    const int n = (int)st->inst.size();
    std::vector<double> r((size_t)n * mp::DIAG_VALS);
    int rc = hip_check(hipMemcpyAsync(r.data(),
                                      (double*)st->ws + (size_t)mp::DIAG_BLOCKS_MAX * mp::DIAG_VALS,
                                      sizeof(double) * r.size(), hipMemcpyDeviceToHost, s),
                       "diagnostics copy");
    if (rc) return rc;
    rc = hip_check(hipStreamSynchronize(s), "diagnostics sync");
    if (rc) return rc;
    int64_t bad = 0;
    for (int i = 0; i < n; ++i) {
        unpack_diag(st, i, &r[(size_t)i * mp::DIAG_VALS], st->step, &out[i]);
        bad += out[i].nonfinite;
    }
    if (bad > 0) return fail(MP_E_NONFINITE, "%lld cells hold NaN or Inf", (long long)bad);
    return ok();
}

int diag_many(mp_state* st, mp_diag* out, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    const int n = (int)st->inst.size();
    for (int i = 0; i < n; ++i) {
        const int rc = diag_instance(st, i, s);
        if (rc) return rc;
    }
    return diag_collect(st, out, s);
}

// ---- adjoint driver -----------------------------------------------------------
template <typename R>
mp::AdjCoef<R> make_adj_coef(const Inst& I) {
    const mp_params& p = I.prm;
    mp::AdjCoef<R> c;
    std::memset(&c, 0, sizeof c);
    const double dx2 = I.grid.dx * I.grid.dx;
    c.kphi = (R)(p.dt / (p.tau * p.eps));
    c.ktj = (R)(p.dt / (2.0 * dx2));
    const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
    for (int q = 0; q < 3; ++q) {
        const double g = p.gamma[pa[q]][pb[q]];
        c.c4e[q] = (R)(2.0 * p.eps * g / dx2);
        c.w18e[q] = (R)(18.0 * g / p.eps);
        c.scB[q] = 2.0 * p.eps / dx2;  // d(c4e K T)/d gamma
        c.scA[q] = -18.0 / p.eps;      // d(-dw)/d gamma per phi_i phi_j (lR_i phi_j + lR_j phi_i)
    }
    c.g3e = (R)(p.gamma3 / p.eps);
    c.scA[9] = -p.dt / (p.tau * p.tau * p.eps);  // d phi^{n+1}/d tau per (R - lambda)
    for (int a = 0; a < I.N; ++a) {
        c.C[a] = (R)p.C[a];
        c.s[a] = (R)p.s[a];
        for (int k = 0; k < I.K - 1; ++k) {
            const double chi = 1.0 / (2.0 * p.A[a][k]);
            c.chi[a][k] = (R)chi;
            c.B[a][k] = (R)p.B[a][k];
            c.Dchi[a][k] = (R)(p.D[a][k] * chi);
            c.scB[3 + 2 * a + k] = chi;  // dM_k/dD_ak per h_a
        }
    }
    return c;
}

struct AdjLayout {
    size_t X0, X1, lam, seg[2], acc, ctr, grad, total;
    size_t state;
    int nrows;
};

// The adjoint strips are planned for the wave slots of at most kAdjCUs
// compute units (gfx950 has 256); the accumulator rows are sized for that
// plan, which has at least as many blocks as the plan of a smaller device.
constexpr int kAdjCUs = 256;

mp::AdjGeom adj_geom(const Inst& I, int cus, bool fp64) {
    mp::AdjGeom g;
    g.nx = (int)I.grid.n[0];
    g.ny = (int)I.grid.n[1];
    g.perx = I.grid.bc[0] == MP_BC_PERIODIC;
    g.pery = I.grid.bc[1] == MP_BC_PERIODIC;
    g.fs = ncells_of(I.grid);
    const int c = cus < 1 ? 1 : (cus > kAdjCUs ? kAdjCUs : cus);
    mp::adj_plan(g, c * (fp64 ? mp::adj_wpb<double>() : mp::adj_wpb<float>()));
    return g;
}

int adj_nblocks(const mp::AdjGeom& g, bool fp64) {
    return fp64 ? mp::adj_blocks<mp::adj_wpb<double>()>(g) : mp::adj_blocks<mp::adj_wpb<float>()>(g);
}

AdjLayout adj_layout(const mp_state* st, int64_t every) {
    const Inst& I = st->inst[0];
    AdjLayout L;
    L.state = align_up(I.bytes);
    const bool fp64 = st->precision == MP_FP64;
    L.nrows = adj_nblocks(adj_geom(I, kAdjCUs, fp64), fp64);
    size_t o = 0;
    L.X0 = o;
    o += L.state;
    L.X1 = o;
    o += L.state;
    L.lam = o;
    o += L.state;
    L.seg[0] = o;
    o += L.state * (size_t)every;
    L.seg[1] = o;
    o += L.state * (size_t)every;
    L.acc = o;
    o += align_up(sizeof(double) * mp::ADJ_NPAR * (size_t)L.nrows);
    L.ctr = o;
    o += kAlign;
    L.grad = o;
    o += kAlign;
    L.total = o;
    return L;
}

int adj_supported(const mp_state* st) {
    if (st->batch) return fail(MP_E_STATE, "adjoint: batched states are not supported");
    if (st->antitrap) return fail(MP_E_STATE, "adjoint: the anti-trapping current is not supported");
    const Inst& I = st->inst[0];
    if (I.ext)
        return fail(MP_E_PARAM, "adjoint: the extended model (Bt, Ct, A01, D01, tau_ab, MP_OBSTACLE_ACTIVE) is not supported");
    if (I.grid.dim != 2) return fail(MP_E_PARAM, "adjoint: 2D grids only");
    if (I.prm.model != MP_GP) return fail(MP_E_PARAM, "adjoint: the KKS variant is not supported");
    if (I.prm.potential != MP_WELL) return fail(MP_E_PARAM, "adjoint: the obstacle projection is not differentiable");
    if (I.aniso) return fail(MP_E_PARAM, "adjoint: anisotropic gradient energy not supported");
    return MP_OK;
}

}  // namespace

namespace mp {
int call_step_f64(const StepLaunch& L, const Coef<double>& c, KernelCall& k) {
    return L.dim == 3 ? call_step_dim<double, true>(L, c, k) : call_step_dim<double, false>(L, c, k);
}
int call_step_f32(const StepLaunch& L, const Coef<float>& c, KernelCall& k) {
    return L.dim == 3 ? call_step_dim<float, true>(L, c, k) : call_step_dim<float, false>(L, c, k);
}
}  // namespace mp

namespace {

// Steps with the anti-trapping current: each step is a one-step launch of the
// step kernel followed by the correction of its mu^{n+1} from states n and n+1.
int step_antitrapping(mp_state* st, int64_t nsteps, hipStream_t s) {
    const Inst& I = st->inst[0];
    mp::AtLaunch A;
    A.g = make_geom(I.grid);
    A.nphases = I.N;
    A.nmu = I.K - 1;
    for (int64_t i = 0; i < nsteps; ++i) {
        mp::KernelCall k;
        int rc = make_step_call(st, (int)i, st->cur, k, 1);
        if (rc) return fail(rc, "no kernel instance for this configuration");
        rc = launch(k, s);
        if (rc) return rc;
        A.prev = st->buf[st->cur];
        A.next = st->buf[1 - st->cur];
        if (I.ext) {
            double tb0, tdn, tslope;
            temperature_law(I, tb0, tdn, tslope);
            rc = st->precision == MP_FP64
                     ? mp::at_launch_gen<double>(A, make_at_coef<double>(I), make_coefx<double>(I), dev_ctr(st), (int)i,
                                                 tb0, tdn, tslope, s)
                     : mp::at_launch_gen<float>(A, make_at_coef<float>(I), make_coefx<float>(I), dev_ctr(st), (int)i,
                                                tb0, tdn, tslope, s);
        } else {
            rc = st->precision == MP_FP64 ? mp::at_launch<double>(A, make_at_coef<double>(I), s)
                                          : mp::at_launch<float>(A, make_at_coef<float>(I), s);
        }
        if (rc) return fail(rc, "anti-trapping kernel launch failed");
        st->cur = 1 - st->cur;
    }
    if (nsteps > 0) {
        mp::KernelCall k;
        mp::call_advance(dev_ctr(st), nsteps, k);
        const int rc = launch(k, s);
        if (rc) return rc;
        st->step += nsteps;
    }
    return ok();
}

}  // namespace

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
    const int rc = validate(grid, nphases, ncomp, params, "");
    if (rc) return rc;
    mp_state* st = new (std::nothrow) mp_state();
    if (!st) return fail(MP_E_PARAM, "out of host memory");
    st->batch = false;
    st->inst.push_back(make_inst(grid, nphases, ncomp, params));
    init_state(st);
    // MP_TILE="bx,seg,vec": the tile shape of new single-grid states, as by mp_set_tile
    if (const char* t = std::getenv("MP_TILE")) {
        int bx = 0, seg = 0, vec = 0;
        if (std::sscanf(t, "%d,%d,%d", &bx, &seg, &vec) != 3 || mp_set_tile(st, bx, seg, vec) != MP_OK) {
            const std::string why = g_err;
            delete st;
            return fail(MP_E_PARAM, "MP_TILE=\"%s\" is not a valid bx,seg,vec for this state%s%s", t,
                        why.empty() ? "" : ": ", why.c_str());
        }
    }
    *out = st;
    return ok();
}

int mp_create_batch(int ninst, const mp_grid* grids, const int* nphases, const int* ncomp,
                    const mp_params* params, mp_state** out) {
    if (!out) return fail(MP_E_NULLPTR, "out is NULL");
    *out = nullptr;
    if (ninst < 1) return fail(MP_E_PARAM, "ninst must be >= 1");
    if (!grids || !nphases || !ncomp || !params) return fail(MP_E_NULLPTR, "batch array is NULL");
    mp_state* st = new (std::nothrow) mp_state();
    if (!st) return fail(MP_E_PARAM, "out of host memory");
    st->batch = true;
    size_t off = 0;
    for (int i = 0; i < ninst; ++i) {
        char who[64];
        snprintf(who, sizeof who, "instance %d: ", i);
        int rc = validate(&grids[i], nphases[i], ncomp[i], &params[i], who);
        if (rc == MP_OK && grids[i].dim != 2) rc = fail(MP_E_PARAM, "%sbatched grids must be 2D", who);
        if (rc == MP_OK && i > 0 && params[i].precision != params[0].precision)
            rc = fail(MP_E_PARAM, "%sall instances must share one precision", who);
        if (rc == MP_OK && i > 0 && kernel_potential(params[i].potential) != kernel_potential(params[0].potential))
            rc = fail(MP_E_PARAM, "%sall instances must share one potential", who);
        if (rc) {
            delete st;
            return rc;
        }
        Inst I = make_inst(&grids[i], nphases[i], ncomp[i], &params[i]);
        I.off_bytes = off;
        off = align_up(off + I.bytes);
        st->inst.push_back(I);
    }
    init_state(st);
    build_items(st);
    *out = st;
    return ok();
}

size_t mp_state_bytes(const mp_state* st) {
    if (!st) return 0;
    if (!st->batch) return st->inst[0].bytes;
    const Inst& L = st->inst.back();
    return align_up(L.off_bytes + L.bytes);
}

size_t mp_workspace_bytes(const mp_state* st) {
    if (!st) return 0;
    return ws_frec_off(st) + frec_bytes(st);
}

int mp_bind(mp_state* st, void* buf0, void* buf1, void* workspace) {
    if (!st) return fail(MP_E_NULLPTR, "state is NULL");
    if (!buf0 || !buf1 || !workspace) return fail(MP_E_NULLPTR, "buffer pointer is NULL");
    if (buf0 == buf1) return fail(MP_E_PARAM, "buf0 and buf1 must differ");
    if (((uintptr_t)buf0 | (uintptr_t)buf1 | (uintptr_t)workspace) & (kAlign - 1))
        return fail(MP_E_PARAM, "buffers must be 256-byte aligned");
    drop_graphs(st);
    st->buf[0] = buf0;
    st->buf[1] = buf1;
    st->ws = workspace;
    st->bound = true;
    st->cur = 0;
    st->step = 0;
    int64_t zero = 0;
    int rc = hip_check(hipMemcpy(dev_ctr(st), &zero, sizeof zero, hipMemcpyHostToDevice),
                       "time level upload");
    if (rc == MP_OK && st->batch) rc = sync_batch(st);
    if (rc) {
        st->bound = false;
        return rc;
    }
    return ok();
}

int mp_step(mp_state* st, int64_t nsteps, void* stream) {
    if (!st) return fail(MP_E_NULLPTR, "state is NULL");
    if (!st->bound) return fail(MP_E_UNBOUND, "mp_step before mp_bind");
    if (nsteps < 0) return fail(MP_E_PARAM, "nsteps must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    if (st->antitrap && !at_folded(st)) return step_antitrapping(st, nsteps, s);
    int64_t left = nsteps;
    const int C = st->graph_chunk;
    if (C > 0) {
        while (left >= C) {
            if (!st->gexec[st->cur]) {
                const int rc = build_graph(st, st->cur, &st->gexec[st->cur]);
                if (rc) return rc;
            }
            const int rc = hip_check(hipGraphLaunch(st->gexec[st->cur], s), "hipGraphLaunch");
            if (rc) return rc;
            left -= C;
            st->step += C;
            st->cur = st->gend[st->cur];
        }
    }
    // launches of st->fuse steps, then single steps for the remainder
    for (int64_t i = 0; i < left;) {
        const int F = left - i >= launch_fuse(st) ? launch_fuse(st) : 1;
        mp::KernelCall k;
        int rc = make_step_call(st, (int)i, st->cur, k, F);
        if (rc) return fail(rc, "no kernel instance for this configuration");
        rc = launch(k, s);
        if (rc) return rc;
        st->cur = 1 - st->cur;
        i += F;
    }
    if (left > 0) {
        mp::KernelCall k;
        mp::call_advance(dev_ctr(st), left, k);
        const int rc = launch(k, s);
        if (rc) return rc;
        st->step += left;
    }
    return ok();
}

int mp_step_diag(mp_state* st, int64_t nsteps, mp_diag* out, void* stream) {
    if (!st || !out) return fail(MP_E_NULLPTR, "state or out is NULL");
    if (!st->bound) return fail(MP_E_UNBOUND, "mp_step_diag before mp_bind");
    if (nsteps < 1) return fail(MP_E_PARAM, "nsteps must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    // the other paths: the steps, then the separate pass
    if (!fused_diag(st)) {
        const int rc = mp_step(st, nsteps, stream);
        if (rc) return rc;
        return diag_many(st, out, stream);
    }
    const int F = launch_fuse(st) == 2 && nsteps >= 2 ? 2 : 1;
    int rc = mp_step(st, nsteps - F, stream);
    if (rc) return rc;
    // the last launch also writes the partial records of the state it stores
    mp::DiagOut d;
    d.part = dev_frec(st);
    d.dc = make_diag_coef(st, 0, st->step + F);
    mp::KernelCall k;
    rc = make_single_call(st, st->buf[st->cur], st->buf[1 - st->cur], dev_ctr(st), 0, k, F, nullptr, &d);
    if (rc) return fail(rc, "no kernel instance for this configuration");
    if (k.nrec < 1 || k.nrec > frec_cap(st)) {
        // more records than the workspace holds (very short segments)
        rc = mp_step(st, F, stream);
        if (rc) return rc;
        return diag_many(st, out, stream);
    }
    rc = launch(k, s);
    if (rc) return rc;
    st->cur = 1 - st->cur;
    mp::KernelCall adv;
    mp::call_advance(dev_ctr(st), F, adv);
    rc = launch(adv, s);
    if (rc) return rc;
    st->step += F;
    rc = mp::launch_diag_final(dev_frec(st), k.nrec, (double*)st->ws + (size_t)mp::DIAG_BLOCKS_MAX * mp::DIAG_VALS,
                               s);
    if (rc) return fail(rc, "diagnostics reduction");
    rc = hip_check(hipGetLastError(), "diagnostics launch");
    if (rc) return rc;
    return diag_collect(st, out, s);
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
    if (st->bound) {
        const int rc = hip_check(hipMemcpy(dev_ctr(st), &step, sizeof step, hipMemcpyHostToDevice),
                                 "time level upload");
        if (rc) return rc;
    }
    st->step = step;
    st->cur = which_buf;
    return ok();
}

int mp_diagnostics(mp_state* st, mp_diag* out, void* stream) {
    if (!st || !out) return fail(MP_E_NULLPTR, "state or out is NULL");
    if (st->batch) return fail(MP_E_STATE, "batched state: use mp_diagnostics_batch");
    if (!st->bound) return fail(MP_E_UNBOUND, "mp_diagnostics before mp_bind");
    return diag_many(st, out, stream);
}

int mp_diagnostics_batch(mp_state* st, mp_diag* out, void* stream) {
    if (!st || !out) return fail(MP_E_NULLPTR, "state or out is NULL");
    if (!st->bound) return fail(MP_E_UNBOUND, "mp_diagnostics_batch before mp_bind");
    return diag_many(st, out, stream);
}

int mp_diagnostics_static(const mp_state* st, const void* state_buf, int64_t step, mp_diag* out,
                          void* stream) {
    if (!st || !state_buf || !out) return fail(MP_E_NULLPTR, "state, state_buf or out is NULL");
    const int n = (int)st->inst.size();
    if (n > mp::DIAG_STATIC_INST)
        return fail(MP_E_PARAM, "mp_diagnostics_static reduces at most %d instances (got %d)",
                    mp::DIAG_STATIC_INST, n);
    if (step < 0) return fail(MP_E_PARAM, "step must be >= 0");
    double* scr = nullptr;
    int rc = hip_check(mp::diag_static_scratch(&scr), "static diagnostics scratch");
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    for (int i = 0; i < n; ++i) {
        if (mp::diag_blocks(ncells_of(st->inst[i].grid)) > mp::DIAG_BLOCKS_MAX)
            return fail(MP_E_PARAM, "instance %d needs more partial records than the scratch holds", i);
        rc = diag_instance_at(st, i, state_buf, step, scr, scr + (size_t)(mp::DIAG_BLOCKS_MAX + i) * mp::DIAG_VALS,
                              s);
        if (rc) return rc;
    }
    // result records into host memory in fixed-size pieces (no allocation)
    double r[16 * mp::DIAG_VALS];
    int64_t bad = 0;
    for (int i0 = 0; i0 < n; i0 += 16) {
        const int m = std::min(16, n - i0);
        rc = hip_check(hipMemcpyAsync(r, scr + (size_t)(mp::DIAG_BLOCKS_MAX + i0) * mp::DIAG_VALS,
                                      sizeof(double) * mp::DIAG_VALS * m, hipMemcpyDeviceToHost, s),
                       "diagnostics copy");
        if (rc == MP_OK) rc = hip_check(hipStreamSynchronize(s), "diagnostics sync");
        if (rc) return rc;
        for (int j = 0; j < m; ++j) {
            unpack_diag(st, i0 + j, &r[(size_t)j * mp::DIAG_VALS], step, &out[i0 + j]);
            bad += out[i0 + j].nonfinite;
        }
    }
    if (bad > 0) return fail(MP_E_NONFINITE, "%lld cells hold NaN or Inf", (long long)bad);
    return ok();
}

int mp_set_tile(mp_state* st, int bx, int seg, int vec) {
    if (!st) return fail(MP_E_NULLPTR, "state is NULL");
    const bool d3 = st->inst[0].grid.dim == 3;
    if (bx) {
        bool okbx = d3 ? (bx == 256 || (bx == 512 && d3_tall_ok(st)))
                       : (bx == 64 || bx == 128 || bx == 256);
        if (st->batch) okbx = bx == 64 * mp::BATCH_WPB_HOST;
        if (!okbx) return fail(MP_E_PARAM, "unsupported tile width %d", bx);
    }
    if (seg < 0) return fail(MP_E_PARAM, "seg must be >= 1");
    if (vec) {
        const int vmax = st->precision == MP_FP64 ? 2 : 4;
        const bool okv = d3 ? vec == 1 : (vec == -1 || vec == 1 || vec == 2 || vec == 4);
        if (!okv || vec > vmax || (st->batch && vec > 2))
            return fail(MP_E_PARAM, "unsupported cells per lane %d", vec);
    }
    drop_graphs(st);
    if (bx) st->bx = bx;
    if (vec) st->vec = d3 ? -1 : vec;
    if (seg) st->seg = seg;
    if ((seg || vec) && st->batch) {
        const int rc = sync_batch(st);
        if (rc) return rc;
    }
    return ok();
}

int mp_get_tile(const mp_state* st, int* bx, int* seg, int* vec) {
    if (!st) return fail(MP_E_NULLPTR, "state is NULL");
    if (bx) *bx = st->bx;
    if (seg) *seg = st->seg;
    if (vec) *vec = st->vec;
    return ok();
}

int mp_tune_candidates(const mp_state* st, int32_t* cand, int cap) {
    if (!st) return fail(MP_E_NULLPTR, "state is NULL");
    if (cap < 0) return fail(MP_E_PARAM, "cap must be >= 0");
    std::vector<int32_t> v;
    const bool d3 = st->inst[0].grid.dim == 3;
    const int vmax = st->precision == MP_FP64 ? 2 : 4;
    if (d3) {
        for (int bx : {256, 512})
            if (bx == 256 || d3_tall_ok(st))
                for (int seg : {4, 8, 16, 32, 64}) v.insert(v.end(), {bx, seg, 1, 1});
    } else if (st->batch) {
        for (int fuse = 1; fuse <= 2; ++fuse)
            for (int vec = 1; vec <= 2; vec *= 2)
                for (int seg : {4, 8, 16, 32, 64})
                    v.insert(v.end(), {64 * mp::BATCH_WPB_HOST, seg, vec, fuse});
    } else {
        for (int fuse = 1; fuse <= 2; ++fuse)
            for (int vec = 1; vec <= vmax; vec *= 2)
                for (int bx : {64, 128, 256})
                    for (int seg : {4, 8, 16, 32, 64}) v.insert(v.end(), {bx, seg, vec, fuse});
    }
    const int n = (int)(v.size() / 4);
    if (cand)
        for (int i = 0; i < n && i < cap; ++i)
            for (int j = 0; j < 4; ++j) cand[4 * i + j] = v[4 * i + j];
    ok();
    return n;
}

int mp_tune(mp_state* st, const int32_t* cand, int ncand, int reps, double* ms, int* best,
            void* stream) {
    if (!st || !cand || !ms || !best) return fail(MP_E_NULLPTR, "state, cand, ms or best is NULL");
    if (!st->bound) return fail(MP_E_UNBOUND, "mp_tune before mp_bind");
    if (ncand < 1 || reps < 1) return fail(MP_E_PARAM, "ncand and reps must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    const int bx0 = st->bx, seg0 = st->seg, vec0 = st->vec, fuse0 = st->fuse;
    hipEvent_t e[2] = {nullptr, nullptr};
    int rc = hip_check(hipEventCreate(&e[0]), "hipEventCreate");
    if (rc == MP_OK) rc = hip_check(hipEventCreate(&e[1]), "hipEventCreate");
    int bi = -1;
    for (int i = 0; i < ncand && rc == MP_OK; ++i) {
        ms[i] = -1.0;
        const int32_t* c = cand + 4 * i;
        if (mp_set_fusion(st, c[3]) != MP_OK) continue;
        if (mp_set_tile(st, c[0], c[1], c[2]) != MP_OK) continue;
        mp::KernelCall k;
        if (make_step_call(st, 0, st->cur, k, launch_fuse(st)) != MP_OK) continue;
        rc = launch(k, s);
        if (rc == MP_OK) rc = hip_check(hipEventRecord(e[0], s), "hipEventRecord");
        for (int r = 0; r < reps && rc == MP_OK; ++r) rc = launch(k, s);
        if (rc == MP_OK) rc = hip_check(hipEventRecord(e[1], s), "hipEventRecord");
        if (rc == MP_OK) rc = hip_check(hipEventSynchronize(e[1]), "hipEventSynchronize");
        float t = 0.0f;
        if (rc == MP_OK) rc = hip_check(hipEventElapsedTime(&t, e[0], e[1]), "hipEventElapsedTime");
        if (rc != MP_OK) break;
        ms[i] = (double)t / reps / launch_fuse(st);
        if (bi < 0 || ms[i] < ms[bi]) bi = i;
    }
    for (hipEvent_t x : e)
        if (x) (void)hipEventDestroy(x);
    if (rc != MP_OK || bi < 0) {
        const std::string why = rc != MP_OK ? g_err : std::string("no valid tile candidate");
        (void)mp_set_fusion(st, fuse0);
        (void)mp_set_tile(st, bx0, seg0, vec0);
        return fail(rc != MP_OK ? rc : MP_E_PARAM, "mp_tune: %s", why.c_str());
    }
    const int32_t* c = cand + 4 * bi;
    rc = mp_set_fusion(st, c[3]);
    if (rc == MP_OK) rc = mp_set_tile(st, c[0], c[1], c[2]);
    if (rc) return rc;
    *best = bi;
    return ok();
}

int mp_set_fusion(mp_state* st, int steps) {
    if (!st) return fail(MP_E_NULLPTR, "state is NULL");
    if (steps != 1 && steps != 2) return fail(MP_E_PARAM, "steps per launch must be 1 or 2 (got %d)", steps);
    if (steps == 2 && st->inst[0].grid.dim != 2)
        return fail(MP_E_PARAM, "two steps per launch exist for 2D grids only");
    drop_graphs(st);
    st->fuse = steps;
    if (st->batch && st->bound) return choose_batch_blocks(st);
    return ok();
}

int mp_get_fusion(const mp_state* st, int* steps) {
    if (!st || !steps) return fail(MP_E_NULLPTR, "state or steps is NULL");
    *steps = st->fuse;
    return ok();
}

int mp_set_antitrapping(mp_state* st, int on) {
    if (!st) return fail(MP_E_NULLPTR, "state is NULL");
    if (on < 0 || on > 2) return fail(MP_E_PARAM, "on must be 0, 1 or 2 (got %d)", on);
    if (on == 2 && st->batch)
        return fail(MP_E_STATE, "anti-trapping current: batched states take it folded into the step (on = 1) only");
    if (on != 0)
        for (const Inst& I : st->inst)
            if (I.prm.model == MP_KKS)
                return fail(MP_E_STATE, "anti-trapping current: built for the grand-potential model only");
    drop_graphs(st);
    const int was = st->antitrap;
    st->antitrap = on;
    if (st->batch && st->bound && (was != 0) != (on != 0)) {
        // the kernel changes, and with it the resident block count and the work list's deal
        const int rc = choose_batch_blocks(st);
        if (rc) {
            st->antitrap = was;
            return rc;
        }
    }
    return ok();
}

int mp_get_antitrapping(const mp_state* st, int* on) {
    if (!st || !on) return fail(MP_E_NULLPTR, "state or on is NULL");
    *on = st->antitrap;
    return ok();
}

int mp_set_graph(mp_state* st, int chunk) {
    if (!st) return fail(MP_E_NULLPTR, "state is NULL");
    if (chunk < 0 || (chunk > 0 && (chunk < 2 || chunk % 2)))
        return fail(MP_E_PARAM, "graph chunk must be 0 or an even number >= 2 (got %d)", chunk);
    drop_graphs(st);
    st->graph_chunk = chunk;
    return ok();
}

int mp_instance_count(const mp_state* st, int* ninst) {
    if (!st || !ninst) return fail(MP_E_NULLPTR, "state or ninst is NULL");
    *ninst = (int)st->inst.size();
    return ok();
}

int mp_instance_offset(const mp_state* st, int i, size_t* offset_bytes, size_t* nbytes) {
    if (!st) return fail(MP_E_NULLPTR, "state is NULL");
    if (i < 0 || i >= (int)st->inst.size()) return fail(MP_E_PARAM, "instance %d out of range", i);
    if (offset_bytes) *offset_bytes = st->inst[i].off_bytes;
    if (nbytes) *nbytes = st->inst[i].bytes;
    return ok();
}

size_t mp_adjoint_work_bytes(const mp_state* st, int64_t every) {
    if (!st || every < 1 || st->batch) return 0;
    return adj_layout(st, every).total;
}

int mp_step_ckpt(mp_state* st, int64_t nsteps, int64_t every, void* ckpt_buf, void* stream) {
    if (!st || !ckpt_buf) return fail(MP_E_NULLPTR, "state or checkpoint buffer is NULL");
    if (!st->bound) return fail(MP_E_UNBOUND, "mp_step_ckpt before mp_bind");
    if (st->batch) return fail(MP_E_STATE, "checkpointing: batched states are not supported");
    if (nsteps < 0 || every < 1) return fail(MP_E_PARAM, "nsteps must be >= 0 and every >= 1");
    hipStream_t s = (hipStream_t)stream;
    const size_t sb = st->inst[0].bytes;
    const size_t stride = align_up(sb);
    for (int64_t done = 0, c = 0; done < nsteps; done += every, ++c) {
        int rc = hip_check(hipMemcpyAsync((char*)ckpt_buf + (size_t)c * stride, st->buf[st->cur], sb,
                                          hipMemcpyDeviceToDevice, s),
                           "checkpoint copy");
        if (rc) return rc;
        const int64_t len = nsteps - done < every ? nsteps - done : every;
        rc = mp_step(st, len, stream);
        if (rc) return rc;
    }
    return ok();
}

int mp_adjoint(mp_state* st, const void* ckpt_buf, int64_t nsteps, int64_t every, int64_t n0,
               const void* lam_final, void* lam_initial, double* grad_theta, void* work, void* stream) {
    if (!st) return fail(MP_E_NULLPTR, "mp_adjoint: state is NULL");
    int rc = adj_supported(st);
    if (rc) return rc;
    if (!ckpt_buf || !lam_final || !lam_initial || !grad_theta || !work)
        return fail(MP_E_NULLPTR, "mp_adjoint: NULL argument");
    if (!st->bound) return fail(MP_E_UNBOUND, "mp_adjoint before mp_bind");
    if (nsteps < 0 || every < 1 || n0 < 0) return fail(MP_E_PARAM, "nsteps, n0 must be >= 0 and every >= 1");
    if (((uintptr_t)work | (uintptr_t)ckpt_buf) & (kAlign - 1))
        return fail(MP_E_PARAM, "work and checkpoint buffers must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    const Inst& I = st->inst[0];
    const AdjLayout L = adj_layout(st, every);
    char* w = (char*)work;
    const size_t sb = I.bytes;
    void* X[2] = {w + L.X0, w + L.X1};
    void* lam = w + L.lam;  // lambda, updated in place
    double* acc = (double*)(w + L.acc);
    int64_t* zctr = (int64_t*)(w + L.ctr);
    double* gdev = (double*)(w + L.grad);
    rc = hip_check(hipMemcpyAsync(lam, lam_final, sb, hipMemcpyDeviceToDevice, s), "lambda copy");
    if (rc) return rc;
    mp::adj_fill(acc, (int64_t)L.nrows * mp::ADJ_NPAR, 0.0, s);
    mp::adj_fill((double*)zctr, 1, 0.0, s);  // all-zero bits: the int64 time-level base 0
    int dev = 0, cus = 0;
    rc = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (rc == MP_OK) rc = hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "CU count");
    if (rc) return rc;
    mp::AdjLaunch A;
    A.g = adj_geom(I, cus, st->precision == MP_FP64);
    if (adj_nblocks(A.g, st->precision == MP_FP64) > L.nrows)
        return fail(MP_E_STATE, "adjoint: wave plan exceeds the accumulator rows");
    A.nphases = I.N;
    A.nmu = I.K - 1;
    A.lam = lam;
    A.acc = acc;
    double tb0, tdn, tslope;
    temperature_law(I, tb0, tdn, tslope);
    A.tt_slope = tslope;
    const mp::AdjCoef<double> cd = make_adj_coef<double>(I);
    const mp::AdjCoef<float> cf = make_adj_coef<float>(I);
    auto run = [&](int which, const char* sB, const void* XB, const char* sA, void* XA, int64_t nA) {
        A.which = which;
        A.sB = sB;
        A.XB = XB;
        A.sA = sA;
        A.XA = XA;
        A.tt_row0 = tb0 + tdn * (double)nA;
        int r = st->precision == MP_FP64 ? mp::adj_launch<double>(A, cd, s) : mp::adj_launch<float>(A, cf, s);
        if (r) return fail(r, "no adjoint instance for this configuration");
        return hip_check(hipGetLastError(), "adjoint launch");
    };
    const int64_t nseg = (nsteps + every - 1) / every;
    auto len_of = [&](int64_t k) { return (nsteps - k * every) < every ? (nsteps - k * every) : every; };
    // Segment k's states, restored from checkpoint k and recomputed into
    // buffer k mod 2, on stream q.
    // Two steps per launch where the kernel can also store the state between
    // them (2D single grid at one cell per lane), else one.
    auto recompute = [&](int64_t k, hipStream_t q) {
        char* seg = w + L.seg[k & 1];
        auto at = [&](int64_t i) { return seg + (size_t)i * L.state; };
        int r = hip_check(hipMemcpyAsync(seg, (const char*)ckpt_buf + (size_t)k * L.state, sb,
                                         hipMemcpyDeviceToDevice, q),
                          "checkpoint restore");
        for (int64_t i = 0; r == MP_OK && i + 1 < len_of(k);) {
            const int kstep = (int)(n0 + k * every + i);
            mp::KernelCall kc;
            if (i + 2 < len_of(k) && make_single_call(st, at(i), at(i + 2), zctr, kstep, kc, 2, at(i + 1)) == MP_OK) {
                i += 2;
            } else {
                r = make_single_call(st, at(i), at(i + 1), zctr, kstep, kc);
                if (r) return fail(r, "no kernel instance for this configuration");
                i += 1;
            }
            r = launch(kc, q);
        }
        return r;
    };
    // Reverse sweep of segment k on the caller's stream: part A of its last
    // step, then part B of each step fused with part A of the step before it,
    // then part B of its first step.
    auto sweep = [&](int64_t k) {
        char* seg = w + L.seg[k & 1];
        const int64_t base = n0 + k * every, len = len_of(k);
        auto at = [&](int64_t i) { return seg + (size_t)i * L.state; };
        int p = 0;
        int r = run(0, nullptr, nullptr, at(len - 1), X[p], base + len - 1);
        for (int64_t i = len - 1; i >= 1 && r == MP_OK; --i) {
            r = run(2, at(i), X[p], at(i - 1), X[1 - p], base + i - 1);
            p = 1 - p;
        }
        if (r == MP_OK) r = run(1, at(0), X[p], nullptr, nullptr, base);
        return r;
    };
    // Segment k-1 is recomputed on the second stream while segment k is swept
    // (it waits for the sweep of k+1, the last reader of its buffer).
    if (!st->aux) {
        rc = hip_check(hipStreamCreateWithFlags(&st->aux, hipStreamNonBlocking), "adjoint stream");
        for (hipEvent_t& e : st->ev)
            if (rc == MP_OK) rc = hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "adjoint event");
        if (rc) return rc;
    }
    hipEvent_t* evrec = st->ev + 1;
    hipEvent_t* evsw = st->ev + 3;
    rc = hip_check(hipEventRecord(st->ev[0], s), "hipEventRecord");
    if (rc == MP_OK) rc = hip_check(hipStreamWaitEvent(st->aux, st->ev[0], 0), "hipStreamWaitEvent");
    if (rc == MP_OK && nseg > 0) rc = recompute(nseg - 1, st->aux);
    if (rc == MP_OK && nseg > 0) rc = hip_check(hipEventRecord(evrec[(nseg - 1) & 1], st->aux), "hipEventRecord");
    for (int64_t k = nseg - 1; k >= 0 && rc == MP_OK; --k) {
        if (k >= 1) {
            if (k + 1 <= nseg - 1)
                rc = hip_check(hipStreamWaitEvent(st->aux, evsw[(k + 1) & 1], 0), "hipStreamWaitEvent");
            if (rc == MP_OK) rc = recompute(k - 1, st->aux);
            if (rc == MP_OK) rc = hip_check(hipEventRecord(evrec[(k - 1) & 1], st->aux), "hipEventRecord");
        }
        if (rc == MP_OK) rc = hip_check(hipStreamWaitEvent(s, evrec[k & 1], 0), "hipStreamWaitEvent");
        if (rc == MP_OK) rc = sweep(k);
        if (rc == MP_OK) rc = hip_check(hipEventRecord(evsw[k & 1], s), "hipEventRecord");
    }
    if (rc) return rc;
    rc = hip_check(hipMemcpyAsync(lam_initial, lam, sb, hipMemcpyDeviceToDevice, s), "lambda copy");
    if (rc) return rc;
    mp::adj_reduce(acc, L.nrows, gdev, s);
    rc = hip_check(hipMemcpyAsync(grad_theta, gdev, sizeof(double) * mp::ADJ_NPAR, hipMemcpyDeviceToHost, s),
                   "gradient copy");
    if (rc) return rc;
    return hip_check(hipStreamSynchronize(s), "adjoint sync");
}

int mp_front_row(mp_state* st, int64_t* row, void* stream) {
    if (!st || !row) return fail(MP_E_NULLPTR, "state or row is NULL");
    if (st->batch) return fail(MP_E_STATE, "mp_front_row: batched states are not supported");
    if (!st->bound) return fail(MP_E_UNBOUND, "mp_front_row before mp_bind");
    hipStream_t s = (hipStream_t)stream;
    const Inst& I = st->inst[0];
    // scratch: the diagnostics partials and the first result record of the workspace
    double* ws = (double*)st->ws;
    int64_t* res = (int64_t*)(ws + (size_t)mp::DIAG_BLOCKS_MAX * mp::DIAG_VALS);
    int rc = mp::launch_front(st->buf[st->cur], st->precision, make_geom(I.grid), I.N, (int*)ws, res, s);
    if (rc) return fail(rc, "no front kernel");
    rc = hip_check(hipGetLastError(), "front launch");
    int64_t r = -1;
    if (rc == MP_OK) rc = hip_check(hipMemcpyAsync(&r, res, sizeof r, hipMemcpyDeviceToHost, s), "front copy");
    if (rc == MP_OK) rc = hip_check(hipStreamSynchronize(s), "front sync");
    if (rc) return rc;
    *row = r;
    return ok();
}

int mp_shift(mp_state* st, int64_t rows, const double* mu_melt, int64_t* offset, void* stream) {
    if (!st) return fail(MP_E_NULLPTR, "state is NULL");
    if (st->batch) return fail(MP_E_STATE, "mp_shift: batched states are not supported");
    if (!st->bound) return fail(MP_E_UNBOUND, "mp_shift before mp_bind");
    Inst& I = st->inst[0];
    if (rows < 0 || rows > I.grid.n[1]) return fail(MP_E_PARAM, "rows must lie in [0, ny]");
    if (!mu_melt && I.K > 1) return fail(MP_E_NULLPTR, "mu_melt is NULL");
    for (int k = 0; k < I.K - 1; ++k)
        if (!std::isfinite(mu_melt[k])) return fail(MP_E_PARAM, "mu_melt[%d] must be finite", k);
    if (rows > 0) {
        int rc = mp::launch_shift(st->buf[st->cur], st->buf[1 - st->cur], st->precision, make_geom(I.grid), I.N,
                                  I.K - 1, (int)rows, mu_melt, (hipStream_t)stream);
        if (rc) return fail(rc, "no shift kernel");
        rc = hip_check(hipGetLastError(), "shift launch");
        if (rc) return rc;
        st->cur = 1 - st->cur;
        I.yshift += rows;
        drop_graphs(st);  // the temperature law's origin is a kernel argument
    }
    if (offset) *offset = I.yshift;
    return ok();
}

void mp_destroy(mp_state* st) {
    if (!st) return;
    drop_graphs(st);
    for (hipEvent_t e : st->ev)
        if (e) (void)hipEventDestroy(e);
    if (st->aux) (void)hipStreamDestroy(st->aux);
    delete st;
}

const char* mp_last_error(void) { return g_err.c_str(); }

}  // extern "C"
