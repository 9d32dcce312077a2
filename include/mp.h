/*
 * mp.h - C ABI of the explicit grand-potential phase-field step (libmpstep.so).
 *
 * The library advances N phase fields phi_a and K-1 diffusion potentials mu_k
 * of the multiphase, multicomponent grand-potential model of MICROSIM
 * (arXiv 2404.01035, Sec. 2.1) by forward-Euler steps on a regular 2D or 3D
 * grid, one fused HIP kernel per step on gfx950:
 *
 *   phi: Eq. phi_eqn (Allen-Cahn with the gradient energy of Eq. Eqn_a and the
 *        four-fold a_c, the potential of Eq. Well or Eq. Obstacle, the driving
 *        force sum_b psi^b dh_b/dphi_a with h of Eq. hphi, and the Lagrange
 *        multiplier that keeps sum_a phi_a = 1; no elastic term);
 *   mu : Eq. Mu_explicit_temperature with M of Eq. Mass_conservation and the
 *        parabolic free energies of Eq. free_energy_density (diagonal
 *        curvatures, or for two mu fields the symmetric 2 x 2 with an
 *        off-diagonal term; B and C optionally functions of T with the dT/dt
 *        term); the anti-trapping current of Eq. jatr is off unless
 *        mp_set_antitrapping switches it on (2D and 3D single grids, batches).
 *
 * Conventions for every call:
 *   - Return value: MP_OK (0) or a negative MP_E_* code; mp_last_error()
 *     gives a message for the calling thread.  No call aborts or throws.
 *   - Device memory is owned by the caller.  The library only borrows the
 *     pointers given to mp_bind and never allocates or frees device memory
 *     itself (mp_destroy frees host-side state only).
 *   - Environment: MP_LOG (anything but "0") echoes every failure message to
 *     stderr; MP_TILE="bx,seg,vec" sets the tile shape of every state made by
 *     mp_create, as mp_set_tile would (an invalid value makes mp_create fail
 *     with MP_E_PARAM).
 *   - ``stream`` is a hipStream_t passed as void* (NULL = the null stream).
 *     mp_step is asynchronous; faults inside a kernel surface at the next
 *     synchronising call (mp_diagnostics, or the caller's own sync).
 *
 * State layout (one state buffer): structure of arrays, field-major,
 *   [N phase fields][K-1 mu fields] x [nz][ny][nx], x fastest, contiguous,
 * elements double (MP_FP64) or float (MP_FP32).  A torch tensor of shape
 * (N + K - 1, nz, ny, nx) (2D: (N + K - 1, ny, nx)) maps onto it 1:1.  Two such
 * buffers are used as ping-pong; after mp_step the current one is reported by
 * mp_current.
 */
#ifndef MPSTEP_MP_H
#define MPSTEP_MP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MP_MAX_PHASES 3
#define MP_MAX_MU 2

enum {
    MP_OK = 0,
    MP_E_PARAM = -1,     /* a size, code or coefficient is outside what the library supports */
    MP_E_UNSTABLE = -2,  /* dt above the explicit stability limit (mp_dt_limit) */
    MP_E_NULLPTR = -3,   /* a required pointer is NULL */
    MP_E_UNBOUND = -4,   /* mp_step / mp_diagnostics before mp_bind */
    MP_E_HIP = -5,       /* a HIP runtime call failed (message holds hipGetErrorString) */
    MP_E_NONFINITE = -6, /* mp_diagnostics found NaN/Inf in the state */
    MP_E_STATE = -7      /* call not valid for this state (e.g. batch vs single) */
};

enum { MP_BC_PERIODIC = 0, MP_BC_NOFLUX = 1 };   /* BOUNDARY codes 3 and 1 of Sec. 5 */
enum { MP_FP64 = 0, MP_FP32 = 1 };
/* Function_W of Sec. 5: Eq. Well, Eq. Obstacle.  The obstacle's "infinite outside
 * [0, 1]" is imposed either by clipping the forward-Euler update to [0, 1] and
 * renormalising (MP_OBSTACLE) or with the Lagrange multiplier over the active
 * phases, i.e. the update's nearest point of the simplex {phi >= 0, sum phi = 1}
 * (MP_OBSTACLE_ACTIVE). */
enum { MP_WELL = 0, MP_OBSTACLE = 1, MP_OBSTACLE_ACTIVE = 2, MP_THETA = 3 };
/* The model (Sec. 2): grand potential (Sec. 2.1), or the KKS variant (Sec.
 * 2.2) whose phase fields follow Eq. aceq; MP_THETA, the sextic potential of
 * Eq. Well1, is a KKS potential. */
enum { MP_GP = 0, MP_KKS = 1 };

typedef struct mp_state mp_state; /* opaque */

/* Regular grid.  dim = 2 or 3; n = (nx, ny, nz) with nz = 1 in 2D; each n >= 1.
 * bc per axis (x, y, z): MP_BC_PERIODIC wraps, MP_BC_NOFLUX mirrors the edge
 * cell into the ghost (zero normal flux).  Cell j of an axis sits at j*dx. */
typedef struct {
    int32_t dim;
    int32_t bc[3];
    int64_t n[3];
    double dx;
} mp_grid;

/* Model coefficients (host FP64; converted once to the run precision).
 * Only entries [a][b] with a, b < N and [a][k] with k < K-1 are read.
 *   gamma[a][b]  interface energy gamma_ab (symmetric), Eq. Well / Eq. Obstacle
 *   gamma3       third-order gamma_abd of the same equations (N = 3)
 *   delta[a][b]  four-fold anisotropy strength delta_ab (symmetric; 0 = isotropic)
 *   eps, tau     interface width and relaxation constant of Eq. phi_eqn
 *   dt           time step; must satisfy dt <= mp_dt_limit(...)
 *   A, B, C      f^a(c) = sum_k A[a][k] c_k^2 + B[a][k] c_k + C[a]   (A > 0)
 *   s            C^a(T) = C[a] + s[a] (T - Te)
 *   D            diffusivity per phase and component, >= 0 (Eq. Mass_conservation)
 *   Te, T0, G, V, y0  temperature T(y,t) = T0 + G (y - y0 - V t), t = step * dt
 *                (the Tempgrady key of Sec. 5)
 * Extended model (all zero: the terms are absent; a state that uses any of them
 * runs the general kernels, see mp_create):
 *   Bt, Ct       temperature dependence of the parabolic coefficients from the
 *                slopes of the coexistence lines (Sec. 3):
 *                B^a_k(T) = B[a][k] + Bt[a][k] (T - Te),
 *                C^a(T) = C[a] + s[a] (T - Te) + Ct[a] (T - Te)^2; the mu update
 *                then carries the dT/dt term of Eq. Mu_explicit_temperature
 *   A01          off-diagonal curvature: f^a gains A01[a] c_0 c_1 (Eq.
 *                free_energy_density with its i < j term; K = 3); every
 *                [[2 A[a][0], A01[a]], [A01[a], 2 A[a][1]]] must be positive definite
 *   D01          symmetric off-diagonal diffusivity D^a_01 = D^a_10 (Eq.
 *                Mass_conservation with a full D^a; K = 3), D^a positive semidefinite
 *   tau_ab       relaxation constant per phase pair (the Tau key of Sec. 5;
 *                symmetric, all > 0 or all 0): tau of Eq. phi_eqn becomes
 *                sum_{a<b} tau_ab phi_a phi_b / sum_{a<b} phi_a phi_b, and tau
 *                where that pair sum is <= 1e-30
 * KKS variant (model = MP_KKS; Sec. 2.2): the phase fields follow Eq. aceq,
 *   (1/Mphi) dphi_a/dt = (eps^2/2)(div da/dgrad phi_a - da/dphi_a) - dg/dphi_a
 *                        - sum_b psi^b dh_b/dphi_a - lambda,
 *   with eps the gradient-energy coefficient of Eq. fe, the same a, faces and
 *   driving force as above, and g of the form of Eq. Well (potential MP_WELL,
 *   with gamma and gamma3, no 1/eps) or Eq. Well1 (MP_THETA):
 *   sum_a theta[a] phi_a^2 (1-phi_a)^2 + sum_{a<b} theta_ab[a][b] phi_a^2 phi_b^2
 *   + theta3 phi_0^2 phi_1^2 phi_2^2 (N = 3).  The diffusion potentials take
 *   the same update (the linearised composition equation of Eq. cheq is Eq.
 *   Mu_explicit_temperature).  tau and tau_ab are not read (tau_ab must be 0).
 *   Mphi         phase-field mobility M_phi of Eq. aceq (> 0)
 *   theta, theta_ab, theta3  the Theta coefficients of Eq. Well1 (>= 0;
 *                theta_ab symmetric) */
typedef struct {
    int32_t precision; /* MP_FP64 | MP_FP32 */
    int32_t potential; /* MP_WELL | MP_OBSTACLE | MP_OBSTACLE_ACTIVE | MP_THETA (KKS) */
    double eps, tau, dt;
    double gamma[3][3];
    double gamma3;
    double delta[3][3];
    double A[3][2], B[3][2], C[3];
    double s[3];
    double D[3][2];
    double Te, T0, G, V, y0;
    double Bt[3][2], Ct[3];
    double A01[3], D01[3];
    double tau_ab[3][3];
    int32_t model;     /* MP_GP | MP_KKS */
    int32_t reserved;  /* 0 */
    double Mphi;
    double theta[3];
    double theta_ab[3][3];
    double theta3;
} mp_params;

/* Global diagnostics of the current state, reduced in FP64 with Neumaier
 * compensation in a fixed order (bitwise reproducible run to run). */
typedef struct {
    int64_t step;          /* time level of the state */
    int64_t nonfinite;     /* cells holding a NaN or Inf in any field */
    double max_sum_dev;    /* max over cells of |sum_a phi_a - 1| (Sec. 2.1 constraint) */
    double mass[2];        /* sum over cells of c_k dx^d, c_k = sum_a h_a c^a_k(mu) */
    double volume[3];      /* sum over cells of phi_a dx^d */
    double min_chi[2];     /* min over cells of sum_a h_a dc^a_k/dmu_k */
} mp_diag;

/* Explicit stability limit used by mp_create (host only, no GPU needed):
 * dx^2/(2d) * min( tau / (2 gamma_max (N-1)/N (1 + 20 delta_max)),
 *                  min_k min_a chi^a_k / max_a (D^a_k chi^a_k) ), chi = 1/(2A);
 * with per-pair tau_ab the smallest of them and tau counts, and with A01 or D01
 * the mu part is min_a lambda_min(chi^a) / max_a |D^a chi^a|_2 (chi^a the
 * inverse curvature matrix), a bound on the eigenvalues of chi^-1 M.  KKS:
 * tau is replaced by 2 / (Mphi eps^2) (the gradient term of Eq. aceq) and the
 * potential's stiffness adds dt <= 1 / (Mphi S), S = max_a of
 * 2 theta[a] + sum_b 2 theta_ab[a][b] (MP_THETA) or sum_b 18 gamma[a][b] (MP_WELL).
 * Returns a negative value for invalid input. */
double mp_dt_limit(const mp_grid* grid, int nphases, int ncomp, const mp_params* params);

/* Validate the problem and build a solver state (host only, no GPU needed):
 * the grand-potential step of Sec. 2.1 (Eq. phi_eqn for the phase fields, Eq.
 * Mu_explicit_temperature for the diffusion potentials) on this grid, or with
 * model = MP_KKS the KKS variant of Sec. 2.2 (Eq. aceq for the phase fields).
 * nphases N in {2, 3}; ncomp K in {2, 3} (K - 1 diffusion potentials).  A
 * problem that uses the extended model (non-zero Bt, Ct, A01, D01 or tau_ab,
 * MP_OBSTACLE_ACTIVE, or the KKS potential MP_THETA) runs the general
 * kernels: one cell per lane in 2D and 64 x 4 tiles in 3D whatever
 * mp_set_tile says (batched instances too, and with the anti-trapping
 * current); the adjoint does not take it.  The KKS variant with MP_WELL runs
 * the plain kernels with its own folded coefficients.
 * Errors: MP_E_NULLPTR, MP_E_PARAM (dim, n, bc, dx, N, K, precision, model,
 * potential, eps, tau, Mphi, A, D, gamma, delta, theta or an extended
 * coefficient out of range), MP_E_UNSTABLE. */
int mp_create(const mp_grid* grid, int nphases, int ncomp, const mp_params* params,
              mp_state** out);

/* Bytes of one state buffer, and of the workspace mp_bind needs. */
size_t mp_state_bytes(const mp_state* st);
size_t mp_workspace_bytes(const mp_state* st);

/* Attach caller-owned device buffers: buf0 and buf1 each mp_state_bytes()
 * long, 256-byte aligned; workspace mp_workspace_bytes() long (reduction
 * partial sums, the device copy of the time level, for a single grid the
 * partial records of mp_step_diag (at most 8 MiB) and, for a batch, the
 * instance table, the work list and the anti-trapping and extended-model
 * coefficients).  buf0 is the current buffer afterwards and the time level
 * is reset to 0 (use mp_set_step to resume).  Needs the GPU: it writes the
 * workspace with a synchronous copy. */
int mp_bind(mp_state* st, void* buf0, void* buf1, void* workspace);

/* Advance nsteps >= 0 forward-Euler steps (Sec. 2.1: the explicit scheme of
 * Eq. phi_eqn and Eq. Mu_explicit_temperature) on ``stream`` (asynchronous).
 * Each kernel launch reads the current buffer and writes the other one, and
 * performs one step, or two (mp_set_fusion; an odd remainder is a single
 * step), so the current buffer flips once per launch: mp_current
 * reports it.  The time level advances by nsteps.  Results are bitwise the
 * same either way. */
int mp_step(mp_state* st, int64_t nsteps, void* stream);

/* Which bound buffer (0 or 1) holds the current state, and its time level. */
int mp_current(const mp_state* st, int* which_buf, int64_t* step);

/* Declare that buffer ``which_buf`` holds the state at time level ``step``
 * (updates the device copy of the time level synchronously when bound). */
int mp_set_step(mp_state* st, int64_t step, int which_buf);

/* Reduce the current state into *out (synchronises ``stream``).
 * Returns MP_E_NONFINITE (with *out filled) when a NaN/Inf is present, and
 * MP_E_STATE for a batched state (use mp_diagnostics_batch). */
int mp_diagnostics(mp_state* st, mp_diag* out, void* stream);

/* Advance nsteps >= 1 steps as mp_step does, then reduce the state reached
 * into *out with the diagnostics' partial sums formed inside the last step
 * launch from the values it stores, so the state is not read again (the
 * global checks of Sec. 2.1: the constraint sum_a phi_a = 1, the solute of the
 * composition constraint, phase volumes, the susceptibility).  The fields are
 * those of mp_diagnostics: max_sum_dev, min_chi and nonfinite equal its values
 * bit for bit; mass and volume agree with them to rounding (FP64 Neumaier
 * partial sums grouped by the step kernel's strips or tiles, reproducible run
 * to run for one tile shape).  The state after the call is bitwise that of
 * mp_step.  Formed in the step launch for single grids in FP64 2D and in 3D;
 * a batched state (out then takes one record per instance), the anti-trapping
 * current, an FP32 2D grid (there the separate pass is faster) or a tile
 * whose last launch would write more than 65536 partial records (2D: one per
 * strip wave, 3D: one per tile) takes mp_step followed by the separate
 * reduction.  Partial records live in the
 * workspace.  Synchronises ``stream``.  Errors: MP_E_NULLPTR, MP_E_UNBOUND,
 * MP_E_PARAM (nsteps < 1), MP_E_NONFINITE (*out filled), MP_E_HIP. */
int mp_step_diag(mp_state* st, int64_t nsteps, mp_diag* out, void* stream);

/* mp_diagnostics without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  state_buf is a device buffer holding the state at time
 * level ``step`` in the layout of ``st`` (mp_create or mp_create_batch; st need
 * not be bound); out receives one mp_diag per instance (host memory).  The
 * reduction's partial sums and result records live in a static device array
 * of the library (about 160 KiB: 1024 partial records and one record per
 * instance, at most 256 instances), which each GPU holds until the process
 * ends; the call allocates no memory.  Every call on a GPU shares that array:
 * calls that overlap on one GPU (other streams or host threads) race.  Same
 * kernels and results as mp_diagnostics / mp_diagnostics_batch.  Synchronises
 * ``stream``.  Errors: MP_E_NULLPTR, MP_E_PARAM (more than 256 instances,
 * step < 0), MP_E_NONFINITE (out filled), MP_E_HIP. */
int mp_diagnostics_static(const mp_state* st, const void* state_buf, int64_t step, mp_diag* out,
                          void* stream);

/* Tile shape of the step kernel.  2D: bx = threads per block (64, 128 or
 * 256: 1, 2 or 4 independent strip waves), seg = rows per strip segment and
 * vec = the most cells one lane holds (1, 2, or 4 in FP32 only; each lane
 * takes the largest power of two <= vec that divides nx; -1 = the widest the
 * precision allows).  A batched state takes bx = 256 and vec in {-1, 1, 2}
 * (-1 acts as 2).  3D: bx = 256 (64 x 4 tiles) or 512 (64 x 8 tiles, where
 * the tile's LDS ring fits in 64 KiB), seg = z planes per block, vec must be
 * 0 or 1.  0 keeps the current value of a
 * field.  Results do not depend on the tile shape (bitwise). */
int mp_set_tile(mp_state* st, int bx, int seg, int vec);
int mp_get_tile(const mp_state* st, int* bx, int* seg, int* vec);

/* Autotuning support.  mp_tune_candidates writes up to ``cap`` candidates
 * (bx, seg, vec, steps per launch) valid for this state into
 * cand[4*i .. 4*i+3] and returns how many there are (a negative MP_E_* on
 * error); cand may be NULL to query the count.  mp_tune times each of the
 * ncand candidates in ``cand``: one untimed launch, then ``reps`` launches
 * from the current buffer into the other one, bracketed by events on
 * ``stream``, and stores the mean milliseconds per step in ms[i] (-1 for a
 * candidate the state rejects).  The current buffer and the time level are
 * untouched; the other buffer is overwritten.  The fastest candidate is set
 * (as by mp_set_fusion and mp_set_tile) and its index stored in *best.
 * Synchronises ``stream``.  Errors: MP_E_NULLPTR, MP_E_UNBOUND, MP_E_PARAM
 * (ncand < 1, reps < 1 or no valid candidate), MP_E_HIP. */
int mp_tune_candidates(const mp_state* st, int32_t* cand, int cap);
int mp_tune(mp_state* st, const int32_t* cand, int ncand, int reps, double* ms, int* best,
            void* stream);

/* Steps per launch of the 2D step kernels (single grid or batch): 1 or 2
 * (the default for 2D states; 3D states take 1).
 * With 2, one launch reads a state, computes the next one in registers and
 * writes the one after it, so the state crosses HBM once per two steps
 * (temporal blocking); every cell gets the same arithmetic, and results are
 * bitwise those of two single steps.  Errors: MP_E_PARAM for other values
 * and for 3D states. */
int mp_set_fusion(mp_state* st, int steps);
int mp_get_fusion(const mp_state* st, int* steps);

/* Anti-trapping current of Eq. jatr (Sec. 2.1) in the mu update of Eq.
 * Mu_explicit_temperature: on = 1 or 2 switches it on, 0 off (the default).  With
 * it, mu^{n+1} = mu^n + (dt div(M grad mu - j_at) - sum_a c^a dh_a) / chi, where
 * j_at = sum over the solid phases a (the liquid is the last phase) of
 * P (c^a - c^liq) dphi_a/dt n_a (-n_a . n_liq), n = grad phi / |grad phi| of
 * phi^n, P = eps / (2 sqrt 2) for the multi-well potential and
 * pi eps phi (1 - h(phi)) / (4 sqrt(phi (1 - phi))) for the obstacle one.  On a
 * face: the normal gradient is the difference of its two cells, a tangential
 * one the mean of their central differences; dphi/dt = (phi^{n+1} - phi^n)/dt,
 * c^a(mu^n) and the prefactor's phi are means of the two cells; a unit normal
 * with |grad phi|^2 <= 1e-30 is zero.  mp_step then runs one step per launch
 * and ignores mp_set_fusion.  On a 2D grid or a batch with on = 1 the current
 * is formed inside the step kernel (the state is read once per step) and
 * mp_set_graph is honoured; with on = 2, and on a 3D grid, each step is
 * followed by a correction kernel that reads states n and n+1 and
 * mp_set_graph is ignored.  Both give the same bits, and a batched instance
 * the bits of the same instance stepped alone.  mp_adjoint returns
 * MP_E_STATE while it is on.  2D and 3D single grids and batches.  Host only
 * for a single grid; for a bound batch switching it on or off re-deals the
 * work list (a synchronous copy).  With the extended model (Bt, Ct, A01, D01,
 * tau_ab, MP_OBSTACLE_ACTIVE) the compositions of the current are those at each
 * row's temperature of time level n and the correction solves with the 2 x 2
 * susceptibility.  Errors: MP_E_NULLPTR, MP_E_PARAM (on not 0, 1 or 2),
 * MP_E_STATE (on = 2 for a batch; on != 0 for a state with a KKS instance). */
int mp_set_antitrapping(mp_state* st, int on);
int mp_get_antitrapping(const mp_state* st, int* on);

/* Replay steps as a HIP graph: chunk = steps per graph (even, >= 2), or 0 to
 * launch kernel by kernel (the default).  The graph is built explicitly (no
 * stream capture), so any stream works, the null stream included; it is
 * rebuilt after mp_bind or mp_set_tile.  Results are bitwise those of the
 * kernel-by-kernel path. */
int mp_set_graph(mp_state* st, int chunk);

/* Batched states (many independent 2D simulations stepped together by one
 * persistent kernel launch per step: an ensemble of uneven runs, which the
 * paper itself does not have; its nearest notion is a set of boxes).
 * Instance i has grid grids[i] (dim must be 2), nphases[i] phases, ncomp[i]
 * components and coefficients params[i], each validated as by mp_create
 * (including its own dt limit).  All instances share precision and
 * potential.  One state buffer holds every instance's state, each at a
 * 256-byte aligned offset (mp_instance_offset) in the single-state layout.
 * mp_step advances every instance by the same number of steps, each with its
 * own dt; mp_diagnostics_batch reduces each instance.  When one instance uses
 * the extended model (Bt, Ct, A01, D01, tau_ab, MP_OBSTACLE_ACTIVE) every
 * instance is stepped with the general kernels (bitwise as a single grid of
 * the extended model would be).  Errors: as mp_create, plus MP_E_PARAM for
 * ninst < 1, a 3D grid, or mixed precision/potential. */
int mp_create_batch(int ninst, const mp_grid* grids, const int* nphases, const int* ncomp,
                    const mp_params* params, mp_state** out);

/* Number of instances (1 for a state made by mp_create). */
int mp_instance_count(const mp_state* st, int* ninst);

/* Byte offset and size of instance i's state inside each state buffer. */
int mp_instance_offset(const mp_state* st, int i, size_t* offset_bytes, size_t* nbytes);

/* Per-instance diagnostics: out[i] for i < ninst (synchronises ``stream``).
 * Returns MP_E_NONFINITE (with out filled) if any instance holds NaN/Inf. */
int mp_diagnostics_batch(mp_state* st, mp_diag* out, void* stream);

/* Checkpointed forward run (single 2D or 3D state): before every chunk of
 * ``every`` steps the current state is copied into checkpoint slot c of
 * ckpt_buf (slot stride = mp_state_bytes rounded up to 256 bytes;
 * ceil(nsteps / every) slots), then the chunk is stepped as by mp_step.  The
 * checkpoints are the forward states at time levels n0, n0 + every, ... where
 * n0 is the time level on entry.  The adjoint's recomputation reproduces the
 * stepped states bit for bit from them. */
int mp_step_ckpt(mp_state* st, int64_t nsteps, int64_t every, void* ckpt_buf, void* stream);

/* Bytes of the caller-owned work buffer mp_adjoint needs for ``every``
 * (two cotangent buffers, the adjoint state, two segments of recomputed
 * states, per-block gradient partial sums); 0 for unsupported states. */
size_t mp_adjoint_work_bytes(const mp_state* st, int64_t every);

/* Discrete adjoint of nsteps steps recorded by mp_step_ckpt starting at time
 * level n0: the exact transpose of the explicit step of Sec. 2.1 (2D,
 * isotropic, multi-well, base model only; the obstacle projection is not
 * differentiable).  lam_final holds dL/ds at the final state (state layout);
 * lam_initial receives dL/ds at the initial state.  grad_theta (host, 10
 * doubles) receives dL/dtheta with theta = (gamma_01, gamma_02, gamma_12,
 * D[0][0], D[0][1], D[1][0], D[1][1], D[2][0], D[2][1], tau) and dt held
 * fixed.  Each segment between checkpoints is recomputed from its checkpoint
 * into the work buffer and swept backwards; the recomputation of the next
 * segment runs on a second stream (created on first use, kept until
 * mp_destroy) while the current one is swept.  Results do not depend on
 * ``every`` (bitwise).  Synchronises ``stream``.  Errors: MP_E_STATE (batched
 * state), MP_E_PARAM (3D, obstacle, anisotropy, the KKS variant, bad sizes or
 * alignment). */
int mp_adjoint(mp_state* st, const void* ckpt_buf, int64_t nsteps, int64_t every, int64_t n0,
               const void* lam_final, void* lam_initial, double* grad_theta, void* work,
               void* stream);

/* Moving frame (the SHIFT / Shiftj keys of Sec. 5, the moving box of the
 * directional-solidification runs): mp_front_row reduces the current state to
 * the highest row (y index) holding a cell whose liquid fraction (the last
 * phase) is below 1/2, or -1 (synchronises ``stream``).  mp_shift moves the
 * frame up by ``rows`` (0 <= rows <= ny): row j of the new current buffer is
 * row j + rows of the old one, the top ``rows`` rows are melt (liquid fraction
 * 1, mu_k = mu_melt[k] for k < K-1, host memory), and from then on row j stands
 * at y = (j + offset) dx in the temperature law, offset being the sum of all
 * shifts (returned in *offset when offset is not NULL).  One copy kernel on
 * ``stream``; the current buffer flips, the time level is unchanged.  In 3D the
 * shift is along y as well.  Checkpoints taken before a shift do not replay
 * across it.  Single grids only.  Errors: MP_E_NULLPTR, MP_E_UNBOUND,
 * MP_E_STATE (batched state), MP_E_PARAM (rows out of range), MP_E_HIP. */
int mp_front_row(mp_state* st, int64_t* row, void* stream);
int mp_shift(mp_state* st, int64_t rows, const double* mu_melt, int64_t* offset, void* stream);

/* Free host-side state (device buffers stay with the caller). NULL is a no-op. */
void mp_destroy(mp_state* st);

/* Message of the last failed call on this thread ("" if none). */
const char* mp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MPSTEP_MP_H */
