"""FP64 CPU oracle of the explicit grand-potential phase-field step.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark use this module.  It shares no code with the HIP path: it
is plain numpy, slow and written to be checked against MICROSIM
(arXiv 2404.01035) Sec. 2.1 by eye.  It also runs on complex arrays, which lets
the tests take complex-step derivatives of it.

What one step computes (forward Euler; the paper states only the continuous
equations, so this discrete scheme is the reading both implementations follow):

Phase fields, Eq. phi_eqn without the elastic term:
    tau eps dphi_a/dt = eps (div da/dgrad(phi_a) - da/dphi_a) - w_{,a}/eps - psi_{,a} - lambda
  * a = sum_{a<b} gamma_ab a_c(q_ab)^2 |q_ab|^2, q_ab = phi_a grad phi_b - phi_b grad phi_a
    (Eq. Eqn_a), evaluated on cell faces: on a face normal to axis n between
    cells L and R, phi_bar = (phi_L + phi_R)/2, g = (phi_R - phi_L)/dx and
    q_n = phi_bar_a g_b - phi_bar_b g_a.  For anisotropic pairs the tangential
    components use the mean of the two cells' central differences.
  * G_n = d(a_c^2 |q|^2)/dq_n; the face carries the flux
    F_a = sum_b gamma_ab G_n dq_n/dg_a and the source s_a = sum_b gamma_ab G_n dq_n/dphi_bar_a;
    a cell gets eps[sum_axes (F_hi - F_lo)/dx - (s_hi + s_lo)/2].
  * w: multi-well (Eq. Well) or double obstacle (Eq. Obstacle); psi = sum_b h_b psi^b
    with h from Eq. hphi and psi^b(mu, T) of a parabolic free energy (Sec. 3).
  * lambda = (1/N) sum_a R_a keeps sum_a phi_a fixed.  The obstacle variant
    clips to [0, 1] and renormalises after the update.

Diffusion potentials, Eq. Mu_explicit_temperature with j_at = 0:
    mu^{n+1} = mu^n + (dt div(M grad mu) - sum_a c^a(mu^n) [h_a(phi^{n+1}) - h_a(phi^n)]) / chi
  * M_k = sum_a D^a_k chi^a_k h_a(phi^n) per cell (Eq. Mass_conservation), face
    value the mean of the two cells; chi_k = sum_a h_a(phi^{n+1}) chi^a_k.
  * B^a is temperature independent, so the dT/dt term vanishes.

KKS variant (Sec. 2.2, ``p.model == "kks"``): the phase fields follow Eq. aceq,
    (1/M_phi) dphi_a/dt = (eps^2/2)(div da/dgrad(phi_a) - da/dphi_a) - g_{,a} - d/dphi_a[f - c.mu] - lambda
  with eps the gradient-energy coefficient of Eq. fe, the same a and face
  discretisation as above, g either of the form of Eq. Well (no 1/eps) or the
  sextic Eq. Well1 (``potential == "theta"``), and the driving force
  d/dphi_a[f - c.mu] = sum_b psi^b dh_b/dphi_a: with the equal-potential
  condition (Eq. eqmu) and the composition constraint (Eq. cint), f^b(c^b) -
  mu.c^b is the grand potential psi^b(mu) of the phase.  The diffusion
  potentials follow the linearised composition equation, which the paper states
  is Eq. Mu_explicit_temperature (the same update as above).

With the anti-trapping current of Eq. jatr (``step_antitrapping``, kept apart
from ``step``), the mu update divides dt div(M grad mu - j_at) - sum_a c^a dh_a
instead; ``antitrapping_faces`` states how the current is placed on faces.

Boundaries: periodic (wrap) or zero-flux (ghost = mirror of the edge cell),
per axis; corners by composition.  Temperature T(y, t) = T0 + G (y - y0 - V t)
with t = n dt and y = j dx.

Parity: every function here is pinned by tests against closed forms,
invariants or brute force (see the test modules named test_oracle_*).
"""
from __future__ import annotations

import numpy as np

PERIODIC = 0
NOFLUX = 1


# ----------------------------------------------------------------------------
# Grid helpers
# ----------------------------------------------------------------------------

def spatial_axes(p):
    """(array axis, boundary code) for x, y[, z]; arrays are laid out (field, [z,] y, x)."""
    ax = [(-1, p.bc[0]), (-2, p.bc[1])]
    if p.dim == 3:
        ax.append((-3, p.bc[2]))
    return ax


def pad(f, p):
    """One ghost layer on every spatial axis: wrap (periodic) or edge copy (zero flux)."""
    for a, bc in spatial_axes(p):
        n = f.shape[a]
        if bc == PERIODIC:
            lo, hi = np.take(f, [n - 1], axis=a), np.take(f, [0], axis=a)
        else:
            lo, hi = np.take(f, [0], axis=a), np.take(f, [n - 1], axis=a)
        f = np.concatenate([lo, f, hi], axis=a)
    return f


def _sub(F, nd, spec):
    """Slice of a padded array: interior (1:-1) on every spatial axis unless overridden."""
    idx = [slice(None)] * (F.ndim - nd) + [slice(1, -1)] * nd
    for a, s in spec.items():
        idx[F.ndim + a] = s
    return F[tuple(idx)]


def _along(F, a, s):
    """Slice s along (negative) axis a."""
    idx = [slice(None)] * F.ndim
    idx[F.ndim + a] = s
    return F[tuple(idx)]


# ----------------------------------------------------------------------------
# Point-wise model functions
# ----------------------------------------------------------------------------

def h(phi):
    """Interpolation functions h_a (Eq. hphi); phi has the phase index first."""
    N = phi.shape[0]
    out = []
    for a in range(N):
        others = [b for b in range(N) if b != a]
        cross = 0.0
        for i in range(len(others)):
            for j in range(i + 1, len(others)):
                cross = cross + phi[others[i]] * phi[others[j]]
        out.append(3.0 * phi[a] ** 2 - 2.0 * phi[a] ** 3 + 2.0 * phi[a] * cross)
    return np.stack(out)


def dh(phi):
    """dh[b][a] = dh_b / dphi_a, differentiated by hand from Eq. hphi."""
    N = phi.shape[0]
    rows = []
    for b in range(N):
        others = [g for g in range(N) if g != b]
        row = []
        for a in range(N):
            if a == b:
                cross = 0.0
                for i in range(len(others)):
                    for j in range(i + 1, len(others)):
                        cross = cross + phi[others[i]] * phi[others[j]]
                row.append(6.0 * phi[b] - 6.0 * phi[b] ** 2 + 2.0 * cross)
            else:
                rest = 0.0
                for g in others:
                    if g != a:
                        rest = rest + phi[g]
                row.append(2.0 * phi[b] * rest)
        rows.append(np.stack(row))
    return np.stack(rows)


def w(phi, p):
    """Potential w: multi-well (Eq. Well) or double obstacle inside [0,1] (Eq. Obstacle)."""
    N = phi.shape[0]
    out = 0.0
    for a in range(N):
        for b in range(a + 1, N):
            g = p.gamma[a][b]
            if p.potential == "well":
                out = out + 9.0 * g * phi[a] ** 2 * phi[b] ** 2
            else:
                out = out + 16.0 / np.pi ** 2 * g * phi[a] * phi[b]
    if N == 3:
        out = out + p.gamma3 * phi[0] * phi[1] * phi[2]
    return out


def dw(phi, p):
    """dw/dphi_a for both potentials, each unordered triple counted once."""
    N = phi.shape[0]
    out = []
    for a in range(N):
        acc = 0.0
        for b in range(N):
            if b == a:
                continue
            g = p.gamma[a][b]
            if p.potential == "well":
                acc = acc + 18.0 * g * phi[a] * phi[b] ** 2
            else:
                acc = acc + 16.0 / np.pi ** 2 * g * phi[b]
        if N == 3:
            prod = 1.0
            for b in range(N):
                if b != a:
                    prod = prod * phi[b]
            acc = acc + p.gamma3 * prod
        out.append(acc)
    return np.stack(out)


def kks(p):
    """The KKS variant of Sec. 2.2 (Eq. aceq for the phase fields)."""
    return getattr(p, "model", "gp") == "kks"


def g_theta(phi, p):
    """Sextic multi-well potential of Eq. Well1:
    sum_a Theta_a phi_a^2 (1 - phi_a)^2 + sum_{a<b} Theta_ab phi_a^2 phi_b^2
    + sum_{a<b<d} Theta_abd phi_a^2 phi_b^2 phi_d^2 (one triple for N = 3)."""
    N = phi.shape[0]
    out = 0.0
    for a in range(N):
        out = out + p.theta[a] * phi[a] ** 2 * (1.0 - phi[a]) ** 2
        for b in range(a + 1, N):
            out = out + p.theta_ab[a][b] * phi[a] ** 2 * phi[b] ** 2
    if N == 3:
        out = out + p.theta3 * phi[0] ** 2 * phi[1] ** 2 * phi[2] ** 2
    return out


def dg_theta(phi, p):
    """dg/dphi_a of Eq. Well1, differentiated by hand term by term."""
    N = phi.shape[0]
    out = []
    for a in range(N):
        acc = 2.0 * p.theta[a] * phi[a] * (1.0 - phi[a]) * (1.0 - 2.0 * phi[a])
        for b in range(N):
            if b != a:
                acc = acc + 2.0 * p.theta_ab[min(a, b)][max(a, b)] * phi[a] * phi[b] ** 2
        if N == 3:
            rest = 1.0
            for b in range(N):
                if b != a:
                    rest = rest * phi[b] ** 2
            acc = acc + 2.0 * p.theta3 * phi[a] * rest
        out.append(acc)
    return np.stack(out)


def is_obstacle(p):
    """Both obstacle variants use the potential of Eq. Obstacle."""
    return p.potential in ("obstacle", "obstacle_active")


def extended(p):
    """True when the parameters use temperature-dependent B or C, off-diagonal
    A or D, per-pair relaxation constants or the active-set obstacle."""
    N, K1 = p.nphases, p.nmu
    return bool(np.any(np.asarray(p.Bt)[:N, :K1] != 0.0) or np.any(np.asarray(p.Ct)[:N] != 0.0)
                or np.any(np.asarray(p.A01)[:N] != 0.0) or np.any(np.asarray(p.D01)[:N] != 0.0)
                or np.any(np.asarray(p.tau_ab)[:N, :N] != 0.0) or p.potential == "obstacle_active")


def hessian(p):
    """H^a_kj = d^2 f^a / (dc_k dc_j) of Eq. free_energy_density, read with i <= j:
    2 A^a_k on the diagonal and A^a_01 off it; shape (N, K-1, K-1)."""
    N, K1 = p.nphases, p.nmu
    H = np.zeros((N, K1, K1), dtype=np.result_type(np.asarray(p.A), np.asarray(p.A01)))
    for a in range(N):
        for k in range(K1):
            H[a, k, k] = 2.0 * p.A[a][k]
        if K1 == 2:
            H[a, 0, 1] = H[a, 1, 0] = p.A01[a]
    return H


def chi_matrix(p):
    """Susceptibilities dc^a/dmu = (H^a)^-1, shape (N, K-1, K-1) (a library inverse)."""
    return np.linalg.inv(hessian(p))


def chi_phase(p):
    """Diagonal susceptibility dc^a_k/dmu_k = 1/(2 A^a_k) (no off-diagonal A)."""
    if p.nmu == 2 and np.any(np.asarray(p.A01)[: p.nphases] != 0.0):
        raise ValueError("chi_phase: off-diagonal A; use chi_matrix")
    return 1.0 / (2.0 * np.asarray(p.A)[: p.nphases, : p.nmu])


def _t_dependent(p):
    return bool(np.any(np.asarray(p.Bt)[: p.nphases, : p.nmu] != 0.0))


def B_of_T(p, T):
    """B^a_k(T) = B^a_k + Bt^a_k (T - Te); shape (N, K-1) + shape of T."""
    T = np.asarray(T)
    return np.stack([np.stack([p.B[a][k] + p.Bt[a][k] * (T - p.Te) for k in range(p.nmu)])
                     for a in range(p.nphases)])


def C_of_T(p, T):
    """C^a(T) = C^a + s^a (T - Te) + Ct^a (T - Te)^2; shape (N,) + shape of T."""
    T = np.asarray(T)
    return np.stack([p.C[a] + p.s[a] * (T - p.Te) + p.Ct[a] * (T - p.Te) ** 2 for a in range(p.nphases)])


def c_phase(mu, p, T=None):
    """Phase compositions c^a(mu, T) = chi^a (mu - B^a(T)), the stationary point of
    f^a(c) - mu . c; shape (N, K-1, ...).  T may be omitted when B does not
    depend on temperature."""
    if T is None:
        if _t_dependent(p):
            raise ValueError("c_phase: B depends on T; pass T")
        T = p.Te
    chi = chi_matrix(p)
    Bm = B_of_T(p, T)
    out = []
    for a in range(p.nphases):
        comp = []
        for k in range(p.nmu):
            acc = 0.0
            for j in range(p.nmu):
                acc = acc + chi[a, k, j] * (mu[j] - Bm[a][j])
            comp.append(acc)
        out.append(np.stack(comp))
    return np.stack(out)


def free_energy(c, a, p, T=None):
    """f^a(c) = sum_k A^a_k c_k^2 + A^a_01 c_0 c_1 + sum_k B^a_k(T) c_k + C^a(T)
    (Eq. free_energy_density with V_m = 1, read with i <= j)."""
    if T is None:
        if _t_dependent(p) or np.any(np.asarray(p.Ct) != 0.0):
            raise ValueError("free_energy: coefficients depend on T; pass T")
        T = p.Te
    Bm = B_of_T(p, T)
    out = C_of_T(p, T)[a]
    for k in range(p.nmu):
        out = out + p.A[a][k] * c[k] ** 2 + Bm[a][k] * c[k]
    if p.nmu == 2:
        out = out + p.A01[a] * c[0] * c[1]
    return out


def psi_phase(mu, T, p):
    """Grand potentials psi^a(mu, T) = f^a(c^a(mu, T); T) - mu . c^a; shape (N, ...)."""
    ca = c_phase(mu, p, T)
    out = []
    for a in range(p.nphases):
        val = free_energy(ca[a], a, p, T)
        for k in range(p.nmu):
            val = val - mu[k] * ca[a][k]
        out.append(val)
    return np.stack(out)


def dc_dT(p):
    """(dc^a_k/dT) at fixed mu = -(chi^a Bt^a)_k; shape (N, K-1)."""
    chi = chi_matrix(p)
    return np.stack([-(chi[a] @ np.asarray(p.Bt[a][: p.nmu], dtype=np.float64)) for a in range(p.nphases)])


def diffusivity(p):
    """D^a as (K-1) x (K-1) matrices: D^a_kk on the diagonal, D^a_01 off it."""
    N, K1 = p.nphases, p.nmu
    D = np.zeros((N, K1, K1), dtype=np.result_type(np.asarray(p.D), np.asarray(p.D01)))
    for a in range(N):
        for k in range(K1):
            D[a, k, k] = p.D[a][k]
        if K1 == 2:
            D[a, 0, 1] = D[a, 1, 0] = p.D01[a]
    return D


def relaxation(phi, p):
    """tau of Eq. phi_eqn at every cell.  With per-pair constants tau_ab (the Tau
    key of Sec. 5) it is their weighted mean
        tau(phi) = sum_{a<b} tau_ab phi_a phi_b / sum_{a<b} phi_a phi_b,
    falling back to the single tau where the pair sum is <= 1e-30 (bulk);
    otherwise the single tau."""
    N = p.nphases
    pairs = [(a, b) for a in range(N) for b in range(a + 1, N)]
    if not any(p.tau_ab[a][b] != 0.0 for a, b in pairs):
        return p.tau + 0.0 * phi[0]
    num = 0.0 * phi[0]
    den = 0.0 * phi[0]
    for a, b in pairs:
        w = phi[a] * phi[b]
        num = num + p.tau_ab[a][b] * w
        den = den + w
    ok = np.real(den) > 1e-30
    return np.where(ok, num / np.where(ok, den, 1.0), p.tau)


def temperature(p, n, shape, y_origin=0):
    """T(y, t) = T0 + G (y - y0 - V t) with y = j dx and t = n dt, broadcast to ``shape``."""
    ny = shape[-2]
    y = (np.arange(ny) + y_origin) * p.dx
    t = n * p.dt
    T = p.T0 + p.G * (y - p.y0 - p.V * t)
    T = T.reshape((ny, 1))
    return np.broadcast_to(T, shape)


def G_normal(qn, qt, delta):
    """Normal component of d(a_c^2 |q|^2)/dq for the four-fold a_c of Sec. 2.1.

    a_c = 1 - delta (3 - 4 sum_i q_i^4 / |q|^4).  With m = q/|q| and
    S4 = sum_i m_i^4, the derivative is
    2 a_c^2 q_n + 32 delta a_c |q| (m_n^3 - m_n S4).  For |q|^2 <= 1e-30 the
    direction is undefined and the isotropic limit 2 (1 - 3 delta)^2 q_n is used.
    """
    Q2 = qn * qn
    for t in qt:
        Q2 = Q2 + t * t
    small = np.real(Q2) <= 1e-30
    Q2s = np.where(small, 1.0, Q2)
    rq = np.sqrt(Q2s)
    mn = qn / rq
    S4 = mn ** 4
    for t in qt:
        S4 = S4 + (t / rq) ** 4
    ac = 1.0 - delta * (3.0 - 4.0 * S4)
    full = 2.0 * ac * ac * qn + 32.0 * delta * ac * rq * (mn ** 3 - mn * S4)
    lim = 2.0 * (1.0 - 3.0 * delta) ** 2 * qn
    return np.where(small, lim, full)


# ----------------------------------------------------------------------------
# The step
# ----------------------------------------------------------------------------

def obstacle_clip(phin):
    """Projection of the obstacle step: Eq. Obstacle makes w infinite outside
    [0, 1], read here as clipping every phi_a of the forward-Euler update to
    [0, 1] and then dividing by the sum over the phases, so sum_a phi_a = 1
    again.  phin has the phase index first."""
    out = np.clip(phin, 0.0, 1.0)
    return out / out.sum(axis=0, keepdims=True)


def simplex_projection(y):
    """Projection of the active-set obstacle step: every cell's (y_a) goes to the
    nearest point (Euclidean) of the simplex {phi_a >= 0, sum_a phi_a = 1}.  The
    active set starts as all phases; the multiplier shift theta = (sum over the
    active set of y - 1) / (its size) is subtracted from the active phases, and
    phases that come out negative leave the set (set to 0) until none does.
    In the terms of Eq. phi_eqn: lambda is the mean of the right-hand sides over
    the phases that stay present, plus the share of the mass of the phases that
    left.  y has the phase index first."""
    N = y.shape[0]
    active = np.ones(np.shape(y), dtype=bool)
    x = y
    for _ in range(N):
        cnt = active.sum(axis=0)
        theta = (np.where(active, y, 0.0).sum(axis=0) - 1.0) / cnt
        x = np.where(active, y - theta, 0.0)
        neg = active & (np.real(x) < 0.0)
        if not neg.any():
            break
        active = active & ~neg
    return x


def _faces(Pphi, p):
    """Per axis: (F, s) face arrays of the gradient term, shape (N, ..., n_a + 1, ...)."""
    nd = p.dim
    N = p.nphases
    dx = p.dx
    axes = [a for a, _ in spatial_axes(p)]
    out = []
    for a in axes:
        L = _sub(Pphi, nd, {a: slice(0, -1)})
        R = _sub(Pphi, nd, {a: slice(1, None)})
        pb = 0.5 * (L + R)
        g = (R - L) / dx
        tang = []
        aniso = any(p.delta[i][j] != 0.0 for i in range(N) for j in range(i + 1, N))
        if aniso:
            for b in axes:
                if b == a:
                    continue
                tl = (_sub(Pphi, nd, {a: slice(0, -1), b: slice(2, None)})
                      - _sub(Pphi, nd, {a: slice(0, -1), b: slice(0, -2)})) / (2.0 * dx)
                tr = (_sub(Pphi, nd, {a: slice(1, None), b: slice(2, None)})
                      - _sub(Pphi, nd, {a: slice(1, None), b: slice(0, -2)})) / (2.0 * dx)
                tang.append(0.5 * (tl + tr))
        F = [0.0 * pb[0] for _ in range(N)]
        S = [0.0 * pb[0] for _ in range(N)]
        for i in range(N):
            for j in range(i + 1, N):
                qn = pb[i] * g[j] - pb[j] * g[i]
                if p.delta[i][j] != 0.0:
                    qt = [pb[i] * t[j] - pb[j] * t[i] for t in tang]
                    Gn = G_normal(qn, qt, p.delta[i][j])
                else:
                    Gn = 2.0 * qn
                gG = p.gamma[i][j] * Gn
                F[i] = F[i] - gG * pb[j]
                F[j] = F[j] + gG * pb[i]
                S[i] = S[i] + gG * g[j]
                S[j] = S[j] - gG * g[i]
        out.append((a, np.stack(F), np.stack(S)))
    return out


def _rhs_padded(Pphi, Pmu, n, p, y_origin=0):
    """R_a (before the Lagrange multiplier) on the interior of padded fields."""
    nd = p.dim
    phi = _sub(Pphi, nd, {})
    mu = _sub(Pmu, nd, {})
    grad = 0.0 * phi
    for a, F, S in _faces(Pphi, p):
        grad = grad + (_along(F, a, slice(1, None)) - _along(F, a, slice(0, -1))) / p.dx \
            - 0.5 * (_along(S, a, slice(1, None)) + _along(S, a, slice(0, -1)))
    T = temperature(p, n, phi.shape[1:], y_origin)
    psi = psi_phase(mu, T, p)
    dhm = dh(phi)
    dpsi = [sum(psi[b] * dhm[b][a] for b in range(p.nphases)) for a in range(p.nphases)]
    if kks(p):
        # Eq. aceq: gradient energy eps^2/2 a, potential g without a 1/eps
        dg = dg_theta(phi, p) if p.potential == "theta" else dw(phi, p)
        return 0.5 * p.eps ** 2 * grad - dg - np.stack(dpsi)
    return p.eps * grad - dw(phi, p) / p.eps - np.stack(dpsi)


def _step_padded(Pphi, Pmu, n, p, y_origin=0):
    """One forward-Euler step of (phi, mu) on the interior of padded fields."""
    nd = p.dim
    N, K1 = p.nphases, p.nmu
    phi = _sub(Pphi, nd, {})
    mu = _sub(Pmu, nd, {})
    # phase fields
    R = _rhs_padded(Pphi, Pmu, n, p, y_origin)
    lam = sum(R[a] for a in range(N)) / N
    if kks(p):
        phin = phi + p.dt * p.Mphi * (R - lam)
    else:
        phin = phi + p.dt * (R - lam) / (relaxation(phi, p) * p.eps)
    if p.potential == "obstacle":
        phin = obstacle_clip(phin)
    elif p.potential == "obstacle_active":
        phin = simplex_projection(phin)
    # diffusion potentials: M = sum_b h_b(phi^n) D^b chi^b per cell, face value
    # the mean of the two cells, J = M_face grad mu
    chi = chi_matrix(p)
    Dm = diffusivity(p)
    hP = h(Pphi)
    DC = np.stack([Dm[b] @ chi[b] for b in range(N)])
    div = [0.0 * mu[k] for k in range(K1)]
    for k in range(K1):
        for a, _ in spatial_axes(p):
            for jj in range(K1):
                M = sum(DC[b, k, jj] * hP[b] for b in range(N))[None]
                ML = _sub(M, nd, {a: slice(0, -1)})[0]
                MR = _sub(M, nd, {a: slice(1, None)})[0]
                muL = _sub(Pmu[jj:jj + 1], nd, {a: slice(0, -1)})[0]
                muR = _sub(Pmu[jj:jj + 1], nd, {a: slice(1, None)})[0]
                J = 0.5 * (ML + MR) * (muR - muL) / p.dx
                div[k] = div[k] + (_along(J, a, slice(1, None)) - _along(J, a, slice(0, -1))) / p.dx
    T0 = temperature(p, n, phi.shape[1:], y_origin)
    T1 = temperature(p, n + 1, phi.shape[1:], y_origin)
    h0 = h(phi)
    h1 = h(phin)
    ca = c_phase(mu, p, T0)
    dcdT = dc_dT(p)
    rhs = []
    for k in range(K1):
        src = sum(ca[b][k] * (h1[b] - h0[b]) for b in range(N))
        # the dT/dt term of Eq. Mu_explicit_temperature, at h(phi^{n+1})
        theta = sum(h1[b] * dcdT[b][k] for b in range(N)) * (T1 - T0)
        rhs.append(p.dt * div[k] - src - theta)
    # [sum_b h_b(phi^{n+1}) chi^b] dmu = rhs
    if K1 == 1:
        chik = sum(h1[b] * chi[b, 0, 0] for b in range(N))
        return phin, np.stack([mu[0] + rhs[0] / chik])
    chit = np.empty(phi.shape[1:] + (2, 2), dtype=np.result_type(h1, chi))
    for k in range(2):
        for jj in range(2):
            chit[..., k, jj] = sum(h1[b] * chi[b, k, jj] for b in range(N))
    rv = np.stack(rhs, axis=-1)[..., None]
    dmu = np.linalg.solve(chit, rv)[..., 0]
    return phin, np.stack([mu[k] + dmu[..., k] for k in range(2)])


def rhs_phi(phi, mu, n, p):
    """R_a of the phase-field equation before the Lagrange multiplier (full grid)."""
    return _rhs_padded(pad(phi, p), pad(mu, p), n, p)


def step(phi, mu, n, p, y_origin=0):
    """One step from time level n: returns (phi^{n+1}, mu^{n+1}).  y_origin: the
    frame's offset in rows (cell j sits at y = (j + y_origin) dx; see ``shift``)."""
    return _step_padded(pad(phi, p), pad(mu, p), n, p, y_origin)


def run(phi, mu, n0, nsteps, p, y_origin=0):
    """nsteps steps starting at time level n0."""
    for i in range(nsteps):
        phi, mu = step(phi, mu, n0 + i, p, y_origin)
    return phi, mu


def _ghost_index(lo, hi, n, bc):
    """Source indices of cells lo-1 .. hi along one axis with the ghost rule of ``pad``."""
    idx = np.arange(lo - 1, hi + 1)
    if bc == PERIODIC:
        return np.mod(idx, n)
    return np.clip(idx, 0, n - 1)


def step_window(phi, mu, n, p, lo, hi, y_origin=0):
    """One step evaluated only on the box lo <= index < hi (array order, spatial axes).

    Gathers the box plus a one-cell rim with the same ghost rule as ``pad`` and
    runs the padded step on it, so the result equals the same cells of ``step``
    while costing only the window.  ``lo``/``hi`` are tuples in array order
    ((z,) y, x).
    """
    nd = p.dim
    bcs = [bc for _, bc in spatial_axes(p)][::-1]  # array order
    shape = phi.shape[1:]
    ix = [_ghost_index(lo[i], hi[i], shape[i], bcs[i]) for i in range(nd)]
    grid = np.ix_(*ix)
    # promote (e.g. an FP32 state) so the window is stepped in FP64 or complex
    Pphi = np.asarray(phi[(slice(None),) + grid], dtype=np.result_type(phi, np.float64))
    Pmu = np.asarray(mu[(slice(None),) + grid], dtype=np.result_type(mu, np.float64))
    return _step_padded(Pphi, Pmu, n, p, y_origin=y_origin + lo[-2])


# ----------------------------------------------------------------------------
# Energy and diagnostics
# ----------------------------------------------------------------------------

def energy(phi, mu, n, p):
    """Discrete grand potential of the isotropic scheme (used as a brute-force pin).

    Omega_h = dx^d [ sum_faces eps sum_{a<b} gamma_ab q_n^2
                    + sum_cells (w(phi)/eps + sum_a h_a(phi) psi^a(mu, T)) ]
    (Eq. grand_eqn with a from Eq. Eqn_a and a_c = 1), each physical face once.
    """
    nd = p.dim
    N = p.nphases
    Pphi = pad(phi, p)
    Eg = 0.0
    for a, _ in spatial_axes(p):
        # faces 1..n of the padded set: each physical face once
        L = _along(_sub(Pphi, nd, {a: slice(0, -1)}), a, slice(1, None))
        R = _along(_sub(Pphi, nd, {a: slice(1, None)}), a, slice(1, None))
        pb = 0.5 * (L + R)
        g = (R - L) / p.dx
        for i in range(N):
            for j in range(i + 1, N):
                q = pb[i] * g[j] - pb[j] * g[i]
                Eg = Eg + np.sum(p.gamma[i][j] * q * q)
    T = temperature(p, n, phi.shape[1:])
    bulk = w(phi, p) / p.eps + np.sum(h(phi) * psi_phase(mu, T, p), axis=0)
    return p.dx ** nd * (p.eps * Eg + np.sum(bulk))


def composition(phi, mu, p, n=0, y_origin=0):
    """Mixture composition c_k = sum_a h_a(phi) c^a_k(mu, T) (the composition
    constraint of Sec. 2.1), T that of time level n."""
    hh = h(phi)
    ca = c_phase(mu, p, temperature(p, n, phi.shape[1:], y_origin))
    return np.stack([sum(hh[a] * ca[a][k] for a in range(p.nphases)) for k in range(p.nmu)])


def diagnostics(phi, mu, p, n=0, y_origin=0):
    """Reference values of the diagnostics reductions (plain FP64 sums) of the
    state at time level n; min_chi is the smallest diagonal entry
    sum_a h_a (chi^a)_kk."""
    vol = p.dx ** p.dim
    c = composition(phi, mu, p, n, y_origin)
    hh = h(phi)
    chi = chi_matrix(p)
    chik = np.stack([sum(hh[a] * chi[a, k, k] for a in range(p.nphases)) for k in range(p.nmu)])
    finite = np.isfinite(phi).all(axis=0) & np.isfinite(mu).all(axis=0)
    return {
        "max_sum_dev": float(np.max(np.abs(phi.sum(axis=0) - 1.0))),
        "mass": [float(np.sum(c[k]) * vol) for k in range(p.nmu)],
        "volume": [float(np.sum(phi[a]) * vol) for a in range(p.nphases)],
        "min_chi": [float(np.min(chik[k])) for k in range(p.nmu)],
        "nonfinite": int(np.size(finite) - np.count_nonzero(finite)),
    }


# ----------------------------------------------------------------------------
# Discrete adjoint (isotropic gradient term, multi-well potential)
# ----------------------------------------------------------------------------

def unpad_add(Pf, p):
    """Transpose of ``pad``: fold the ghost layer's values onto the cells it copies."""
    f = Pf
    for a, bc in reversed(spatial_axes(p)):
        n = f.shape[a] - 2
        core = _along(f, a, slice(1, -1)).copy()
        lo = _along(f, a, slice(0, 1))
        hi = _along(f, a, slice(n + 1, n + 2))
        first = [slice(None)] * core.ndim
        last = [slice(None)] * core.ndim
        first[core.ndim + a] = slice(0, 1)
        last[core.ndim + a] = slice(n - 1, n)
        if bc == PERIODIC:
            core[tuple(last)] += lo
            core[tuple(first)] += hi
        else:
            core[tuple(first)] += lo
            core[tuple(last)] += hi
        f = core
    return f


def _zpad_along(x, a):
    """Zero cell on both ends of axis a (cotangents of the ghost cells are zero)."""
    z = np.zeros_like(_along(x, a, slice(0, 1)))
    return np.concatenate([z, x, z], axis=a)


PAIRS = [(0, 1), (0, 2), (1, 2)]


def adjoint_step(phi, mu, n, p, lphi1, lmu1):
    """Transpose of one step: from dL/d(phi^{n+1}, mu^{n+1}) to dL/d(phi^n, mu^n).

    Also returns this step's contribution to the parameter gradient, a dict
    with 'gamma' (3 pairs: 01, 02, 12), 'D' (3 x 2, per phase and component)
    and 'tau'.  Written by hand, term by term, from the forward scheme of
    ``step``; only the isotropic multi-well variant is differentiable here.
    """
    if p.potential != "well" or kks(p):
        raise ValueError("adjoint: the obstacle projection and the KKS variant are not supported")
    if extended(p):
        raise ValueError("adjoint: temperature-dependent B/C, off-diagonal A/D and per-pair tau "
                         "are not supported")
    N, K1, nd = p.nphases, p.nmu, p.dim
    if any(p.delta[i][j] != 0.0 for i in range(N) for j in range(i + 1, N)):
        raise ValueError("adjoint: anisotropic gradient energy not supported")
    dx, eps, tau, dt = p.dx, p.eps, p.tau, p.dt
    A = np.asarray(p.A)
    Dm = np.asarray(p.D)
    chi = chi_phase(p)
    Pphi, Pmu = pad(phi, p), pad(mu, p)

    # ---- forward recomputation of the cell quantities ------------------------
    R = _rhs_padded(Pphi, Pmu, n, p)
    lam = sum(R[a] for a in range(N)) / N
    phin = phi + dt * (R - lam) / (tau * eps)
    hP = h(Pphi)
    div = [0.0 * mu[k] for k in range(K1)]
    M = [sum(Dm[b][k] * chi[b][k] * hP[b] for b in range(N))[None] for k in range(K1)]
    for k in range(K1):
        for a, _ in spatial_axes(p):
            ML = _sub(M[k], nd, {a: slice(0, -1)})[0]
            MR = _sub(M[k], nd, {a: slice(1, None)})[0]
            muL = _sub(Pmu[k:k + 1], nd, {a: slice(0, -1)})[0]
            muR = _sub(Pmu[k:k + 1], nd, {a: slice(1, None)})[0]
            J = 0.5 * (ML + MR) * (muR - muL) / dx
            div[k] = div[k] + (_along(J, a, slice(1, None)) - _along(J, a, slice(0, -1))) / dx
    h0, h1 = h(phi), h(phin)
    ca = c_phase(mu, p)
    T = temperature(p, n, phi.shape[1:])
    psi = psi_phase(mu, T, p)

    g_gamma = np.zeros(3)
    g_D = np.zeros((3, 2))

    # ---- mu update ------------------------------------------------------------
    lmu = [lmu1[k].copy() for k in range(K1)]
    lh1 = [0.0 * phi[0] for _ in range(N)]
    lh0 = [0.0 * phi[0] for _ in range(N)]
    ldiv = []
    for k in range(K1):
        src = sum(ca[b][k] * (h1[b] - h0[b]) for b in range(N))
        chik = sum(h1[b] * chi[b][k] for b in range(N))
        Q = dt * div[k] - src
        lQ = lmu1[k] / chik
        lchi = -lmu1[k] * Q / chik ** 2
        ldiv.append(dt * lQ)
        lsrc = -lQ
        for b in range(N):
            lh1[b] = lh1[b] + lsrc * ca[b][k] + lchi * chi[b][k]
            lh0[b] = lh0[b] - lsrc * ca[b][k]
            lmu[k] = lmu[k] + lsrc * (h1[b] - h0[b]) / (2.0 * A[b][k])   # through c^b_k(mu)

    # ---- phi update: phin = phi + dt (R - lam) / (tau eps) -----------------------
    dh1 = dh(phin)
    lphin = [lphi1[a] + sum(lh1[b] * dh1[b][a] for b in range(N)) for a in range(N)]
    dh0 = dh(phi)
    lphi = [lphin[a] + sum(lh0[b] * dh0[b][a] for b in range(N)) for a in range(N)]
    kk = dt / (tau * eps)
    lmean = sum(lphin) / N
    lR = [kk * (lphin[a] - lmean) for a in range(N)]
    g_tau = float(np.sum(sum(lphin[a] * (-(dt * (R[a] - lam)) / (tau ** 2 * eps)) for a in range(N))))

    # R_a = eps grad_a - dw_a / eps - sum_b psi_b dh_b/dphi_a
    lgrad = [eps * lR[a] for a in range(N)]
    # potential: dw_c = sum_{b != c} 18 g_cb phi_c phi_b^2 + g3 prod_{b != c} phi_b
    for c in range(N):
        for a in range(N):
            if a == c:
                d = sum(18.0 * p.gamma[c][b] * phi[b] ** 2 for b in range(N) if b != c)
            else:
                d = 36.0 * p.gamma[c][a] * phi[c] * phi[a]
                if N == 3:
                    d = d + p.gamma3 * phi[3 - a - c]
            lphi[a] = lphi[a] - lR[c] * d / eps
    for c in range(N):
        for b in range(N):
            if b != c:
                q = PAIRS.index((min(b, c), max(b, c)))
                g_gamma[q] += float(np.sum(-lR[c] / eps * 18.0 * phi[c] * phi[b] ** 2))
    # driving force: second derivatives of h (differentiated by hand from Eq. hphi)
    for c in range(N):
        for a in range(N):
            acc = 0.0
            for b in range(N):
                if N == 2:
                    d2 = (6.0 - 12.0 * phi[b]) if (a == b and c == b) else 0.0
                else:
                    if a == b and c == b:
                        d2 = 6.0 - 12.0 * phi[b]
                    elif a == c:
                        d2 = 0.0
                    elif a == b or c == b:
                        d2 = 2.0 * phi[3 - a - c]
                    else:
                        d2 = 2.0 * phi[b]
                acc = acc + psi[b] * d2
            lphi[a] = lphi[a] - lR[c] * acc
    lpsi = [-sum(lR[c] * dh0[b][c] for c in range(N)) for b in range(N)]
    for k in range(K1):
        for b in range(N):
            lmu[k] = lmu[k] - lpsi[b] * ca[b][k]   # dpsi_b/dmu_k = -c^b_k

    # ---- faces: gradient term and mu flux ------------------------------------
    lPphi = np.zeros_like(Pphi)
    lPmu = np.zeros_like(Pmu)
    lPM = [np.zeros_like(M[k]) for k in range(K1)]
    for a, _ in spatial_axes(p):
        sL = {a: slice(0, -1)}
        sR = {a: slice(1, None)}
        L = _sub(Pphi, nd, sL)
        Rf = _sub(Pphi, nd, sR)
        pb = 0.5 * (L + Rf)
        g = (Rf - L) / dx
        lgz = [_zpad_along(lgrad[c], a) for c in range(N)]
        lF = [(_along(lgz[c], a, slice(0, -1)) - _along(lgz[c], a, slice(1, None))) / dx for c in range(N)]
        lS = [-0.5 * (_along(lgz[c], a, slice(0, -1)) + _along(lgz[c], a, slice(1, None))) for c in range(N)]
        lpb = [0.0 * pb[0] for _ in range(N)]
        lg = [0.0 * pb[0] for _ in range(N)]
        for i in range(N):
            for j in range(i + 1, N):
                qn = pb[i] * g[j] - pb[j] * g[i]
                Gn = 2.0 * qn
                gG = p.gamma[i][j] * Gn
                lgG = -lF[i] * pb[j] + lF[j] * pb[i] + lS[i] * g[j] - lS[j] * g[i]
                lpb[j] = lpb[j] - lF[i] * gG
                lpb[i] = lpb[i] + lF[j] * gG
                lg[j] = lg[j] + lS[i] * gG
                lg[i] = lg[i] - lS[j] * gG
                g_gamma[PAIRS.index((i, j))] += float(np.sum(lgG * Gn))
                lqn = 2.0 * p.gamma[i][j] * lgG
                lpb[i] = lpb[i] + lqn * g[j]
                lg[j] = lg[j] + lqn * pb[i]
                lpb[j] = lpb[j] - lqn * g[i]
                lg[i] = lg[i] - lqn * pb[j]
        lL = np.stack([0.5 * lpb[c] - lg[c] / dx for c in range(N)])
        lRr = np.stack([0.5 * lpb[c] + lg[c] / dx for c in range(N)])
        _sub(lPphi, nd, sL)[...] += lL
        _sub(lPphi, nd, sR)[...] += lRr
        for k in range(K1):
            ML = _sub(M[k], nd, sL)[0]
            MR = _sub(M[k], nd, sR)[0]
            muL = _sub(Pmu[k:k + 1], nd, sL)[0]
            muR = _sub(Pmu[k:k + 1], nd, sR)[0]
            ldz = _zpad_along(ldiv[k], a)
            lJ = (_along(ldz, a, slice(0, -1)) - _along(ldz, a, slice(1, None))) / dx
            lMf = lJ * 0.5 * (muR - muL) / dx
            lmuf = lJ * 0.5 * (ML + MR) / dx
            _sub(lPM[k], nd, sL)[0] += lMf
            _sub(lPM[k], nd, sR)[0] += lMf
            _sub(lPmu[k:k + 1], nd, sL)[0] -= lmuf
            _sub(lPmu[k:k + 1], nd, sR)[0] += lmuf
    # cell mobility M_k = sum_b D_bk chi_bk h_b(phi) on the padded cells
    dhP = dh(Pphi)
    for k in range(K1):
        for b in range(N):
            g_D[b][k] += float(np.sum(lPM[k][0] * chi[b][k] * hP[b]))
            for a in range(N):
                lPphi[a] = lPphi[a] + lPM[k][0] * Dm[b][k] * chi[b][k] * dhP[b][a]
    lphi_faces = unpad_add(lPphi, p)
    lmu_faces = unpad_add(lPmu, p)
    lphi0 = np.stack(lphi) + lphi_faces
    lmu0 = np.stack(lmu) + lmu_faces
    return lphi0, lmu0, {"gamma": g_gamma, "D": g_D, "tau": g_tau}


def adjoint_run(phi0, mu0, n0, nsteps, p, lphiN, lmuN):
    """Adjoint of ``run``: stores every forward state (small grids only) and sweeps back."""
    states = [(phi0, mu0)]
    for i in range(nsteps):
        states.append(step(*states[-1], n0 + i, p))
    lphi, lmu = lphiN, lmuN
    tot = {"gamma": np.zeros(3), "D": np.zeros((3, 2)), "tau": 0.0}
    for i in reversed(range(nsteps)):
        lphi, lmu, g = adjoint_step(states[i][0], states[i][1], n0 + i, p, lphi, lmu)
        tot["gamma"] += g["gamma"]
        tot["D"] += g["D"]
        tot["tau"] += g["tau"]
    return lphi, lmu, tot


# ----------------------------------------------------------------------------
# Anti-trapping current (Eq. jatr).  Not part of ``step``: ``step_antitrapping``
# is the step with it.
# ----------------------------------------------------------------------------

AT_TINY = 1e-30  # |grad phi|^2 at or below this: the unit normal is taken as zero


def at_prefactor(phi0, p):
    """The scalar in front of (c^a - c^liq) dphi_a/dt n_a in Eq. jatr.

    Multi-well potential: eps / (2 sqrt 2).  Double obstacle:
    pi eps phi0 (1 - h(phi0)) / (4 sqrt(phi0 (1 - phi0))) with the two-phase
    h(phi0) = phi0^2 (3 - 2 phi0); it tends to 0 at phi0 = 0 and 1 and is taken
    as 0 outside (0, 1).
    """
    if not is_obstacle(p):
        return p.eps / (2.0 * np.sqrt(2.0)) + 0.0 * phi0
    inside = (phi0 > 0.0) & (phi0 < 1.0)
    f = np.where(inside, phi0, 0.5)
    val = np.pi * p.eps * f * (1.0 - f * f * (3.0 - 2.0 * f)) / (4.0 * np.sqrt(f * (1.0 - f)))
    return np.where(inside, val, 0.0)


def _face_gradient(Pf, p, a):
    """Gradient of padded fields on the faces normal to axis a, one array per
    spatial axis in ``spatial_axes`` order: the normal component is the
    difference of the two cells, a tangential one the mean of the two cells'
    central differences (the same stencil as the anisotropic face term)."""
    nd = p.dim
    comps = []
    for b, _ in spatial_axes(p):
        if b == a:
            comps.append((_sub(Pf, nd, {a: slice(1, None)}) - _sub(Pf, nd, {a: slice(0, -1)})) / p.dx)
        else:
            tl = (_sub(Pf, nd, {a: slice(0, -1), b: slice(2, None)})
                  - _sub(Pf, nd, {a: slice(0, -1), b: slice(0, -2)})) / (2.0 * p.dx)
            tr = (_sub(Pf, nd, {a: slice(1, None), b: slice(2, None)})
                  - _sub(Pf, nd, {a: slice(1, None), b: slice(0, -2)})) / (2.0 * p.dx)
            comps.append(0.5 * (tl + tr))
    return comps


def antitrapping_faces(phi, phin, mu, p, n=0, y_origin=0, T=None):
    """Per axis a: (a, j) with j the normal component of j_at on the faces normal
    to a, shape (K-1, ..., n_a + 1, ...).

    Eq. jatr summed over the solid phases (the liquid is the last phase):
        j_k = sum_{a < N-1} P(phi_a) (c^a_k - c^liq_k) dphi_a/dt n_a . e_axis (-n_a . n_liq),
    n = grad phi / |grad phi| from phi^n.  On a face, dphi_a/dt = (phi^{n+1} - phi^n)/dt,
    c^a(mu^n, T^n) and the prefactor's phi are means of the two cells (a ghost
    cell takes the c^a of the cell it stands for); the gradient is
    ``_face_gradient``.  T: temperature of phi's cells (default: that of time
    level n in the frame y_origin).
    """
    nd = p.dim
    N = p.nphases
    liq = N - 1
    Pphi, Pphin = pad(phi, p), pad(phin, p)
    if T is None:
        T = temperature(p, n, phi.shape[1:], y_origin)
    Pc = pad(c_phase(mu, p, T), p)
    out = []
    for a, _ in spatial_axes(p):
        def mean(F):
            return 0.5 * (_sub(F, nd, {a: slice(0, -1)}) + _sub(F, nd, {a: slice(1, None)}))

        grads = _face_gradient(Pphi, p, a)
        norm2 = sum(g * g for g in grads)
        ok = norm2 > AT_TINY
        inv = np.where(ok, 1.0 / np.sqrt(np.where(ok, norm2, 1.0)), 0.0)
        units = [g * inv for g in grads]
        normal = [i for i, (b, _) in enumerate(spatial_axes(p)) if b == a][0]
        rate = (mean(Pphin) - mean(Pphi)) / p.dt
        pbar = mean(Pphi)
        cbar = mean(Pc)
        j = [0.0 * pbar[0] for _ in range(p.nmu)]
        for al in range(N - 1):
            weight = -sum(u[al] * u[liq] for u in units)
            common = at_prefactor(pbar[al], p) * rate[al] * units[normal][al] * weight
            for k in range(p.nmu):
                j[k] = j[k] + common * (cbar[al][k] - cbar[liq][k])
        out.append((a, np.stack(j)))
    return out


def _correct_mu(mun, phin, div, p):
    """mu^{n+1} - dt chi(phi^{n+1})^-1 div j_at, chi = sum_b h_b chi^b."""
    chi = chi_matrix(p)
    h1 = h(phin)
    N, K1 = p.nphases, p.nmu
    if K1 == 1:
        chik = sum(h1[b] * chi[b, 0, 0] for b in range(N))
        return np.stack([mun[0] - p.dt * div[0] / chik])
    chit = np.empty(phin.shape[1:] + (2, 2), dtype=np.result_type(h1, chi))
    for k in range(2):
        for jj in range(2):
            chit[..., k, jj] = sum(h1[b] * chi[b, k, jj] for b in range(N))
    d = np.linalg.solve(chit, np.stack([p.dt * div[0], p.dt * div[1]], axis=-1)[..., None])[..., 0]
    return np.stack([mun[k] - d[..., k] for k in range(2)])


def step_antitrapping(phi, mu, n, p, y_origin=0):
    """One step with the anti-trapping current in Eq. Mu_explicit_temperature:
        mu^{n+1} = mu^n + chi^-1 (dt div(M grad mu - j_at) - sum_a c^a(mu^n) [h_a(phi^{n+1}) - h_a(phi^n)] - Theta).
    phi^{n+1} and the rest of mu^{n+1} are those of ``step``; j_at is
    ``antitrapping_faces`` of (phi^n, phi^{n+1}, mu^n)."""
    if kks(p):
        raise ValueError("anti-trapping current: defined here for the grand-potential model only")
    phin, mun = step(phi, mu, n, p, y_origin)
    div = [0.0 * mu[k] for k in range(p.nmu)]
    for a, j in antitrapping_faces(phi, phin, mu, p, n, y_origin):
        for k in range(p.nmu):
            div[k] = div[k] + (_along(j[k], a, slice(1, None)) - _along(j[k], a, slice(0, -1))) / p.dx
    return phin, _correct_mu(mun, phin, div, p)


def _runs(idx):
    """Maximal stretches of consecutive source indices: (position, first, last + 1)."""
    out = []
    start = 0
    for k in range(1, len(idx) + 1):
        if k == len(idx) or idx[k] != idx[k - 1] + 1:
            out.append((start, int(idx[start]), int(idx[k - 1]) + 1))
            start = k
    return out


def step_antitrapping_window(phi, mu, n, p, lo, hi, y_origin=0):
    """``step_antitrapping`` evaluated only on the box lo <= index < hi (array order).

    The current of a box cell needs phi^{n+1} of its face neighbours: the box
    and a one-cell rim, each rim cell being, by the ghost rule of ``pad``, the
    grid cell it stands for.  Their phi^{n+1} and plain mu^{n+1} come from
    ``step_window`` over the stretches of consecutive grid cells the rim maps
    to; the current is then evaluated on that patch, whose own outer ghosts
    reach only faces the box does not use.
    """
    import itertools

    if kks(p):
        raise ValueError("anti-trapping current: defined here for the grand-potential model only")
    nd = p.dim
    bcs = [bc for _, bc in spatial_axes(p)][::-1]  # array order
    shape = phi.shape[1:]
    ix = [_ghost_index(lo[i], hi[i], shape[i], bcs[i]) for i in range(nd)]
    grid = np.ix_(*ix)
    dt_ = np.result_type(phi, np.float64)
    Pphi = np.asarray(phi[(slice(None),) + grid], dtype=dt_)
    Pmu = np.asarray(mu[(slice(None),) + grid], dtype=np.result_type(mu, np.float64))
    Pphin = np.empty_like(Pphi)
    Pmun = np.empty_like(Pmu)
    for pieces in itertools.product(*[_runs(i) for i in ix]):
        wlo = tuple(r[1] for r in pieces)
        whi = tuple(r[2] for r in pieces)
        f, m = step_window(phi, mu, n, p, wlo, whi, y_origin)
        dst = (slice(None),) + tuple(slice(r[0], r[0] + r[2] - r[1]) for r in pieces)
        Pphin[dst] = f
        Pmun[dst] = m
    box = (slice(None),) + (slice(1, -1),) * nd
    # temperature of each patch cell: that of the grid row it stands for
    yrows = ix[-2].reshape((-1, 1) if nd == 2 else (1, -1, 1))
    Tp = np.broadcast_to(p.T0 + p.G * ((yrows + y_origin) * p.dx - p.y0 - p.V * (n * p.dt)), Pphi.shape[1:])
    div = 0.0
    for a, j in antitrapping_faces(Pphi, Pphin, Pmu, p, T=Tp):
        L = j.shape[a]  # faces along a: the patch's cells + 1; box cells sit at 1 .. L - 3
        hi_f = _sub(_along(j, a, slice(2, L - 1)), nd, {a: slice(None)})
        lo_f = _sub(_along(j, a, slice(1, L - 2)), nd, {a: slice(None)})
        div = div + (hi_f - lo_f) / p.dx
    phin = Pphin[box]
    mun = Pmun[box]
    return phin, _correct_mu(mun, phin, [div[k] for k in range(p.nmu)], p)


# ----------------------------------------------------------------------------
# Moving frame (the SHIFT / Shiftj keys of Sec. 5; the moving box of the
# directional-solidification examples): solid rows leave the domain at the
# bottom and melt of the original alloy composition enters at the top.
# ----------------------------------------------------------------------------

def front_row(phi):
    """Highest row index (y, the second-slowest array axis in 3D, the slowest in
    2D) holding a cell whose liquid fraction (the last phase) is below 1/2; -1
    if there is none."""
    liq = phi[-1]
    yax = liq.ndim - 2  # y is axis 0 of (ny, nx) and axis 1 of (nz, ny, nx)
    other = tuple(i for i in range(liq.ndim) if i != yax)
    rows = np.nonzero(np.any(np.real(liq) < 0.5, axis=other))[0]
    return int(rows[-1]) if rows.size else -1


def shift(phi, mu, s, mu_melt):
    """Shift the frame up by s >= 0 rows along y: row j takes row j + s, the top
    s rows become melt (liquid fraction 1, mu = mu_melt per component).  After
    it the grid's row j stands at y = (j + y_origin + s) dx, so the caller adds
    s to the frame offset it passes to ``step``."""
    nd = phi.ndim - 1
    yax = 1 if nd == 2 else 2
    ny = phi.shape[yax]
    s = int(s)
    if s < 0 or s > ny:
        raise ValueError("shift: s must lie in [0, ny]")
    keep = [slice(None)] * phi.ndim
    keep[yax] = slice(s, ny)
    melt_shape = list(phi.shape)
    melt_shape[yax] = s
    mphi = np.zeros(melt_shape, dtype=phi.dtype)
    mphi[-1] = 1.0
    mu_shape = list(mu.shape)
    mu_shape[yax] = s
    mmu = np.empty(mu_shape, dtype=mu.dtype)
    for k in range(mu.shape[0]):
        mmu[k] = mu_melt[k]
    return (np.concatenate([phi[tuple(keep)], mphi], axis=yax),
            np.concatenate([mu[tuple(keep)], mmu], axis=yax))
