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


def chi_phase(p):
    """Susceptibility dc^a_k/dmu_k = 1/(2 A^a_k) of the diagonal parabolic free energy."""
    return 1.0 / (2.0 * np.asarray(p.A)[: p.nphases, : p.nmu])


def c_phase(mu, p):
    """Phase compositions c^a_k(mu) = (mu_k - B^a_k) / (2 A^a_k); shape (N, K-1, ...)."""
    A = np.asarray(p.A)
    B = np.asarray(p.B)
    return np.stack([np.stack([(mu[k] - B[a][k]) / (2.0 * A[a][k]) for k in range(p.nmu)])
                     for a in range(p.nphases)])


def free_energy(c, a, p):
    """f^a(c) = sum_k A^a_k c_k^2 + B^a_k c_k + C^a (Eq. free_energy_density, V_m = 1)."""
    out = p.C[a]
    for k in range(p.nmu):
        out = out + p.A[a][k] * c[k] ** 2 + p.B[a][k] * c[k]
    return out


def psi_phase(mu, T, p):
    """Grand potentials psi^a(mu, T) = f^a(c^a) - mu . c^a plus s^a (T - Te); shape (N, ...)."""
    ca = c_phase(mu, p)
    out = []
    for a in range(p.nphases):
        val = free_energy(ca[a], a, p)
        for k in range(p.nmu):
            val = val - mu[k] * ca[a][k]
        out.append(val + p.s[a] * (T - p.Te))
    return np.stack(out)


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
    return p.eps * grad - dw(phi, p) / p.eps - np.stack(dpsi)


def _step_padded(Pphi, Pmu, n, p, y_origin=0):
    """One forward-Euler step of (phi, mu) on the interior of padded fields."""
    nd = p.dim
    N = p.nphases
    phi = _sub(Pphi, nd, {})
    mu = _sub(Pmu, nd, {})
    # phase fields
    R = _rhs_padded(Pphi, Pmu, n, p, y_origin)
    lam = sum(R[a] for a in range(N)) / N
    phin = phi + p.dt * (R - lam) / (p.tau * p.eps)
    if p.potential == "obstacle":
        phin = obstacle_clip(phin)
    # diffusion potentials
    chi = chi_phase(p)
    D = np.asarray(p.D)[:N, : p.nmu]
    hP = h(Pphi)
    div = [0.0 * mu[k] for k in range(p.nmu)]
    for k in range(p.nmu):
        M = sum(D[b][k] * chi[b][k] * hP[b] for b in range(N))[None]
        for a, _ in spatial_axes(p):
            ML = _sub(M, nd, {a: slice(0, -1)})[0]
            MR = _sub(M, nd, {a: slice(1, None)})[0]
            muL = _sub(Pmu[k:k + 1], nd, {a: slice(0, -1)})[0]
            muR = _sub(Pmu[k:k + 1], nd, {a: slice(1, None)})[0]
            J = 0.5 * (ML + MR) * (muR - muL) / p.dx
            div[k] = div[k] + (_along(J, a, slice(1, None)) - _along(J, a, slice(0, -1))) / p.dx
    h0 = h(phi)
    h1 = h(phin)
    ca = c_phase(mu, p)
    mun = []
    for k in range(p.nmu):
        src = sum(ca[b][k] * (h1[b] - h0[b]) for b in range(N))
        chik = sum(h1[b] * chi[b][k] for b in range(N))
        mun.append(mu[k] + (p.dt * div[k] - src) / chik)
    return phin, np.stack(mun)


def rhs_phi(phi, mu, n, p):
    """R_a of the phase-field equation before the Lagrange multiplier (full grid)."""
    return _rhs_padded(pad(phi, p), pad(mu, p), n, p)


def step(phi, mu, n, p):
    """One step from time level n: returns (phi^{n+1}, mu^{n+1})."""
    return _step_padded(pad(phi, p), pad(mu, p), n, p)


def run(phi, mu, n0, nsteps, p):
    """nsteps steps starting at time level n0."""
    for i in range(nsteps):
        phi, mu = step(phi, mu, n0 + i, p)
    return phi, mu


def _ghost_index(lo, hi, n, bc):
    """Source indices of cells lo-1 .. hi along one axis with the ghost rule of ``pad``."""
    idx = np.arange(lo - 1, hi + 1)
    if bc == PERIODIC:
        return np.mod(idx, n)
    return np.clip(idx, 0, n - 1)


def step_window(phi, mu, n, p, lo, hi):
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
    return _step_padded(Pphi, Pmu, n, p, y_origin=lo[-2])


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


def composition(phi, mu, p):
    """Mixture composition c_k = sum_a h_a(phi) c^a_k(mu) (the composition constraint of Sec. 2.1)."""
    hh = h(phi)
    ca = c_phase(mu, p)
    return np.stack([sum(hh[a] * ca[a][k] for a in range(p.nphases)) for k in range(p.nmu)])


def diagnostics(phi, mu, p):
    """Reference values of the diagnostics reductions (plain FP64 sums)."""
    vol = p.dx ** p.dim
    c = composition(phi, mu, p)
    hh = h(phi)
    chi = chi_phase(p)
    chik = np.stack([sum(hh[a] * chi[a][k] for a in range(p.nphases)) for k in range(p.nmu)])
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
    if p.potential != "well":
        raise ValueError("adjoint: the obstacle projection is not differentiable")
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
    if p.potential != "obstacle":
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


def antitrapping_faces(phi, phin, mu, p):
    """Per axis a: (a, j) with j the normal component of j_at on the faces normal
    to a, shape (K-1, ..., n_a + 1, ...).

    Eq. jatr summed over the solid phases (the liquid is the last phase):
        j_k = sum_{a < N-1} P(phi_a) (c^a_k - c^liq_k) dphi_a/dt n_a . e_axis (-n_a . n_liq),
    n = grad phi / |grad phi| from phi^n.  On a face, dphi_a/dt = (phi^{n+1} - phi^n)/dt,
    c^a(mu^n) and the prefactor's phi are means of the two cells; the gradient
    is ``_face_gradient``.
    """
    nd = p.dim
    N = p.nphases
    liq = N - 1
    Pphi, Pphin, Pmu = pad(phi, p), pad(phin, p), pad(mu, p)
    Pc = c_phase(Pmu, p)
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


def step_antitrapping(phi, mu, n, p):
    """One step with the anti-trapping current in Eq. Mu_explicit_temperature:
        mu^{n+1} = mu^n + (dt div(M grad mu - j_at) - sum_a c^a(mu^n) [h_a(phi^{n+1}) - h_a(phi^n)]) / chi.
    phi^{n+1} is that of ``step``; j_at is ``antitrapping_faces`` of (phi^n, phi^{n+1}, mu^n)."""
    phin, mun = step(phi, mu, n, p)
    chi = chi_phase(p)
    h1 = h(phin)
    out = []
    div = [0.0 * mu[k] for k in range(p.nmu)]
    for a, j in antitrapping_faces(phi, phin, mu, p):
        for k in range(p.nmu):
            div[k] = div[k] + (_along(j[k], a, slice(1, None)) - _along(j[k], a, slice(0, -1))) / p.dx
    for k in range(p.nmu):
        chik = sum(h1[b] * chi[b][k] for b in range(p.nphases))
        out.append(mun[k] - p.dt * div[k] / chik)
    return phin, np.stack(out)


def _runs(idx):
    """Maximal stretches of consecutive source indices: (position, first, last + 1)."""
    out = []
    start = 0
    for k in range(1, len(idx) + 1):
        if k == len(idx) or idx[k] != idx[k - 1] + 1:
            out.append((start, int(idx[start]), int(idx[k - 1]) + 1))
            start = k
    return out


def step_antitrapping_window(phi, mu, n, p, lo, hi):
    """``step_antitrapping`` evaluated only on the box lo <= index < hi (array order).

    The current of a box cell needs phi^{n+1} of its face neighbours: the box
    and a one-cell rim, each rim cell being, by the ghost rule of ``pad``, the
    grid cell it stands for.  Their phi^{n+1} and plain mu^{n+1} come from
    ``step_window`` over the stretches of consecutive grid cells the rim maps
    to; the current is then evaluated on that patch, whose own outer ghosts
    reach only faces the box does not use.
    """
    import itertools

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
        f, m = step_window(phi, mu, n, p, wlo, whi)
        dst = (slice(None),) + tuple(slice(r[0], r[0] + r[2] - r[1]) for r in pieces)
        Pphin[dst] = f
        Pmun[dst] = m
    box = (slice(None),) + (slice(1, -1),) * nd
    div = 0.0
    for a, j in antitrapping_faces(Pphi, Pphin, Pmu, p):
        L = j.shape[a]  # faces along a: the patch's cells + 1; box cells sit at 1 .. L - 3
        hi_f = _sub(_along(j, a, slice(2, L - 1)), nd, {a: slice(None)})
        lo_f = _sub(_along(j, a, slice(1, L - 2)), nd, {a: slice(None)})
        div = div + (hi_f - lo_f) / p.dx
    phin = Pphin[box]
    mun = Pmun[box]
    chi = chi_phase(p)
    h1 = h(phin)
    out = []
    for k in range(p.nmu):
        chik = sum(h1[b] * chi[b][k] for b in range(p.nphases))
        out.append(mun[k] - p.dt * div[k] / chik)
    return phin, np.stack(out)
