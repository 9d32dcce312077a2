"""Seeded synthetic workloads for the grand-potential phase-field step.

This module only builds inputs: parameter sets and initial fields.  It holds no
part of the time step itself, so both the HIP path and the FP64 reference
stepper can consume what it produces.

Parameter meaning follows the grand-potential model of MICROSIM
(arXiv 2404.01035, Sec. 2.1 and Sec. 3):

* ``gamma[a][b]``  interface energy of the a-b interface (Eq. Obstacle / Eq. Well)
* ``gamma3``       third-order coefficient gamma_abd (same equations, N = 3 only)
* ``delta[a][b]``  four-fold anisotropy strength delta_ab (anisotropy function a_c)
* ``eps``, ``tau`` interface width and relaxation constant (Eq. phi_eqn)
* ``A, B, C``      diagonal parabolic free-energy coefficients per phase and
                   independent component, f^a(c) = sum_k A_k c_k^2 + B_k c_k + C
                   (Eq. free_energy_density with V_m = 1)
* ``s``            slope of C^a with temperature, C^a(T) = C^a + s^a (T - Te) + Ct^a (T - Te)^2
* ``Bt``, ``Ct``   temperature dependence of the parabolic coefficients (Sec. 3: B and C
                   as functions of T from the slopes of the coexistence lines):
                   B^a_k(T) = B^a_k + Bt^a_k (T - Te); zero by default
* ``A01``          off-diagonal curvature A^a_01 of Eq. free_energy_density (i < j term,
                   K = 3 only): f^a gains A01 c_0 c_1; zero by default
* ``D``            diffusivity per phase and component (Eq. Mass_conservation); ``D01``
                   its symmetric off-diagonal entry D^a_01 = D^a_10 (K = 3), zero by default
* ``tau_ab``       relaxation constant per phase pair (the Tau key of Sec. 5); all zero
                   (the default) means the single ``tau`` everywhere
* ``potential``    "well" (Eq. Well), "obstacle" (Eq. Obstacle; clip-and-renormalise
                   projection) or "obstacle_active" (Eq. Obstacle with the Lagrange
                   multiplier over the active phases: projection onto the simplex)
* ``model``        "gp" (Sec. 2.1) or "kks": the KKS variant of Sec. 2.2, whose phase
                   fields follow Eq. aceq: ``eps`` is then the gradient-energy coefficient
                   of Eq. fe (the gradient term carries eps^2/2), ``Mphi`` the phase-field
                   mobility M_phi (``tau`` and ``tau_ab`` unused), and the potential g is
                   "well" (the form of Eq. Well without the 1/eps) or "theta" (Eq. Well1
                   with ``theta[a]`` = Theta_a, ``theta_ab[a][b]`` = Theta_ab and
                   ``theta3`` = Theta_abd); the diffusion potentials follow the same
                   linearised update as the grand-potential model
* ``Te``           temperature at which C^a is given (Equilibrium_temperature, Sec. 5)
* ``T0, G, V, y0`` frozen, translating temperature field
                   T(y, t) = T0 + G (y - y0 - V t) (the Tempgrady input of Sec. 5:
                   base temperature, gradient, offset, velocity)

Arrays use the layout of the C ABI: ``phi`` has shape ``(N, ny, nx)`` in 2D and
``(N, nz, ny, nx)`` in 3D, ``mu`` has shape ``(K-1, ...)`` likewise; x is the
fastest axis.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

BC_PERIODIC = 0
BC_NOFLUX = 1

MAX_PHASES = 3
MAX_MU = 2


def _z33():
    return np.zeros((MAX_PHASES, MAX_PHASES))


@dataclass
class Params:
    """One simulation: grid, model sizes and coefficients (all FP64 on the host)."""

    dim: int = 2
    n: tuple = (64, 64, 1)          # (nx, ny, nz); nz = 1 in 2D
    dx: float = 1.0
    bc: tuple = (BC_PERIODIC, BC_PERIODIC, BC_PERIODIC)
    nphases: int = 2                # N, the liquid is the last phase
    ncomp: int = 2                  # K, components; K - 1 independent mu fields
    precision: str = "f64"          # "f64" | "f32"
    potential: str = "well"         # "well" | "obstacle" | "obstacle_active" | "theta" (KKS)
    eps: float = 4.0
    tau: float = 1.0
    dt: float = 0.05
    gamma: np.ndarray = field(default_factory=_z33)
    gamma3: float = 0.0
    delta: np.ndarray = field(default_factory=_z33)
    A: np.ndarray = field(default_factory=lambda: np.ones((MAX_PHASES, MAX_MU)))
    B: np.ndarray = field(default_factory=lambda: np.zeros((MAX_PHASES, MAX_MU)))
    C: np.ndarray = field(default_factory=lambda: np.zeros(MAX_PHASES))
    s: np.ndarray = field(default_factory=lambda: np.zeros(MAX_PHASES))
    D: np.ndarray = field(default_factory=lambda: np.zeros((MAX_PHASES, MAX_MU)))
    Bt: np.ndarray = field(default_factory=lambda: np.zeros((MAX_PHASES, MAX_MU)))
    Ct: np.ndarray = field(default_factory=lambda: np.zeros(MAX_PHASES))
    A01: np.ndarray = field(default_factory=lambda: np.zeros(MAX_PHASES))
    D01: np.ndarray = field(default_factory=lambda: np.zeros(MAX_PHASES))
    tau_ab: np.ndarray = field(default_factory=_z33)
    model: str = "gp"               # "gp" | "kks"
    Mphi: float = 1.0               # KKS phase-field mobility
    theta: np.ndarray = field(default_factory=lambda: np.zeros(MAX_PHASES))
    theta_ab: np.ndarray = field(default_factory=_z33)
    theta3: float = 0.0
    Te: float = 1.0
    T0: float = 1.0
    G: float = 0.0
    V: float = 0.0
    y0: float = 0.0

    @property
    def nmu(self) -> int:
        return self.ncomp - 1

    @property
    def nfields(self) -> int:
        return self.nphases + self.nmu

    @property
    def spatial(self) -> tuple:
        nx, ny, nz = self.n
        return (nz, ny, nx) if self.dim == 3 else (ny, nx)

    @property
    def ncells(self) -> int:
        return int(np.prod(self.spatial))

    def copy(self, **kw) -> "Params":
        p = replace(self, **kw)
        for name in ("gamma", "delta", "A", "B", "C", "s", "D", "Bt", "Ct", "A01", "D01", "tau_ab", "theta",
                     "theta_ab"):
            if name not in kw:
                setattr(p, name, np.array(getattr(self, name), dtype=np.float64))
        return p


# ----------------------------------------------------------------------------
# Thermodynamic inputs
# ----------------------------------------------------------------------------

def parabolic_coefficients(A, ceq, liquid):
    """B and C of the parabolic free energies from curvatures and equilibrium compositions.

    Follows Eq. Coeff_B and Eq. Coeff_C (Sec. 3) for a diagonal A: with the
    liquid as reference (B^l = C^l = 0), each solid a gets
    B^a_j = 2 (A^l_j c^l_j - A^a_j c^a_j) and C^a = sum_j (A^a_j (c^a_j)^2 - A^l_j (c^l_j)^2),
    so that every solid is in equilibrium with the liquid at mu_j = 2 A^l_j c^l_j.
    The common linear term -mu_e . c is then subtracted from every phase (a pure
    gauge: it shifts mu by mu_e and leaves the physics unchanged), which puts the
    equilibrium point at mu = 0.  A and ceq have shape (N, K-1).
    """
    A = np.asarray(A, dtype=np.float64)
    ceq = np.asarray(ceq, dtype=np.float64)
    npha = A.shape[0]
    B = np.zeros_like(A)
    C = np.zeros(npha)
    for a in range(npha):
        if a == liquid:
            continue
        B[a] = 2.0 * (A[liquid] * ceq[liquid] - A[a] * ceq[a])
        C[a] = np.sum(A[a] * ceq[a] ** 2 - A[liquid] * ceq[liquid] ** 2)
    mu_e = 2.0 * A[liquid] * ceq[liquid]
    B = B - mu_e[None, :]
    return B, C


def hessians(A, A01=None):
    """Curvature matrices H^a = d^2 f^a / dc dc of Eq. free_energy_density read with
    i <= j: 2 A^a_k on the diagonal and A^a_01 off it; shape (N, K-1, K-1)."""
    A = np.asarray(A, dtype=np.float64)
    npha, K1 = A.shape
    H = np.zeros((npha, K1, K1))
    for a in range(npha):
        for k in range(K1):
            H[a, k, k] = 2.0 * A[a, k]
        if K1 == 2 and A01 is not None:
            H[a, 0, 1] = H[a, 1, 0] = float(A01[a])
    return H


def parabolic_coefficients_T(A, ceq, slopes, liquid, A01=None):
    """B(T), C(T) of the parabolic free energies from curvatures, equilibrium
    compositions at Te and the slopes of the coexistence lines (Sec. 3).

    The equilibrium compositions move linearly with temperature,
    c^a_eq(T) = ceq^a + (T - Te) / slopes^a (slopes = dT/dc per phase and
    component), and every solid a is put in equilibrium with the liquid at each T
    by Eq. Coeff_B and Eq. Coeff_C with the liquid as reference (B^l = C^l = 0):
    B^a = H^l c^l_eq - H^a c^a_eq (H of ``hessians``; the cross-term sign as the
    equal-mu condition gives it) and C^a = (c^a_eq H^a c^a_eq - c^l_eq H^l c^l_eq) / 2.
    B is then linear in T and C quadratic.  The common linear term -mu_e . c,
    mu_e = H^l ceq^l, is subtracted from every phase (a gauge: it shifts mu
    only), so all phases coexist at mu = 0 at Te.  Returns (B, Bt, C, s, Ct)
    with B^a(T) = B^a + Bt^a (T - Te) and C^a(T) = C^a + s^a (T - Te) + Ct^a (T - Te)^2.
    """
    A = np.asarray(A, dtype=np.float64)
    ceq = np.asarray(ceq, dtype=np.float64)
    u = 1.0 / np.asarray(slopes, dtype=np.float64)
    npha, K1 = A.shape
    H = hessians(A, A01)
    B = np.zeros((npha, K1))
    Bt = np.zeros((npha, K1))
    C = np.zeros(npha)
    s = np.zeros(npha)
    Ct = np.zeros(npha)
    l = liquid
    for a in range(npha):
        if a == l:
            continue
        B[a] = H[l] @ ceq[l] - H[a] @ ceq[a]
        Bt[a] = H[l] @ u[l] - H[a] @ u[a]
        C[a] = 0.5 * (ceq[a] @ H[a] @ ceq[a] - ceq[l] @ H[l] @ ceq[l])
        s[a] = u[a] @ H[a] @ ceq[a] - u[l] @ H[l] @ ceq[l]
        Ct[a] = 0.5 * (u[a] @ H[a] @ u[a] - u[l] @ H[l] @ u[l])
    mu_e = H[l] @ ceq[l]
    B = B - mu_e[None, :]
    return B, Bt, C, s, Ct


def _sym2_min_eig(a, b, c):
    """Smaller eigenvalue of the symmetric 2 x 2 matrix [[a, b], [b, c]]."""
    return 0.5 * (a + c) - math.sqrt(0.25 * (a - c) ** 2 + b * b)


def _norm2_2x2(m):
    """Spectral norm of a 2 x 2 matrix: the square root of the larger eigenvalue of m^T m."""
    a = m[0][0] * m[0][0] + m[1][0] * m[1][0]
    b = m[0][0] * m[0][1] + m[1][0] * m[1][1]
    c = m[0][1] * m[0][1] + m[1][1] * m[1][1]
    return math.sqrt(0.5 * (a + c) + math.sqrt(0.25 * (a - c) ** 2 + b * b))


def dt_limit(p: Params) -> float:
    """Explicit (forward Euler) stability limit used to size dt.

    Phase fields: the projected gradient term acts like diffusion with
    coefficient at most 2 gamma_max (N-1)/N / tau, raised by a margin of
    (1 + 20 delta_max) for the anisotropic stiffness.  Diffusion potentials: the
    mu equation is a diffusion with coefficient M/chi <= max_a(D^a chi^a) / min_a chi^a.
    The FTCS bound dx^2 / (2 d coefficient) applies to both.  With per-pair
    relaxation constants the smallest of them (and tau) counts.  With
    off-diagonal A or D (K = 3) the mu coefficient is the matrix chi^-1 M, whose
    eigenvalues are at most max_a |D^a chi^a|_2 / min_a lambda_min(chi^a)
    (sum_a h_a = 1, h_a >= 0 on the simplex).
    """
    N, K1, d = p.nphases, p.nmu, p.dim
    g = np.asarray(p.gamma)[:N, :N]
    dl = np.asarray(p.delta)[:N, :N]
    gmax = float(np.max(g[np.triu_indices(N, 1)]))
    dmax = float(np.max(np.abs(dl[np.triu_indices(N, 1)])))
    base = p.dx * p.dx / (2.0 * d)
    lim = math.inf
    tau = float(p.tau)
    tab = np.asarray(p.tau_ab)[:N, :N][np.triu_indices(N, 1)]
    if np.any(tab != 0.0):
        tau = min(tau, float(np.min(tab)))
    if p.model == "kks":
        # Eq. aceq: the gradient term's coefficient is M_phi eps^2/2 where the
        # grand-potential model has 1/tau; the potential's stiffness
        # max_a d^2 g/dphi_a^2 <= S bounds dt M_phi S <= 1 as well
        tau = 2.0 / (p.Mphi * p.eps ** 2)
        th = np.asarray(p.theta_ab)[:N, :N]
        if p.potential == "theta":
            S = max(2.0 * p.theta[a] + sum(2.0 * th[min(a, b), max(a, b)] for b in range(N) if b != a)
                    for a in range(N))
        else:
            S = max(sum(18.0 * g[min(a, b), max(a, b)] for b in range(N) if b != a) for a in range(N))
        if S > 0:
            lim = 1.0 / (p.Mphi * S)
    if gmax > 0:
        lim = min(lim, base * tau / (2.0 * gmax * (N - 1) / N * (1.0 + 20.0 * dmax)))
    Dm = np.asarray(p.D)[:N, :K1]
    if K1 == 2 and (np.any(np.asarray(p.A01)[:N] != 0.0) or np.any(np.asarray(p.D01)[:N] != 0.0)):
        chi = np.linalg.inv(hessians(np.asarray(p.A)[:N, :K1], np.asarray(p.A01)[:N]))
        lmin = min(_sym2_min_eig(chi[a, 0, 0], chi[a, 0, 1], chi[a, 1, 1]) for a in range(N))
        top = 0.0
        for a in range(N):
            Da = np.array([[Dm[a, 0], p.D01[a]], [p.D01[a], Dm[a, 1]]])
            top = max(top, _norm2_2x2(Da @ chi[a]))
        if top > 0:
            lim = min(lim, base * lmin / top)
        return lim
    chi = 1.0 / (2.0 * np.asarray(p.A)[:N, :K1])
    for k in range(K1):
        top = float(np.max(Dm[:, k] * chi[:, k]))
        if top > 0:
            lim = min(lim, base * float(np.min(chi[:, k])) / top)
    return lim


# ----------------------------------------------------------------------------
# Initial-condition building blocks (the FILL* shapes of Sec. 5, made diffuse)
# ----------------------------------------------------------------------------

def diffuse_step(dist, eps):
    """Solid fraction across a diffuse front: 1 inside (dist < 0), 0 outside.

    The tanh width 2 eps / 3 matches the planar multi-well profile, so a seed
    starts close to its relaxed shape instead of a sharp FILL* edge.
    """
    return 0.5 * (1.0 - np.tanh(3.0 * dist / (2.0 * eps)))


def grid_coords(p: Params):
    """Cell-centre coordinates (x, y[, z]) at integer multiples of dx, as broadcastable axes."""
    nx, ny, nz = p.n
    if p.dim == 3:
        return (np.arange(nx).reshape(1, 1, nx) * p.dx, np.arange(ny).reshape(1, ny, 1) * p.dx,
                np.arange(nz).reshape(nz, 1, 1) * p.dx)
    return np.arange(nx).reshape(1, nx) * p.dx, np.arange(ny).reshape(ny, 1) * p.dx


def fields_from_solid(p: Params, solid_frac, solid_phase_of_cell, mu_value=0.0):
    """Assemble phi (N, ...) and mu (K-1, ...) from a solid fraction field.

    ``solid_phase_of_cell`` gives, per cell, which solid phase (0..N-2) the solid
    fraction belongs to; the liquid (phase N-1) takes the rest.
    """
    N, K1 = p.nphases, p.nmu
    phi = np.zeros((N,) + p.spatial)
    for a in range(N - 1):
        phi[a] = np.where(solid_phase_of_cell == a, solid_frac, 0.0)
    phi[N - 1] = 1.0 - solid_frac
    mu = np.full((K1,) + p.spatial, float(mu_value))
    return phi, mu


# ----------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------

def binary_two_phase(dim=2, n=(64, 64, 1), bc=(0, 0, 0), precision="f64",
                     potential="well", delta=0.0, gamma=1.0, undercooling=0.0,
                     c_solid=0.2, c_liquid=0.8, A=1.0, D_solid=0.0, D_liquid=1.0,
                     eps=4.0, tau=1.0, dt_frac=0.2) -> Params:
    """Two phases (solid, liquid), one independent component."""
    p = Params(dim=dim, n=tuple(n), bc=tuple(bc), nphases=2, ncomp=2,
               precision=precision, potential=potential, eps=eps, tau=tau)
    p.gamma[0, 1] = p.gamma[1, 0] = gamma
    p.delta[0, 1] = p.delta[1, 0] = delta
    Am = np.full((2, 1), float(A))
    ceq = np.array([[c_solid], [c_liquid]])
    B, C = parabolic_coefficients(Am, ceq, liquid=1)
    p.A[:2, :1] = Am
    p.B[:2, :1] = B
    p.C[:2] = C
    p.s[:2] = (1.0, 0.0)
    p.D[:2, 0] = (D_solid, D_liquid)
    # uniform undercooling: T = Te - dT everywhere (no gradient)
    p.Te = 1.0
    p.T0 = 1.0 - float(undercooling)
    p.G, p.V, p.y0 = 0.0, 0.0, 0.0
    p.dt = dt_frac * dt_limit(p)
    return p


def kks_from(p: Params, eps_k=None, Mphi=None, potential="well", theta=None, theta_ab=None, theta3=0.0,
             dt_frac=0.2) -> Params:
    """The KKS variant (Sec. 2.2) of a parameter set: the same phases, free
    energies, diffusivities, boundaries and temperature law; gradient-energy
    coefficient eps_k (default 1.5 eps), mobility Mphi (default 2 / (tau eps_k^2),
    the grand-potential set's relaxation of the gradient term), potential
    "well" (Eq. Well's form with the same gamma) or "theta" (Eq. Well1; Theta_ab
    defaults to 9 gamma_ab), dt a fraction of the explicit limit."""
    eps_k = 1.5 * p.eps if eps_k is None else eps_k
    q = p.copy(model="kks", eps=float(eps_k), potential=potential, tau_ab=_z33())
    q.Mphi = 2.0 / (p.tau * eps_k ** 2) if Mphi is None else float(Mphi)
    N = p.nphases
    if theta is not None:
        q.theta[:N] = theta
    q.theta_ab[:] = 0.0
    for a in range(N):
        for b in range(a + 1, N):
            q.theta_ab[a, b] = q.theta_ab[b, a] = 9.0 * p.gamma[a][b] if theta_ab is None else theta_ab[a][b]
    q.theta3 = float(theta3)
    q.dt = dt_frac * dt_limit(q)
    return q


def config_c1(seed: int = 0):
    """2D 64x64 periodic, 2 phases, binary alloy, FP64; circular nucleus R=10 plus noise.

    f_a(c) = A (c - c_a)^2 with A = 1, c_solid = 0.2, c_liquid = 0.8; gamma = 1,
    eps = 4 dx, tau = 1, D = (0, 1), dt = 0.2 of the explicit limit.  Noise:
    U(-0.01, 0.01) on phi_solid (liquid takes 1 - phi_solid), then on mu, drawn
    in that order from numpy's default_rng(seed).
    """
    p = binary_two_phase(dim=2, n=(64, 64, 1), bc=(0, 0, 0))
    x, y = grid_coords(p)
    r = np.hypot(x - 32.0, y - 32.0)
    sol = diffuse_step(r - 10.0, p.eps)
    rng = np.random.default_rng(seed)
    sol = sol + rng.uniform(-0.01, 0.01, size=sol.shape)
    phi, mu = fields_from_solid(p, sol, np.zeros(sol.shape, dtype=int))
    mu = mu + rng.uniform(-0.01, 0.01, size=mu.shape)
    return p, phi, mu


def eutectic_params(n=(4096, 4096, 1), seed=1, precision="f64", G=1e-3, V=0.01,
                    y0=64.0, eps=4.0, tau=1.0, dt_frac=0.2) -> Params:
    """Three phases (alpha, beta, liquid), ternary (2 independent mu), directional growth.

    A ~ U[0.5, 2] and c_eq ~ U[0.1, 0.9] per phase and component (seeded),
    B and C from Eq. Coeff_B / Eq. Coeff_C against the liquid, so alpha, beta and
    liquid coexist at mu = 0 and T = Te.  Temperature T = Te + G (y - y0 - V t),
    x periodic, y no-flux, D = (0, 0, 1), s = (1, 1, 0).
    """
    rng = np.random.default_rng(seed)
    A = rng.uniform(0.5, 2.0, size=(3, 2))
    ceq = rng.uniform(0.1, 0.9, size=(3, 2))
    p = Params(dim=2, n=tuple(n), bc=(BC_PERIODIC, BC_NOFLUX, BC_PERIODIC),
               nphases=3, ncomp=3, precision=precision, eps=eps, tau=tau)
    for a in range(3):
        for b in range(3):
            if a != b:
                p.gamma[a, b] = 1.0
    B, C = parabolic_coefficients(A, ceq, liquid=2)
    p.A[:3, :2] = A
    p.B[:3, :2] = B
    p.C[:3] = C
    p.s[:3] = (1.0, 1.0, 0.0)
    p.D[2, :2] = 1.0
    p.Te, p.T0, p.G, p.V, p.y0 = 1.0, 1.0, G, V, y0
    p.dt = dt_frac * dt_limit(p)
    return p


def eutectic_initial(p: Params, slab=64, wmin=16, wmax=48, seed=1):
    """Bottom slab ``slab`` cells thick of alternating alpha/beta lamellae in melt at mu = 0.

    Lamella widths are integers drawn uniformly from [wmin, wmax] (the last one
    is cut at the domain edge); the slab top is diffuse (tanh across y = slab),
    lamella-lamella boundaries are sharp.
    """
    rng = np.random.default_rng(seed + 1000)
    nx = p.n[0]
    owner = np.zeros(nx, dtype=int)
    x0, k = 0, 0
    while x0 < nx:
        w = int(rng.integers(wmin, wmax + 1))
        owner[x0:x0 + w] = k % 2
        x0 += w
        k += 1
    x, y = grid_coords(p)
    sol = np.broadcast_to(diffuse_step(y - (slab - 0.5), p.eps), p.spatial)
    which = np.broadcast_to(owner[None, :], sol.shape)
    return fields_from_solid(p, sol, which)


def config_c2(precision="f64", n=(4096, 4096, 1), seed=1):
    """2D 4096x4096 directional eutectic solidification (3 phases, ternary)."""
    scale = n[0] / 4096.0
    p = eutectic_params(n=n, seed=seed, precision=precision,
                        y0=max(8.0, 64.0 * scale))
    slab = int(round(p.y0))
    wmin = max(4, int(round(16 * scale)))
    wmax = max(wmin + 2, int(round(48 * scale)))
    phi, mu = eutectic_initial(p, slab=slab, wmin=wmin, wmax=wmax, seed=seed)
    return p, phi, mu


def eutectic_slopes_params(n=(4096, 4096, 1), seed=1, precision="f64", G=1e-3, V=0.01, y0=64.0,
                           eps=4.0, tau=1.0, dt_frac=0.2) -> Params:
    """The directional eutectic with temperature-dependent parabolic coefficients.

    Curvatures and equilibrium compositions at Te are those of
    ``eutectic_params`` (same seed, same draws); the equilibrium compositions
    move with T along seeded coexistence-line slopes (Sec. 3), |slope| ~ U[2, 6]
    (dT per unit composition), so B and C depend on T (``parabolic_coefficients_T``)
    and the mu update carries the dT/dt term of Eq. Mu_explicit_temperature.
    Solid slopes take random signs; the liquid's are drawn until every solid is
    the stable phase below Te: at mu = 0 and Te, d(psi^a - psi^l)/dT =
    (c^a_eq - c^l_eq) . H^l (1 / slope^l), which must be positive.
    """
    p = eutectic_params(n=n, seed=seed, precision=precision, G=G, V=V, y0=y0, eps=eps, tau=tau,
                        dt_frac=dt_frac)
    rng = np.random.default_rng(seed)
    A = rng.uniform(0.5, 2.0, size=(3, 2))
    ceq = rng.uniform(0.1, 0.9, size=(3, 2))
    rs = np.random.default_rng(seed + 500)
    slopes = rs.uniform(2.0, 6.0, size=(3, 2)) * rs.choice([-1.0, 1.0], size=(3, 2))
    H = hessians(A)
    while True:
        u = 1.0 / slopes[2]
        if all((ceq[a] - ceq[2]) @ H[2] @ u > 0.0 for a in range(2)):
            break
        slopes[2] = rs.uniform(2.0, 6.0, size=2) * rs.choice([-1.0, 1.0], size=2)
    B, Bt, C, s, Ct = parabolic_coefficients_T(A, ceq, slopes, liquid=2)
    p.A[:3, :2], p.B[:3, :2], p.Bt[:3, :2] = A, B, Bt
    p.C[:3], p.s[:3], p.Ct[:3] = C, s, Ct
    p.dt = dt_frac * dt_limit(p)
    return p


def config_c2_slopes(precision="f64", n=(4096, 4096, 1), seed=1):
    """``config_c2`` with temperature-dependent coefficients (``eutectic_slopes_params``)."""
    scale = n[0] / 4096.0
    p = eutectic_slopes_params(n=n, seed=seed, precision=precision, y0=max(8.0, 64.0 * scale))
    slab = int(round(p.y0))
    wmin = max(4, int(round(16 * scale)))
    wmax = max(wmin + 2, int(round(48 * scale)))
    phi, mu = eutectic_initial(p, slab=slab, wmin=wmin, wmax=wmax, seed=seed)
    return p, phi, mu


def dendrite_params(n=(512, 512, 512), precision="f32", gamma0=0.5, delta=0.02,
                    undercooling=0.3, eps=4.0, dt_frac=0.2) -> Params:
    """3D binary dendrite: 2 phases, cubic anisotropy, no-flux on every face."""
    return binary_two_phase(dim=3, n=n, bc=(BC_NOFLUX,) * 3, precision=precision,
                            delta=delta, gamma=gamma0, undercooling=undercooling,
                            eps=eps, dt_frac=dt_frac)


def config_c3(precision="f32", n=(512, 512, 512), radius=8.0):
    """3D 512^3 octant dendrite seed (sphere of radius 8 at the mirrored corner)."""
    p = dendrite_params(n=n, precision=precision)
    x, y, z = grid_coords(p)
    # the mirror plane of the no-flux ghost lies half a cell before cell 0
    r = np.sqrt((x + 0.5) ** 2 + (y + 0.5) ** 2 + (z + 0.5) ** 2)
    sol = diffuse_step(r - radius, p.eps)
    phi, mu = fields_from_solid(p, sol, np.zeros(sol.shape, dtype=int))
    return p, phi, mu


def nuclei_initial(p: Params, centres, radii, phases, mu_value=0.0):
    """Solid nuclei (discs or spheres) in melt; overlapping seeds keep the larger fraction."""
    coords = grid_coords(p)
    sol = np.zeros(p.spatial)
    which = np.zeros(p.spatial, dtype=int)
    L = [p.n[i] * p.dx for i in range(p.dim)]
    for c, R, ph in zip(centres, radii, phases):
        d2 = np.zeros(p.spatial)
        for i in range(p.dim):
            dd = coords[i] - c[i]
            if p.bc[i] == BC_PERIODIC:  # nearest periodic image
                dd = dd - L[i] * np.round(dd / L[i])
            d2 = d2 + dd * dd
        f = diffuse_step(np.sqrt(d2) - R, p.eps)
        take = f > sol
        sol = np.where(take, f, sol)
        which = np.where(take, ph, which)
    return fields_from_solid(p, sol, which, mu_value=mu_value)


def random_multiphase(p: Params, seed: int, amp: float = 1.0):
    """Random phase fields on the simplex plus random mu: a harsh parity input.

    Used for one-step and few-step checks where large gradients everywhere
    exercise every term of the update.
    """
    rng = np.random.default_rng(seed)
    raw = rng.uniform(0.0, 1.0, size=(p.nphases,) + p.spatial)
    phi = raw / raw.sum(axis=0, keepdims=True)
    phi = (1 - amp) / p.nphases + amp * phi
    mu = rng.uniform(-0.05, 0.05, size=(p.nmu,) + p.spatial)
    return phi, mu


def random_instance(rng, nx, ny, N, K, precision="f32", undercooling=None, nuclei=None):
    """One batched-ensemble member: seeded sizes, coefficients and nuclei in melt.

    Interface energies gamma_ab ~ U[0.5, 2], liquid diffusivities log-uniform in
    [0.1, 10] (solids 0), parabolic coefficients drawn as in the eutectic
    workload, undercooling ~ U[0.1, 0.5], 1-16 nuclei of radius 10 at uniform
    positions, each of a random solid phase; periodic boundaries; dt = 0.2 of
    the instance's own explicit limit.
    """
    p = Params(dim=2, n=(int(nx), int(ny), 1), bc=(BC_PERIODIC, BC_PERIODIC, BC_PERIODIC),
               nphases=int(N), ncomp=int(K), precision=precision)
    for a in range(N):
        for b in range(a + 1, N):
            p.gamma[a, b] = p.gamma[b, a] = rng.uniform(0.5, 2.0)
    K1 = K - 1
    A = rng.uniform(0.5, 2.0, size=(N, K1))
    ceq = rng.uniform(0.1, 0.9, size=(N, K1))
    B, C = parabolic_coefficients(A, ceq, liquid=N - 1)
    p.A[:N, :K1], p.B[:N, :K1], p.C[:N] = A, B, C
    p.s[:N] = 1.0
    p.s[N - 1] = 0.0
    p.D[N - 1, :K1] = np.exp(rng.uniform(np.log(0.1), np.log(10.0), size=K1))
    dT = rng.uniform(0.1, 0.5) if undercooling is None else undercooling
    p.Te, p.T0 = 1.0, 1.0 - dT
    p.dt = 0.2 * dt_limit(p)
    count = int(rng.integers(1, 17)) if nuclei is None else nuclei
    centres = [(rng.uniform(0, nx), rng.uniform(0, ny)) for _ in range(count)]
    phases = [int(rng.integers(0, N - 1)) for _ in range(count)]
    phi, mu = nuclei_initial(p, centres, [10.0] * count, phases)
    return p, phi, mu


def config_c4(ninst=256, seed=4, precision="f32", side=(64, 1024)):
    """Batched ensemble: ninst independent 2D simulations of uneven size and parameters.

    Grid sides ~ U{64..1024} independently (non-square allowed), N ~ U{2,3},
    K - 1 ~ U{1,2}, per-instance coefficients and nuclei as in random_instance.
    Returns a list of (params, phi, mu).
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(ninst):
        nx = int(rng.integers(side[0], side[1] + 1))
        ny = int(rng.integers(side[0], side[1] + 1))
        N = int(rng.integers(2, 4))
        K = 1 + int(rng.integers(1, 3))
        out.append(random_instance(rng, nx, ny, N, K, precision=precision))
    return out


def theta_into(p: Params, theta) -> Params:
    """Copy of p with theta = (gamma_01, gamma_02, gamma_12, D^liq_1, D^liq_2, tau) written in."""
    q = p.copy()
    N = q.nphases
    for idx, (a, b) in enumerate([(0, 1), (0, 2), (1, 2)]):
        if b < N:
            q.gamma[a, b] = q.gamma[b, a] = float(theta[idx])
    for k in range(q.nmu):
        q.D[N - 1, k] = float(theta[3 + k])
    q.tau = float(theta[5])
    return q


def config_c5(n=512, seed=5, precision="f32", nuclei=8, undercooling=0.3):
    """Differentiable run: 2D n x n, 3 phases, ternary, periodic.

    Returns (p_nominal, phi0, mu0, theta_star).  theta_star = (three gamma_ab ~
    U[0.5, 2], two liquid diffusivities log-uniform in [0.1, 10], tau ~ U[0.5, 2])
    drives the target run; gradients are taken at the nominal theta = all ones.
    dt is one value for both (0.2 of the smaller of the two explicit limits), so
    that it stays fixed under perturbations of theta.
    """
    rng = np.random.default_rng(seed)
    p, phi, mu = random_instance(rng, n, n, 3, 3, precision=precision,
                                 undercooling=undercooling, nuclei=nuclei)
    theta_star = list(rng.uniform(0.5, 2.0, size=3)) + \
        list(np.exp(rng.uniform(np.log(0.1), np.log(10.0), size=2))) + [rng.uniform(0.5, 2.0)]
    p = theta_into(p, [1.0] * 6)
    p.dt = 0.2 * min(dt_limit(p), dt_limit(theta_into(p, theta_star)))
    return p, phi, mu, theta_star
