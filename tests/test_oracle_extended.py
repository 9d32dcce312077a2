"""Pins of the oracle's extended model: temperature-dependent parabolic
coefficients with the dT/dt term and the moving frame (Sec. 3, Eq.
Mu_explicit_temperature, the SHIFT key of Sec. 5), the obstacle potential with
the multiplier over the active phases and per-pair relaxation constants (Eq.
Obstacle, Eq. phi_eqn, the Tau key of Sec. 5), and off-diagonal curvatures and
diffusivities (Eq. free_energy_density, Eq. Mass_conservation).

Each test ties the oracle to something other than its own formulas: hand
values, brute-force minimisation and enumeration, exact discrete solutions,
conservation laws, the reduction of a three-phase system to a two-phase one,
and the same run on a taller domain without the frame shift.
"""
import itertools
import math

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import gp
from paper_2404_01035_amd import inputs


def params(N=3, K1=2, dim=2, n=(10, 8, 1), bc=(0, 0, 0), potential="well", seed=0, G=0.0, V=0.0,
           slopes=False, offdiag=False, tau_pairs=False):
    """Random coefficients of the extended model (each feature switched on by a flag)."""
    rng = np.random.default_rng(seed)
    p = inputs.Params(dim=dim, n=tuple(n), bc=tuple(bc), nphases=N, ncomp=K1 + 1, potential=potential,
                      eps=2.5, tau=1.3, dx=0.9)
    for a in range(N):
        for b in range(a + 1, N):
            p.gamma[a, b] = p.gamma[b, a] = rng.uniform(0.5, 2.0)
    A = rng.uniform(0.6, 2.0, size=(N, K1))
    ceq = rng.uniform(0.1, 0.9, size=(N, K1))
    A01 = rng.uniform(-0.4, 0.4, size=N) if (offdiag and K1 == 2) else np.zeros(N)
    sl = rng.uniform(2.0, 5.0, size=(N, K1)) * rng.choice([-1.0, 1.0], size=(N, K1)) if slopes \
        else np.full((N, K1), np.inf)
    B, Bt, C, s, Ct = inputs.parabolic_coefficients_T(A, ceq, sl, liquid=N - 1, A01=A01)
    p.A[:N, :K1], p.B[:N, :K1], p.C[:N] = A, B, C
    p.Bt[:N, :K1], p.s[:N], p.Ct[:N] = Bt, s, Ct
    p.A01[:N] = A01
    p.D[:N, :K1] = rng.uniform(0.1, 1.0, size=(N, K1))
    if offdiag and K1 == 2:
        # symmetric off-diagonal entries that keep every D^a positive definite
        p.D01[:N] = rng.uniform(-0.5, 0.5, size=N) * np.sqrt(p.D[:N, 0] * p.D[:N, 1])
    if tau_pairs:
        for a in range(N):
            for b in range(a + 1, N):
                p.tau_ab[a, b] = p.tau_ab[b, a] = rng.uniform(0.6, 2.0)
    p.Te, p.T0, p.G, p.V, p.y0 = 1.0, 0.93, G, V, 1.7
    p.dt = 0.2 * inputs.dt_limit(p)
    return p, ceq, sl


def simplex_state(p, seed=1):
    rng = np.random.default_rng(seed)
    phi = rng.uniform(0.0, 1.0, size=(p.nphases,) + p.spatial)
    phi = phi / phi.sum(axis=0, keepdims=True)
    mu = rng.uniform(-0.3, 0.3, size=(p.nmu,) + p.spatial)
    return phi, mu


# ----------------------------------------------------------------------------
# Thermodynamics: Eq. free_energy_density with cross terms, B(T), C(T)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("offdiag", [False, True])
@pytest.mark.parametrize("T", [0.8, 1.0, 1.15])
def test_coexistence_moves_along_the_slopes(offdiag, T):
    """At every T each solid coexists with the liquid (equal mu, equal psi) at the
    compositions c_eq + (T - Te) / slope read off the coexistence lines."""
    p, ceq, sl = params(N=3, K1=2, slopes=True, offdiag=offdiag)
    H = gp.hessian(p)
    cT = ceq + (T - p.Te) / sl
    # the liquid's mu at its coexistence composition, in the gauge mu_e(Te) = 0
    mu = (H[2] @ cT[2] - H[2] @ ceq[2]).reshape(2, 1)
    ca = gp.c_phase(mu, p, np.full((1,), T))[:, :, 0]
    assert np.allclose(ca, cT, rtol=0, atol=1e-13)
    psi = gp.psi_phase(mu, np.full((1,), T), p)[:, 0]
    assert np.ptp(psi) < 1e-13


@pytest.mark.parametrize("T", [0.85, 1.1])
def test_psi_is_legendre_transform_with_cross_terms(T):
    """psi^a(mu, T) = min_c f^a(c; T) - mu . c, minimised numerically (BFGS) with A^a_01 != 0."""
    p, _, _ = params(N=3, K1=2, slopes=True, offdiag=True)
    mu = np.array([[0.137], [-0.21]])
    psi = gp.psi_phase(mu, np.full((1,), T), p)[:, 0]
    Bm = gp.B_of_T(p, T)
    Cm = gp.C_of_T(p, T)
    for a in range(3):
        def obj(c):
            return (p.A[a][0] * c[0] ** 2 + p.A[a][1] * c[1] ** 2 + p.A01[a] * c[0] * c[1]
                    + Bm[a][0] * c[0] + Bm[a][1] * c[1] + Cm[a] - mu[0, 0] * c[0] - mu[1, 0] * c[1])
        r = minimize(obj, x0=np.zeros(2), method="BFGS", options={"gtol": 1e-12})
        assert abs(r.fun - psi[a]) < 1e-10
        assert np.allclose(r.x, gp.c_phase(mu, p, np.full((1,), T))[a, :, 0], atol=1e-5)


def test_free_energy_hand_values():
    """f = A0 c0^2 + A1 c1^2 + A01 c0 c1 + B0(T) c0 + B1(T) c1 + C(T), by hand."""
    p = inputs.Params(nphases=2, ncomp=3)
    p.A[0, :2] = (1.5, 0.5)
    p.A01[0] = 0.25
    p.B[0, :2] = (0.1, -0.2)
    p.Bt[0, :2] = (2.0, 1.0)
    p.C[0], p.s[0], p.Ct[0] = 0.3, 0.5, 4.0
    p.Te = 1.0
    c = np.array([0.4, 0.2])
    T = 1.1  # T - Te = 0.1: B = (0.3, -0.1), C = 0.3 + 0.05 + 0.04 = 0.39
    want = 1.5 * 0.16 + 0.5 * 0.04 + 0.25 * 0.08 + 0.3 * 0.4 - 0.1 * 0.2 + 0.39
    assert abs(gp.free_energy(c, 0, p, T) - want) < 1e-15


# ----------------------------------------------------------------------------
# The dT/dt term of Eq. Mu_explicit_temperature
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("K1,offdiag", [(1, False), (2, False), (2, True)])
def test_single_phase_under_cooling_closed_form(K1, offdiag):
    """A resting single phase keeps its composition while T(y, t) falls: mu stays
    uniform and moves by Bt (T^n - T^0) = -Bt G V n dt exactly, whatever y."""
    p, _, _ = params(N=2, K1=K1, n=(6, 7, 1), bc=(0, 1, 0), slopes=True, offdiag=offdiag, G=0.05, V=0.7)
    assert np.any(p.Bt[0, :K1] != 0.0)
    phi = np.stack([np.ones(p.spatial), np.zeros(p.spatial)])
    mu0 = np.array([0.03, -0.02][:K1])
    mu = np.stack([np.full(p.spatial, v) for v in mu0])
    nsteps = 25
    f, m = gp.run(phi, mu, 3, nsteps, p)
    assert np.array_equal(f, phi)
    for k in range(K1):
        want = mu0[k] - p.Bt[0, k] * p.G * p.V * nsteps * p.dt
        assert np.max(np.abs(m[k] - want)) < 1e-13


@pytest.mark.parametrize("bc", [(0, 0, 0), (0, 1, 0), (1, 1, 0)])
@pytest.mark.parametrize("offdiag", [False, True])
def test_solute_conserved_under_moving_gradient(bc, offdiag):
    """Composition at each time level (with that level's T) is conserved exactly by
    the flux form: the dT/dt term must sit at h(phi^{n+1}) with the sign that
    makes c^{n+1} - c^n = dt div J."""
    p, _, _ = params(N=3, K1=2, n=(9, 8, 1), bc=bc, slopes=True, offdiag=offdiag, G=0.04, V=0.9, seed=3)
    phi, mu = simplex_state(p, seed=4)
    m0 = np.array(gp.diagnostics(phi, mu, p, n=5)["mass"])
    f, m = gp.run(phi, mu, 5, 40, p)
    m1 = np.array(gp.diagnostics(f, m, p, n=45)["mass"])
    assert np.all(np.abs(m1 - m0) <= 1e-13 * np.maximum(1.0, np.abs(m0)))
    # the correction is not negligible: without it the mass would drift
    p0 = p.copy()
    p0.Bt[:] = 0.0
    drift = np.array(gp.diagnostics(f, m, p0, n=45)["mass"]) - np.array(gp.diagnostics(phi, mu, p0, n=5)["mass"])
    assert np.max(np.abs(drift)) > 1e-6


# ----------------------------------------------------------------------------
# Off-diagonal diffusivity and susceptibility
# ----------------------------------------------------------------------------

def test_matrix_diffusion_mode_decay():
    """A resting single phase: mu follows FTCS diffusion with the matrix
    E = chi^-1 D chi (similar to D), so v cos(2 pi m x / L), v an eigenvector of E
    with eigenvalue l, is multiplied by 1 - 4 l dt/dx^2 sum sin^2(pi m / n) each step."""
    p, _, _ = params(N=2, K1=2, n=(8, 6, 1), offdiag=True)
    chi = gp.chi_matrix(p)[1]
    D = gp.diffusivity(p)[1]
    E = np.linalg.inv(chi) @ D @ chi
    lam, vec = np.linalg.eig(E)
    x, y = inputs.grid_coords(p)
    mode = np.cos(2 * np.pi * 1 * x / (8 * p.dx)) * np.cos(2 * np.pi * 2 * y / (6 * p.dx))
    sin2 = math.sin(math.pi / 8) ** 2 + math.sin(2 * math.pi / 6) ** 2
    phi = np.stack([np.zeros(p.spatial), np.ones(p.spatial)])
    for i in range(2):
        v = np.real(vec[:, i])
        mu = 0.01 * np.stack([v[0] * mode, v[1] * mode])
        g = 1.0 - 4.0 * np.real(lam[i]) * p.dt / p.dx ** 2 * sin2
        f, m = gp.run(phi, mu, 0, 10, p)
        assert np.allclose(m, g ** 10 * mu, rtol=0, atol=1e-15)


def test_dt_limit_bounds_the_matrix_diffusion():
    """The limit's diffusion part is at most the true FTCS limit dx^2 / (2 d lambda_max(chi^-1 M))
    over mixtures sampled on the simplex."""
    p, _, _ = params(N=3, K1=2, offdiag=True, seed=7)
    p.gamma[:] = 0.0  # only the diffusion bound counts
    lim = inputs.dt_limit(p)
    chi = gp.chi_matrix(p)
    DC = np.stack([gp.diffusivity(p)[b] @ chi[b] for b in range(3)])
    rng = np.random.default_rng(2)
    for _ in range(500):
        ph = rng.dirichlet([0.5, 0.5, 0.5])
        hh = gp.h(ph.reshape(3, 1))[:, 0]
        E = np.linalg.inv(np.einsum("b,bij->ij", hh, chi)) @ np.einsum("b,bij->ij", hh, DC)
        lmax = float(np.max(np.real(np.linalg.eigvals(E))))
        assert lim <= p.dx ** 2 / (2 * p.dim * lmax) * (1 + 1e-12)


# ----------------------------------------------------------------------------
# Obstacle with the multiplier over the active phases
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("raw,want", [
    ((-0.1, 0.6, 0.5), (0.0, 0.55, 0.45)),   # theta = (1.1 - 1) / 2
    ((1.2, -0.1, -0.1), (1.0, 0.0, 0.0)),
    ((0.6, 0.6, -0.1), (0.5, 0.5, 0.0)),     # first pass keeps all three, second drops phase 2
    ((0.2, 0.3, 0.5), (0.2, 0.3, 0.5)),
    ((1.05, -0.05), (1.0, 0.0)),
    ((0.3, 0.7), (0.3, 0.7)),
])
def test_simplex_projection_hand_values(raw, want):
    got = gp.simplex_projection(np.array(raw, dtype=np.float64).reshape(-1, 1))
    assert np.allclose(got[:, 0], want, rtol=0, atol=1e-15)


def test_simplex_projection_is_the_nearest_point_by_enumeration():
    """Brute force: over every support set S, the candidate y_S - (sum_S y - 1)/|S|
    (zero elsewhere) that is feasible and nearest to y is the projection."""
    rng = np.random.default_rng(3)
    y = rng.uniform(-0.6, 1.4, size=(3, 400))
    y = y - (y.sum(axis=0) - 1.0) / 3.0 + rng.normal(scale=0.05, size=400)  # sums near 1
    got = gp.simplex_projection(y)
    for c in range(y.shape[1]):
        best, bd = None, np.inf
        for r in (1, 2, 3):
            for S in itertools.combinations(range(3), r):
                x = np.zeros(3)
                th = (sum(y[i, c] for i in S) - 1.0) / r
                for i in S:
                    x[i] = y[i, c] - th
                if np.all(x >= -1e-15):
                    d = float(np.sum((x - y[:, c]) ** 2))
                    if d < bd:
                        best, bd = x, d
        assert np.allclose(got[:, c], best, rtol=0, atol=1e-14)


def _binary_three_phase(potential, tau_pairs):
    """Three phases with a diffuse 0-1 interface along x and phase 2 absent; the
    matching two-phase system (phases 0, 1; tau = tau_01)."""
    p3, _, _ = params(N=3, K1=1, n=(24, 3, 1), bc=(1, 0, 0), potential=potential, tau_pairs=tau_pairs, seed=5)
    # the third phase must be unfavourable at the 0-1 interface: large gamma_02,
    # gamma_12 and a high grand potential of phase 2
    p3.gamma[0, 2] = p3.gamma[2, 0] = p3.gamma[1, 2] = p3.gamma[2, 1] = 2.5
    p3.gamma[0, 1] = p3.gamma[1, 0] = 0.8
    p3.C[2] += 0.3
    p3.dt = 0.2 * inputs.dt_limit(p3)
    p2 = inputs.Params(dim=2, n=p3.n, bc=p3.bc, nphases=2, ncomp=2, potential=potential, eps=p3.eps,
                       tau=p3.tau_ab[0, 1] if tau_pairs else p3.tau, dx=p3.dx, dt=p3.dt)
    p2.gamma[0, 1] = p2.gamma[1, 0] = p3.gamma[0, 1]
    for name in ("A", "B", "Bt"):
        getattr(p2, name)[:2, :1] = getattr(p3, name)[:2, :1]
    for name in ("C", "s", "Ct"):
        getattr(p2, name)[:2] = getattr(p3, name)[:2]
    p2.D[:2, :1] = p3.D[:2, :1]
    p2.Te, p2.T0, p2.G, p2.V, p2.y0 = p3.Te, p3.T0, p3.G, p3.V, p3.y0
    x, _ = inputs.grid_coords(p3)
    a = np.broadcast_to(0.5 * (1.0 + np.sin(np.clip((x - 11.7) * 4.0 / (np.pi * p3.eps), -np.pi / 2, np.pi / 2))),
                        p3.spatial)
    phi3 = np.stack([a, 1.0 - a, np.zeros(p3.spatial)])
    rng = np.random.default_rng(8)
    mu = rng.uniform(-0.05, 0.05, size=(1,) + p3.spatial)
    return p3, p2, phi3, mu


@pytest.mark.parametrize("tau_pairs", [False, True])
def test_active_set_binary_interface_is_the_two_phase_system(tau_pairs):
    """With the multiplier over the active phases, a 0-1 interface of a three-phase
    obstacle system with phase 2 absent evolves exactly as the two-phase system
    (tau = tau_01 where only phases 0 and 1 are present) and phase 2 stays absent;
    clip-and-renormalise does not reproduce it."""
    p3, p2, phi3, mu = _binary_three_phase("obstacle_active", tau_pairs)
    # the free update pushes phase 2 below zero where 0 and 1 meet
    R = gp.rhs_phi(phi3, mu, 0, p3)
    raw2 = p3.dt * (R[2] - R.mean(axis=0)) / (gp.relaxation(phi3, p3) * p3.eps)
    inter = (phi3[0] > 0) & (phi3[1] > 0)
    assert inter.sum() >= 6 and np.all(raw2[inter] < 0)
    f3, m3 = phi3, mu
    f2, m2 = phi3[:2], mu
    for n in range(30):
        f3, m3 = gp.step(f3, m3, n, p3)
        f2, m2 = gp.step(f2, m2, n, p2)
        assert np.all(f3[2] == 0.0)
    assert np.max(np.abs(f3[:2] - f2)) < 1e-13
    assert np.max(np.abs(m3 - m2)) < 1e-13
    pc = p3.copy(potential="obstacle")
    fc, _ = gp.run(phi3, mu, 0, 30, pc)
    assert np.max(np.abs(fc[:2] - f2)) > 1e-6


def test_active_set_step_projects_the_euler_update():
    """Where the obstacle pushes a phase below zero in every step, the step is the
    nearest simplex point (by the enumeration above) to the free update."""
    p, _, _ = params(N=3, K1=2, n=(16, 12, 1), potential="obstacle_active", tau_pairs=True, seed=9)
    p.gamma[0, 1] = p.gamma[1, 0] = 0.6
    p.gamma[0, 2] = p.gamma[2, 0] = p.gamma[1, 2] = p.gamma[2, 1] = 1.8
    p.dt = 0.2 * inputs.dt_limit(p)
    phi, mu = simplex_state(p, seed=12)
    rng = np.random.default_rng(7)
    a = rng.uniform(0.3, 0.7, size=(12, 8))
    phi[0, :, :8], phi[1, :, :8], phi[2, :, :8] = a, 1.0 - a, 0.0
    moved = 0
    f, m = phi, mu
    for n in range(20):
        R = gp.rhs_phi(f, m, n, p)
        raw = f + p.dt * (R - R.mean(axis=0)) / (gp.relaxation(f, p) * p.eps)
        moved += int(np.count_nonzero(raw < 0.0))
        f1, m = gp.step(f, m, n, p)
        want = np.empty_like(raw)
        for j in range(raw.shape[1]):
            for i in range(raw.shape[2]):
                y = raw[:, j, i]
                best, bd = None, np.inf
                for r in (1, 2, 3):
                    for S in itertools.combinations(range(3), r):
                        x = np.zeros(3)
                        th = (sum(y[q] for q in S) - 1.0) / r
                        for q in S:
                            x[q] = y[q] - th
                        if np.all(x >= -1e-15) and np.sum((x - y) ** 2) < bd:
                            best, bd = x, np.sum((x - y) ** 2)
                want[:, j, i] = best
        assert np.allclose(f1, want, rtol=0, atol=1e-14)
        f = f1
    assert moved > 100
    assert f.min() >= 0.0 and np.max(np.abs(f.sum(axis=0) - 1.0)) < 1e-14


def test_relaxation_hand_values():
    p = inputs.Params(nphases=3, ncomp=2, tau=0.9)
    p.tau_ab[0, 1], p.tau_ab[0, 2], p.tau_ab[1, 2] = 1.0, 2.0, 4.0
    phi = np.array([[0.5, 0.2, 1.0], [0.5, 0.3, 0.0], [0.0, 0.5, 0.0]])
    got = gp.relaxation(phi, p)
    # pair weights 0.06, 0.10, 0.15 -> (0.06 + 0.2 + 0.6) / 0.31
    assert abs(got[0] - 1.0) < 1e-15
    assert abs(got[1] - 0.86 / 0.31) < 1e-15
    assert got[2] == 0.9  # bulk: the single tau


# ----------------------------------------------------------------------------
# Moving frame
# ----------------------------------------------------------------------------

def test_front_row_hand_values():
    phi = np.zeros((2, 6, 4))
    phi[1] = 1.0
    assert gp.front_row(phi) == -1
    phi[0, 3, 2], phi[1, 3, 2] = 0.6, 0.4
    phi[0, 4, 1], phi[1, 4, 1] = 0.5, 0.5  # exactly 1/2: still liquid
    assert gp.front_row(phi) == 3


@pytest.mark.parametrize("potential", ["well", "obstacle_active"])
def test_shift_equals_the_taller_run(potential):
    """Steps, a frame shift of s rows, more steps == the same steps on a domain s rows
    taller that starts with s more rows of melt, read s rows up -- bitwise, while
    the structure stays away from the bottom and top rows (single solid phase at
    the bottom, uniform melt at the top, information moves one row per step)."""
    s, n1, n2 = 5, 6, 7
    ny = 40
    p, _, _ = params(N=3, K1=2, n=(12, ny, 1), bc=(0, 1, 0), potential=potential, slopes=True,
                     G=0.02, V=0.5, seed=11)
    p.D[:2, :] = 0.0  # solids do not diffuse
    p.dt = 0.2 * inputs.dt_limit(p)
    tall = p.copy(n=(12, ny + s, 1))
    rng = np.random.default_rng(1)
    phi = np.zeros((3, ny + s, 12))
    mu_melt = np.array([0.02, -0.01])
    mu = np.empty((2, ny + s, 12))
    mu[0], mu[1] = mu_melt[0], mu_melt[1]
    phi[2] = 1.0
    # bottom: pure phase 0, uniform mu; rows 25..28: a random front; above: melt.
    # In n1 + n2 = 13 steps the front's influence reaches down to row 12 (> s) and,
    # before the shift, up to row 34 (< ny - 1).
    phi[0, :25], phi[2, :25] = 1.0, 0.0
    mu[:, :25] = np.array([0.05, 0.04])[:, None, None]
    fr = rng.dirichlet([1.0, 1.0, 1.0], size=(4, 12))
    phi[:, 25:29] = np.moveaxis(fr, -1, 0)
    mu[:, 25:29] += rng.uniform(-0.01, 0.01, size=(2, 4, 12))
    assert gp.front_row(phi) >= 25
    # short run: the bottom ny rows, n1 steps, shift, n2 steps in the shifted frame
    f, m = gp.run(phi[:, :ny], mu[:, :ny], 0, n1, p)
    f, m = gp.shift(f, m, s, mu_melt)
    f, m = gp.run(f, m, n1, n2, p, y_origin=s)
    ft, mt = gp.run(phi, mu, 0, n1 + n2, tall)
    assert np.array_equal(f, ft[:, s:])
    assert np.array_equal(m, mt[:, s:])


# ----------------------------------------------------------------------------
# The anti-trapping current (Eq. jatr) with the extended model
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 0)])
@pytest.mark.parametrize("offdiag", [False, True])
def test_antitrapping_conserves_solute_with_the_extended_model(bc, offdiag):
    """The current enters as a divergence and is divided by the same (matrix)
    chi(phi^{n+1}) as the rest of the mu update, so the composition of every time
    level (with its own T under a moving gradient) stays put, while the current
    moves mu well away from the run without it."""
    p, _, _ = params(N=3, K1=2, n=(9, 8, 1), bc=bc, slopes=True, offdiag=offdiag, G=0.04, V=0.9, seed=3)
    phi, mu = simplex_state(p, seed=4)
    m0 = np.array(gp.diagnostics(phi, mu, p, n=5)["mass"])
    f, m = phi, mu
    for i in range(40):
        f, m = gp.step_antitrapping(f, m, 5 + i, p)
    m1 = np.array(gp.diagnostics(f, m, p, n=45)["mass"])
    assert np.all(np.abs(m1 - m0) <= 1e-13 * np.maximum(1.0, np.abs(m0)))
    _, mp = gp.run(phi, mu, 5, 40, p)
    assert np.max(np.abs(m - mp)) > 1e-6


@pytest.mark.parametrize("offdiag", [False, True])
def test_antitrapping_ramp_takes_each_rows_composition_at_time_level_n(offdiag):
    """A two-phase ramp along x under a gradient along y: every x face carries
    P r (c^s - c^l) with the compositions c^a = chi^a (mu - B^a(T)) of its own row
    at the temperature of time level n (the unit normals are exact on the ramp
    and opposite for the two phases); no y face carries anything."""
    p, _, _ = params(N=2, K1=2, n=(9, 8, 1), bc=(1, 1, 0), slopes=True, offdiag=offdiag, G=0.05, V=0.7, seed=6)
    x, y = inputs.grid_coords(p)
    b, r, n = 0.03, 0.21, 7
    ps = np.broadcast_to(0.5 + b * (x - 4 * p.dx), p.spatial)
    phi = np.stack([ps, 1.0 - ps])
    phin = phi + p.dt * r * np.stack([np.ones_like(ps), -np.ones_like(ps)])
    mu = np.stack([np.full(p.spatial, 0.13), np.full(p.spatial, -0.08)])
    rows = np.arange(p.n[1])
    T = p.T0 + p.G * (rows * p.dx - p.y0 - p.V * n * p.dt)  # time level n, one value per row
    chi = np.linalg.inv(np.stack([[[2 * p.A[a, 0], p.A01[a]], [p.A01[a], 2 * p.A[a, 1]]] for a in range(2)]))
    pref = p.eps / (2.0 * math.sqrt(2.0))
    for axis, j in gp.antitrapping_faces(phi, phin, mu, p, n=n):
        if axis != -1:
            assert np.all(j == 0.0)
            continue
        for row in range(1, p.n[1] - 1):
            c = [chi[a] @ (np.array([0.13, -0.08]) - (p.B[a, :2] + p.Bt[a, :2] * (T[row] - p.Te))) for a in range(2)]
            want = pref * r * (c[0] - c[1])
            # faces between interior columns of this row
            np.testing.assert_allclose(j[:, row, 1:-1], np.broadcast_to(want[:, None], (2, p.n[0] - 1)),
                                       rtol=1e-12, atol=1e-15)
