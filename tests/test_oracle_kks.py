"""Pins of the oracle's KKS variant (Sec. 2.2): the phase-field equation Eq.
aceq with the potential of Eq. Well or Eq. Well1, against facts the paper and
the mathematics fix: hand values of Eq. Well1, its derivative by complex steps,
the reduction of Eq. Well1 to Eq. Well's form, the exact map between the KKS
phase equation and the grand-potential one (Eq. phi_eqn with eps = 1 is Eq.
aceq with eps = sqrt 2 and M_phi = 1/tau), the stationary tanh profile of a
two-phase interface under Eq. Well1, and conservation of the solute."""
import math

import numpy as np
import pytest

from oracle import gp
from paper_2404_01035_amd import inputs


def _theta_params(N):
    p = inputs.Params(nphases=N, ncomp=2, model="kks", potential="theta")
    p.theta[:3] = (1.0, 2.0, 3.0)
    p.theta_ab[0, 1] = p.theta_ab[1, 0] = 4.0
    p.theta_ab[0, 2] = p.theta_ab[2, 0] = 5.0
    p.theta_ab[1, 2] = p.theta_ab[2, 1] = 6.0
    p.theta3 = 7.0
    return p


def test_g_theta_hand_values():
    p = _theta_params(3)
    col = lambda *v: np.array(v, dtype=float).reshape(3, 1)
    # pure phase: every term vanishes
    assert gp.g_theta(col(1.0, 0.0, 0.0), p)[0] == 0.0
    # binary midpoint of phases 0 and 1: (Theta_0 + Theta_1 + Theta_01) / 16
    assert gp.g_theta(col(0.5, 0.5, 0.0), p)[0] == pytest.approx((1.0 + 2.0 + 4.0) / 16.0, rel=1e-15)
    # the triple point: 6 * 4/81 + 15/81 + 7/729 = 358/729
    assert gp.g_theta(col(1 / 3, 1 / 3, 1 / 3), p)[0] == pytest.approx(358.0 / 729.0, rel=1e-14)


@pytest.mark.parametrize("N", [2, 3])
def test_dg_theta_is_the_derivative_of_g_theta(N):
    p = _theta_params(N)
    rng = np.random.default_rng(7)
    phi = rng.uniform(-0.2, 1.2, size=(N, 5))
    dg = gp.dg_theta(phi, p)
    h = 1e-30
    for a in range(N):
        z = phi.astype(complex)
        z[a] += 1j * h
        np.testing.assert_allclose(dg[a], gp.g_theta(z, p).imag / h, rtol=1e-13, atol=1e-14)


def _random_state(p, seed):
    phi, mu = inputs.random_multiphase(p, seed=seed, amp=0.6)
    return phi, mu


def _eutectic(n=(24, 20, 1), seed=3, delta=0.0):
    p, _, _ = inputs.config_c2(n=n, seed=seed)
    p = p.copy()
    for a in range(3):
        for b in range(a + 1, 3):
            p.delta[a, b] = p.delta[b, a] = delta
    p.gamma3 = 0.7
    p.G, p.V = 3e-3, 0.4
    return p


@pytest.mark.parametrize("delta", [0.0, 0.03])
def test_kks_phase_equation_is_the_gp_one_under_the_parameter_map(delta):
    # Eq. phi_eqn with eps = 1: dphi/dt = (1/tau)[G - dw - dpsi - lambda]; Eq. aceq
    # with eps_k = sqrt 2 and M_phi = 1/tau: dphi/dt = (1/tau)[(2/2) G - dw - dpsi - lambda]
    g = _eutectic(delta=delta).copy(eps=1.0, tau=1.3)
    g.dt = 0.2 * inputs.dt_limit(g)
    k = inputs.kks_from(g, eps_k=math.sqrt(2.0), Mphi=1.0 / 1.3)
    k.dt = g.dt
    phi, mu = _random_state(g, 5)
    p1, m1 = gp.step(phi, mu, 7, g)
    p2, m2 = gp.step(phi, mu, 7, k)
    np.testing.assert_allclose(p2, p1, rtol=0, atol=1e-14)
    np.testing.assert_allclose(m2, m1, rtol=0, atol=1e-14)
    # and a different map changes the result
    k2 = k.copy(Mphi=1.1 / 1.3)
    assert np.max(np.abs(gp.step(phi, mu, 7, k2)[0] - p1)) > 1e-6


def test_well1_with_matching_thetas_is_the_well_form():
    base = _eutectic().copy(gamma3=0.0)
    kw = inputs.kks_from(base, potential="well")
    kt = inputs.kks_from(base, potential="theta")  # Theta_a = 0, Theta_ab = 9 gamma_ab, Theta_abd = 0
    kt.dt = kw.dt
    phi, mu = _random_state(base, 9)
    a = gp.step(phi, mu, 0, kw)
    b = gp.step(phi, mu, 0, kt)
    np.testing.assert_allclose(b[0], a[0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(b[1], a[1], rtol=0, atol=1e-15)
    # a non-zero Theta_a or Theta_abd shows
    kt.theta[0] = 0.5
    assert np.max(np.abs(gp.step(phi, mu, 0, kt)[0] - a[0])) > 1e-6


def test_two_phase_tanh_profile_is_stationary_under_well1():
    # two phases with equal grand potentials: dphi/dt = M_phi [(eps^2/2) gamma phi'' - W phi (1-phi)(1-2phi)],
    # W = Theta_0 + Theta_1 + Theta_01, stationary for phi = (1 + tanh(x / w)) / 2 with w = eps sqrt(2 gamma / W):
    # the discrete rate of that profile falls as dx^2 (second-order faces), a wrong width's does not
    W = 0.6 + 0.9 + 1.5

    def rate(dx, stretch=1.0, L=60.0):
        nx = int(round(L / dx))
        p = inputs.binary_two_phase(dim=2, n=(nx, 2, 1), bc=(inputs.BC_NOFLUX, inputs.BC_PERIODIC, 0),
                                    undercooling=0.0, c_solid=0.5, c_liquid=0.5).copy(dx=dx)
        k = inputs.kks_from(p, eps_k=2.0, Mphi=1.0, potential="theta", theta=[0.6, 0.9],
                            theta_ab=[[0, 1.5], [1.5, 0]])
        w = stretch * k.eps * math.sqrt(2.0 * p.gamma[0][1] / W)
        x = (np.arange(nx) + 0.5) * dx - nx * dx / 2
        sol = 0.5 * (1.0 + np.tanh(x / w))
        phi = np.stack([np.tile(sol, (2, 1)), np.tile(1.0 - sol, (2, 1))])
        mu = np.zeros((1, 2, nx))
        return np.max(np.abs(gp.step(phi, mu, 0, k)[0] - phi)) / k.dt

    r1, r2 = rate(0.25), rate(0.125)
    assert 3.7 < r1 / r2 < 4.3, (r1, r2)
    assert r2 < 1e-3
    assert rate(0.125, stretch=1.2) > 0.05


def test_kks_conserves_solute():
    base = _eutectic(n=(20, 18, 1)).copy(bc=(inputs.BC_PERIODIC, inputs.BC_PERIODIC, 0), G=0.0, V=0.0)
    k = inputs.kks_from(base, potential="theta", theta=[0.3, 0.2, 0.1], theta3=0.4)
    phi, mu = _random_state(base, 11)
    c0 = gp.composition(phi, mu, k).sum(axis=(1, 2))
    ph, m = gp.run(phi, mu, 0, 40, k)
    c1 = gp.composition(ph, m, k).sum(axis=(1, 2))
    np.testing.assert_allclose(c1, c0, rtol=1e-12)
    assert np.max(np.abs(ph - phi)) > 1e-3  # it moved
