"""Pins of the oracle's anti-trapping current (Eq. jatr) and the step that uses it.

The face current is checked where its discrete parts are exact: on linear
ramps the face gradients (normal and tangential) equal the continuum gradient,
so the unit normals, and with them the current, have closed forms.  A
three-phase ramp with orthogonal solid and liquid normals checks the weight
-n_a . n_liq phase by phase.  Conservation, the zero-flux boundary, mirror and
transpose equivariance and the degenerate cases (equal phase compositions,
stationary phases) pin the rest.
"""
import math

import numpy as np
import pytest

from oracle import gp
from paper_2404_01035_amd import inputs
from test_oracle_pins import random_state, small_params


def _uniform_mu(p, value=0.37):
    return np.full((p.nmu,) + p.spatial, value)


def _coords(p):
    """Cell coordinates (x, y[, z]) in units of length, broadcast to the grid."""
    grids = np.meshgrid(*[np.arange(s) * p.dx for s in p.spatial], indexing="ij")
    return grids[::-1]  # spatial shape is ([z,] y, x)


def _face_block(j, p, axis):
    """Faces normal to ``axis`` whose two cells and their tangential neighbours lie inside the grid."""
    idx = [slice(None)] * j.ndim
    for a, _ in gp.spatial_axes(p):
        idx[j.ndim + a] = slice(1, -1)
    return j[tuple(idx)]


@pytest.mark.parametrize("potential", ["well", "obstacle"])
@pytest.mark.parametrize("theta", [0.0, 0.4, 1.1, math.pi / 2, 2.5, 4.0])
def test_linear_ramp_closed_form_2d(potential, theta):
    p = small_params(N=2, n=(9, 8, 1), bc=(1, 1, 1), potential=potential, seed=2)
    x, y = _coords(p)
    b = 0.03
    ps = 0.5 + b * (math.cos(theta) * (x - 4 * p.dx) + math.sin(theta) * (y - 3.5 * p.dx))
    phi = np.stack([ps, 1.0 - ps])
    r = 0.21
    phin = phi + p.dt * r * np.stack([np.ones_like(ps), -np.ones_like(ps)])
    mu = _uniform_mu(p)
    c = gp.c_phase(mu, p)[:, :, 0, 0]  # (N, K-1), uniform
    n = (math.cos(theta), math.sin(theta))
    for axis, j in gp.antitrapping_faces(phi, phin, mu, p):
        comp = 0 if axis == -1 else 1
        # face centres of the checked block: the ramp's value there is the prefactor's phi
        if axis == -1:
            pf = 0.5 + b * (math.cos(theta) * (x[1:-1, :-1] + 0.5 * p.dx - 4 * p.dx)
                            + math.sin(theta) * (y[1:-1, :-1] - 3.5 * p.dx))
        else:
            pf = 0.5 + b * (math.cos(theta) * (x[:-1, 1:-1] - 4 * p.dx)
                            + math.sin(theta) * (y[:-1, 1:-1] + 0.5 * p.dx - 3.5 * p.dx))
        pref = p.eps / (2.0 * math.sqrt(2.0)) if potential == "well" else gp.at_prefactor(pf, p)
        # n_liq = -n_solid exactly, so the weight -n_s . n_l is 1
        want = pref * r * n[comp] * (c[0, 0] - c[1, 0])
        got = _face_block(j, p, axis)[0]
        assert got.shape == np.broadcast_shapes(got.shape, np.shape(want))
        np.testing.assert_allclose(got, np.broadcast_to(want, got.shape), rtol=1e-12, atol=1e-15)


def test_linear_ramp_closed_form_3d():
    p = small_params(N=2, dim=3, n=(6, 5, 4), bc=(1, 1, 1), seed=3)
    x, y, z = _coords(p)
    d = np.array([0.3, -0.5, 0.8])
    d = d / np.linalg.norm(d)
    b = 0.025
    ps = 0.5 + b * (d[0] * (x - 2.5) + d[1] * (y - 2.0) + d[2] * (z - 1.5))
    phi = np.stack([ps, 1.0 - ps])
    r = -0.13
    phin = phi + p.dt * r * np.stack([np.ones_like(ps), -np.ones_like(ps)])
    mu = _uniform_mu(p, 0.2)
    c = gp.c_phase(mu, p)[:, 0, 0, 0, 0]
    for axis, j in gp.antitrapping_faces(phi, phin, mu, p):
        comp = {-1: 0, -2: 1, -3: 2}[axis]
        want = p.eps / (2.0 * math.sqrt(2.0)) * r * d[comp] * (c[0] - c[1])
        got = _face_block(j, p, axis)[0]
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-15)


def test_three_phase_weight_uses_each_solid_against_the_liquid():
    # phi_0 rises along x, the liquid phi_2 along y, phi_1 = 1 - phi_0 - phi_2:
    # n_0 . n_liq = 0, so phase 0 carries nothing however fast it moves;
    # n_1 = -(1, 1)/sqrt 2 gives n_1,axis = -1/sqrt 2 and weight 1/sqrt 2.
    p = small_params(N=3, n=(8, 7, 1), bc=(1, 1, 1), seed=4)
    x, y = _coords(p)
    b = 0.02
    p0 = 0.3 + b * (x - 3.5 * p.dx)
    p2 = 0.3 + b * (y - 3.0 * p.dx)
    phi = np.stack([p0, 1.0 - p0 - p2, p2])
    r0, r1 = 0.5, -0.17
    phin = phi + p.dt * np.stack([np.full_like(p0, r0), np.full_like(p0, r1), np.full_like(p0, -r0 - r1)])
    mu = np.stack([np.full(p.spatial, 0.31), np.full(p.spatial, -0.12)])
    c = gp.c_phase(mu, p)[:, :, 0, 0]  # (3, 2)
    assert np.all(np.abs(c[0] - c[2]) > 1e-3)  # phase 0 would contribute if its weight were wrong
    for axis, j in gp.antitrapping_faces(phi, phin, mu, p):
        for k in range(2):
            want = p.eps / (2.0 * math.sqrt(2.0)) * r1 * (c[1, k] - c[2, k]) * (-0.5)
            np.testing.assert_allclose(_face_block(j, p, axis)[k], want, rtol=1e-12, atol=1e-15)


def test_zero_when_the_phases_share_their_compositions():
    p = small_params(N=3, n=(7, 6, 1), bc=(0, 1, 0), seed=5)
    for a in range(3):
        p.A[a, :2] = p.A[2, :2]
        p.B[a, :2] = p.B[2, :2]
    phi, mu = random_state(p, seed=6, simplex=True)
    phin, mun = gp.step(phi, mu, 0, p)
    pa, ma = gp.step_antitrapping(phi, mu, 0, p)
    assert np.array_equal(pa, phin) and np.array_equal(ma, mun)


def test_zero_when_the_phases_do_not_move():
    p = small_params(N=3, n=(7, 6, 1), bc=(0, 0, 0), seed=7)
    phi, mu = random_state(p, seed=8, simplex=True)
    for _, j in gp.antitrapping_faces(phi, phi, mu, p):
        assert not np.any(j)


def test_zero_flux_boundary_faces_carry_no_current():
    p = small_params(N=3, n=(7, 6, 1), bc=(1, 1, 1), seed=9)
    phi, mu = random_state(p, seed=10, simplex=True)
    phin, _ = gp.step(phi, mu, 0, p)
    for axis, j in gp.antitrapping_faces(phi, phin, mu, p):
        first = gp._along(j, axis, slice(0, 1))
        last = gp._along(j, axis, slice(-1, None))
        assert not np.any(first) and not np.any(last)
        assert np.any(j)  # the interior does carry a current


@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 1), (0, 1, 0)])
@pytest.mark.parametrize("N", [2, 3])
def test_step_with_antitrapping_conserves_solute(bc, N):
    # chi^{n+1} (mu^{n+1} - mu^n) + sum_a c^a(mu^n) (h^{n+1} - h^n) = dt div(...):
    # its sum over the cells vanishes for any face current on these boundaries.
    p = small_params(N=N, n=(7, 6, 1), bc=bc, seed=11)
    phi, mu = random_state(p, seed=12, simplex=True)
    phin, mun = gp.step_antitrapping(phi, mu, 0, p)
    chi = gp.chi_phase(p)
    h0, h1 = gp.h(phi), gp.h(phin)
    ca = gp.c_phase(mu, p)
    for k in range(p.nmu):
        chik = sum(h1[b] * chi[b][k] for b in range(N))
        total = chik * (mun[k] - mu[k]) + sum(ca[b][k] * (h1[b] - h0[b]) for b in range(N))
        scale = np.sum(np.abs(chik * (mun[k] - mu[k])))
        assert abs(np.sum(total)) <= 1e-13 * max(scale, 1.0)
    # and the current changes the result
    _, mu_plain = gp.step(phi, mu, 0, p)
    assert np.max(np.abs(mun - mu_plain)) > 1e-6


@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 1)])
def test_mirror_equivariance(bc):
    p = small_params(N=3, n=(7, 6, 1), bc=bc, seed=13)
    phi, mu = random_state(p, seed=14, simplex=True)
    a_phi, a_mu = gp.step_antitrapping(phi, mu, 0, p)
    for ax in (-1, -2):
        f_phi, f_mu = gp.step_antitrapping(np.flip(phi, ax), np.flip(mu, ax), 0, p)
        np.testing.assert_allclose(f_phi, np.flip(a_phi, ax), rtol=0, atol=1e-14)
        np.testing.assert_allclose(f_mu, np.flip(a_mu, ax), rtol=0, atol=1e-14)


def test_transpose_equivariance():
    p = small_params(N=3, n=(6, 6, 1), bc=(0, 0, 0), seed=15)
    phi, mu = random_state(p, seed=16, simplex=True)
    a_phi, a_mu = gp.step_antitrapping(phi, mu, 0, p)
    t_phi, t_mu = gp.step_antitrapping(np.swapaxes(phi, -1, -2), np.swapaxes(mu, -1, -2), 0, p)
    np.testing.assert_allclose(t_phi, np.swapaxes(a_phi, -1, -2), rtol=0, atol=1e-14)
    np.testing.assert_allclose(t_mu, np.swapaxes(a_mu, -1, -2), rtol=0, atol=1e-14)


def test_obstacle_prefactor_values_and_limits():
    p = inputs.Params(potential="obstacle", eps=3.0)
    # phi0 = 1/2: h = 1/2 and sqrt(phi0 (1 - phi0)) = 1/2, so pi eps / 8
    assert gp.at_prefactor(np.array(0.5), p) == pytest.approx(math.pi * 3.0 / 8.0, rel=1e-15)
    # near the ends it vanishes like sqrt(phi0) and (1 - phi0)^(3/2) (to leading order)
    e = 1e-10
    assert gp.at_prefactor(np.array(e), p) == pytest.approx(math.pi * 3.0 / 4.0 * math.sqrt(e), rel=1e-6)
    assert gp.at_prefactor(np.array(1.0 - e), p) == pytest.approx(math.pi * 3.0 * 3.0 / 4.0 * e ** 1.5, rel=1e-4)
    assert np.all(gp.at_prefactor(np.array([-0.1, 0.0, 1.0, 1.2]), p) == 0.0)
    pw = inputs.Params(potential="well", eps=3.0)
    assert gp.at_prefactor(np.array(0.3), pw) == pytest.approx(3.0 / (2.0 * math.sqrt(2.0)), rel=1e-15)


@pytest.mark.parametrize("r1", [0.04, -0.07])
def test_divergence_enters_the_mu_update_with_its_sign(r1):
    # A ramp along x whose growth rate varies linearly in x: the face current is
    # P (c^s - c^l) r_face with r_face the mean of the two cells' rates, so its
    # divergence is P (c^s - c^l) dr/dx in every cell whose two faces are
    # interior, and the current moves mu by -dt div j_at / chi^{n+1} there.
    p = small_params(N=2, n=(9, 5, 1), bc=(1, 1, 1), seed=17)
    x, _ = _coords(p)
    b = 0.03
    ps = 0.5 + b * (x - 4 * p.dx)
    phi = np.stack([ps, 1.0 - ps])
    rate = 0.1 + r1 * x
    phin_target = phi + p.dt * np.stack([rate, -rate])
    mu = _uniform_mu(p, 0.25)
    c = gp.c_phase(mu, p)[:, 0, 0, 0]
    # the current uses the phi^{n+1} of the step; feed the linear-rate one through the faces
    div = 0.0
    for axis, j in gp.antitrapping_faces(phi, phin_target, mu, p):
        if axis == -1:
            div = (j[0][:, 1:] - j[0][:, :-1]) / p.dx
    want = p.eps / (2.0 * math.sqrt(2.0)) * (c[0] - c[1]) * r1
    np.testing.assert_allclose(div[:, 1:-1], want, rtol=1e-11, atol=1e-15)
    # and in the step, the update is mu^{n+1} = (plain step) - dt div j_at / chi^{n+1}
    phin, mu_at = gp.step_antitrapping(phi, mu, 0, p)
    _, mu_plain = gp.step(phi, mu, 0, p)
    div_step = 0.0
    for axis, j in gp.antitrapping_faces(phi, phin, mu, p):
        div_step = div_step + (gp._along(j[0], axis, slice(1, None)) - gp._along(j[0], axis, slice(0, -1))) / p.dx
    chi = gp.chi_phase(p)
    h1 = gp.h(phin)
    chik = h1[0] * chi[0][0] + h1[1] * chi[1][0]
    np.testing.assert_allclose(mu_at[0] - mu_plain[0], -p.dt * div_step / chik, rtol=1e-9, atol=1e-16)


@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 1), (0, 1, 0), (1, 0, 0)])
def test_windowed_step_matches_the_full_step(bc):
    p = small_params(N=3, n=(9, 7, 1), bc=bc, seed=21, G=0.02)
    phi, mu = random_state(p, seed=22, simplex=True)
    fphi, fmu = gp.step_antitrapping(phi, mu, 3, p)
    for lo, hi in [((0, 0), (7, 9)), ((0, 0), (2, 3)), ((5, 6), (7, 9)), ((2, 3), (5, 7)), ((0, 8), (7, 9)),
                   ((6, 0), (7, 9))]:
        wphi, wmu = gp.step_antitrapping_window(phi, mu, 3, p, lo, hi)
        sl = (slice(None), slice(lo[0], hi[0]), slice(lo[1], hi[1]))
        np.testing.assert_allclose(wphi, fphi[sl], rtol=0, atol=1e-15)
        np.testing.assert_allclose(wmu, fmu[sl], rtol=0, atol=1e-14)


def test_windowed_step_matches_the_full_step_3d():
    p = small_params(N=2, dim=3, n=(6, 5, 4), bc=(0, 1, 0), seed=23)
    phi, mu = random_state(p, seed=24, simplex=True)
    fphi, fmu = gp.step_antitrapping(phi, mu, 0, p)
    for lo, hi in [((0, 0, 0), (4, 5, 6)), ((1, 2, 3), (3, 5, 6)), ((3, 0, 0), (4, 2, 2))]:
        wphi, wmu = gp.step_antitrapping_window(phi, mu, 0, p, lo, hi)
        sl = (slice(None),) + tuple(slice(a, b) for a, b in zip(lo, hi))
        np.testing.assert_allclose(wphi, fphi[sl], rtol=0, atol=1e-15)
        np.testing.assert_allclose(wmu, fmu[sl], rtol=0, atol=1e-14)
