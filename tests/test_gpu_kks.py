"""GPU parity of the KKS variant (Sec. 2.2: the phase fields of Eq. aceq, the
potential of Eq. Well's form or the sextic Eq. Well1) with the FP64 oracle on
the same seeded inputs: 2D one and two steps per launch, graphs, 3D, FP32, the
extended model's terms together with KKS, batches mixing KKS and
grand-potential instances (each instance bitwise as stepped alone), and the
device form of the exact map between the two phase equations."""
import math

import numpy as np
import pytest

from oracle import gp
from paper_2404_01035_amd import abi, inputs

pytestmark = pytest.mark.gpu


def run_gpu(p, phi, mu, nsteps, fuse=None, graph=0, tile=None):
    from paper_2404_01035_amd.solver import Solver

    s = Solver(p)
    try:
        if fuse:
            s.set_fusion(fuse)
        if graph:
            s.set_graph(graph)
        if tile:
            s.set_tile(*tile)
        s.load(phi, mu)
        s.step(nsteps)
        return s.fields()
    finally:
        s.close()


def errs(a, b):
    return float(np.max(np.abs(a - b)))


def eutectic_kks(potential, n=(150, 96, 1), precision="f64", seed=1, **kw):
    p, phi, mu = inputs.config_c2(n=n, precision=precision, seed=seed)
    theta = [0.3, 0.2, 0.4] if potential == "theta" else None
    k = inputs.kks_from(p, potential=potential, theta=theta, theta3=0.6 if potential == "theta" else 0.0, **kw)
    return k, phi, mu


CASES = [("well", 1), ("well", 2), ("theta", 1), ("theta", 2)]


@pytest.mark.parametrize("potential,fuse", CASES)
def test_2d_kks_fp64_matches_oracle(potential, fuse):
    k, phi, mu = eutectic_kks(potential)
    print(f"kks 2D {potential} fuse {fuse}", flush=True)
    g = run_gpu(k, phi, mu, 120, fuse=fuse)
    o = gp.run(phi, mu, 0, 120, k)
    e = max(errs(g[0], o[0]), errs(g[1], o[1]))
    print(f"  max err {e:.3e}")
    assert e <= 1e-10
    assert errs(o[0], phi) > 1e-3  # it moved


def test_2d_kks_theta_with_extended_terms_and_graphs():
    # Eq. Well1 with B(T) from slopes, off-diagonal curvature and diffusivity, two steps per launch in graphs
    p, phi, mu = inputs.config_c2_slopes(n=(130, 90, 1))
    p = p.copy()
    p.A01[:3] = (0.2, -0.1, 0.15)
    p.D01[2] = 0.3
    k = inputs.kks_from(p, potential="theta", theta=[0.5, 0.1, 0.2], theta3=0.3)
    g = run_gpu(k, phi, mu, 60, fuse=2, graph=6)
    o = gp.run(phi, mu, 0, 60, k)
    assert max(errs(g[0], o[0]), errs(g[1], o[1])) <= 1e-10


@pytest.mark.parametrize("potential", ["well", "theta"])
def test_3d_kks_fp64_matches_oracle(potential):
    p, phi, mu = inputs.config_c3(precision="f64", n=(40, 33, 21), radius=7.0)
    k = inputs.kks_from(p, eps_k=5.0, potential=potential, theta=[0.4, 0.2] if potential == "theta" else None)
    g = run_gpu(k, phi, mu, 40)
    o = gp.run(phi, mu, 0, 40, k)
    assert max(errs(g[0], o[0]), errs(g[1], o[1])) <= 1e-10
    assert errs(o[0], phi) > 1e-4


@pytest.mark.parametrize("potential", ["well", "theta"])
def test_2d_kks_fp32_within_1e4(potential):
    k, phi, mu = eutectic_kks(potential, precision="f32")
    g = run_gpu(k, phi, mu, 100)
    o = gp.run(phi, mu, 0, 100, k.copy(precision="f64"))
    assert errs(g[0], o[0]) <= 1e-4 and errs(g[1], o[1]) <= 1e-4


def test_device_gp_and_kks_phase_equations_coincide_under_the_map():
    # eps = 1 grand potential against eps_k = sqrt 2, M_phi = 1/tau KKS: the same folded coefficients
    p, phi, mu = inputs.config_c2(n=(128, 80, 1))
    g = p.copy(eps=1.0, tau=1.3)
    g.dt = 0.2 * inputs.dt_limit(g)
    k = inputs.kks_from(g, eps_k=math.sqrt(2.0), Mphi=1.0 / 1.3)
    k.dt = g.dt
    a = run_gpu(g, phi, mu, 50)
    b = run_gpu(k, phi, mu, 50)
    assert max(errs(a[0], b[0]), errs(a[1], b[1])) <= 1e-13


def _batch_members():
    k1, phi1, mu1 = eutectic_kks("well", n=(96, 64, 1))
    g2, phi2, mu2 = inputs.config_c2(n=(70, 52, 1), seed=2)
    k3, phi3, mu3 = eutectic_kks("well", n=(64, 64, 1), seed=3)
    return [(k1, phi1, mu1), (g2, phi2, mu2), (k3, phi3, mu3)]


def _run_batch(members, nsteps):
    from paper_2404_01035_amd.solver import BatchSolver

    b = BatchSolver([m[0] for m in members])
    try:
        for i, (_, f, m) in enumerate(members):
            b.load(i, f, m)
        b.step(nsteps)
        return [b.fields(i) for i in range(len(members))]
    finally:
        b.close()


def test_batch_mixing_kks_and_gp_instances():
    members = _batch_members()
    got = _run_batch(members, 40)
    for (p, f, m), (gf, gm) in zip(members, got):
        alone = run_gpu(p, f, m, 40)
        assert np.array_equal(gf, alone[0]) and np.array_equal(gm, alone[1])
        o = gp.run(f, m, 0, 40, p)
        assert max(errs(gf, o[0]), errs(gm, o[1])) <= 1e-10


def test_batch_with_a_well1_instance_runs_the_general_kernels():
    k1, phi1, mu1 = eutectic_kks("theta", n=(96, 64, 1))
    g2, phi2, mu2 = inputs.config_c2(n=(70, 52, 1), seed=2)
    k1 = k1.copy(dt=min(k1.dt, g2.dt))
    g2 = g2.copy(dt=k1.dt)
    members = [(k1, phi1, mu1), (g2, phi2, mu2)]
    got = _run_batch(members, 30)
    for (p, f, m), (gf, gm) in zip(members, got):
        o = gp.run(f, m, 0, 30, p)
        assert max(errs(gf, o[0]), errs(gm, o[1])) <= 1e-10


def test_kks_states_refuse_the_current():
    from paper_2404_01035_amd.solver import Solver

    k, phi, mu = eutectic_kks("well", n=(64, 48, 1))
    s = Solver(k)
    try:
        with pytest.raises(abi.MPError) as ei:
            s.set_antitrapping(1)
        assert ei.value.code == abi.MP_E_STATE
    finally:
        s.close()
