"""Diagnostics formed inside the last step launch (mp_step_diag) against the
separate reduction pass (mp_step + mp_diagnostics) on the same seeded inputs:
the state after the call bitwise that of mp_step; max |sum phi - 1|, min chi
and the non-finite count bitwise (maxima, minima and counts do not depend on
the grouping); solute and phase volumes within 1e-13 relative (FP64 Neumaier
partial sums grouped by the step kernel's strips or tiles instead of the
reduction's blocks).  Cases: 2D FP64 one and two steps per launch, anisotropy
and the obstacle, no-flux and periodic edges, ragged grids; 3D with 64 x 4 and
64 x 8 tiles in FP64 and FP32; the extended model in 2D and 3D; a
graph-stepped run; and the paths that take the separate pass (FP32 2D strips
with one, two and four cells per lane, the anti-trapping current, a batch).
One case also against the oracle's diagnostics of the oracle's state."""
import numpy as np
import pytest

from oracle import gp
from paper_2404_01035_amd import abi, inputs

pytestmark = pytest.mark.gpu


def _pair(p, phi, mu, setup):
    from paper_2404_01035_amd.solver import Solver

    out = []
    for _ in range(2):
        s = Solver(p)
        setup(s)
        s.load(phi, mu)
        out.append(s)
    return out


def _same_diag(a, b, rel=1e-13):
    assert a["step"] == b["step"]
    assert a["nonfinite"] == b["nonfinite"]
    assert a["max_sum_dev"] == b["max_sum_dev"], (a["max_sum_dev"], b["max_sum_dev"])
    assert a["min_chi"] == b["min_chi"], (a["min_chi"], b["min_chi"])
    for key in ("mass", "volume"):
        for x, y in zip(a[key], b[key]):
            assert abs(x - y) <= rel * max(abs(x), abs(y), 1e-300), (key, x, y)


def _check(p, phi, mu, nsteps, setup=lambda s: None, rel=1e-13):
    fused, plain = _pair(p, phi, mu, setup)
    try:
        print(f"step_diag: dim {p.dim} n {tuple(p.n)} {p.precision} nsteps {nsteps}", flush=True)
        d = fused.step_diag(nsteps)
        plain.step(nsteps)
        e = plain.diagnostics()
        _same_diag(d, e, rel)
        assert abi.mp_current(fused.st) == abi.mp_current(plain.st)
        f1, m1 = fused.fields()
        f2, m2 = plain.fields()
        assert np.array_equal(f1, f2) and np.array_equal(m1, m2)
        # the call can be repeated from the state it left
        d2 = fused.step_diag(1)
        plain.step(1)
        _same_diag(d2, plain.diagnostics(), rel)
        return d
    finally:
        fused.close()
        plain.close()


@pytest.mark.parametrize("fuse", [1, 2])
@pytest.mark.parametrize("nsteps", [1, 2, 5])
def test_2d_eutectic_fp64(fuse, nsteps):
    p, phi, mu = inputs.config_c2(n=(333, 217, 1))
    phi2, mu2 = inputs.random_multiphase(p, seed=4, amp=0.3)
    _check(p, 0.5 * (phi + phi2), mu + mu2, nsteps, lambda s: s.set_fusion(fuse))


@pytest.mark.parametrize("vec", [1, 2, 4])
@pytest.mark.parametrize("fuse", [1, 2])
def test_2d_eutectic_fp32_cells_per_lane(vec, fuse):
    p, phi, mu = inputs.config_c2(n=(336, 150, 1), precision="f32")

    def setup(s):
        s.set_fusion(fuse)
        s.set_tile(256, 16, vec)

    _check(p, phi, mu, 4, setup)


@pytest.mark.parametrize("potential,delta,bc", [("obstacle", 0.0, (0, 0, 0)), ("well", 0.03, (1, 1, 0)),
                                                ("obstacle", 0.03, (1, 0, 0))])
def test_2d_binary_variants(potential, delta, bc):
    p = inputs.binary_two_phase(dim=2, n=(130, 97, 1), bc=bc, potential=potential, delta=delta,
                                undercooling=0.2)
    phi, mu = inputs.random_multiphase(p, seed=11, amp=1.0)
    _check(p, phi, mu, 3)


# 64 x 8 tiles only where their LDS ring fits (FP32 here)
@pytest.mark.parametrize("bx,precision", [(256, "f64"), (256, "f32"), (512, "f32")])
def test_3d_dendrite(bx, precision):
    p, phi, mu = inputs.config_c3(precision=precision, n=(70, 37, 19), radius=6.0)
    phi2, mu2 = inputs.random_multiphase(p, seed=2, amp=0.2)

    def setup(s):
        s.set_tile(bx, 5, 0)

    _check(p, 0.5 * (phi + phi2), mu + mu2, 2, setup)


def test_2d_extended_model():
    p, phi, mu = inputs.config_c2_slopes(n=(150, 96, 1))
    for a, b, t in ((0, 1, 0.8), (0, 2, 1.3), (1, 2, 1.1)):
        p.tau_ab[a, b] = p.tau_ab[b, a] = t
    p.potential = "obstacle_active"
    p.dt = 0.2 * inputs.dt_limit(p)
    _check(p, phi, mu, 4)
    _check(p, phi, mu, 3, lambda s: s.set_fusion(1))


def test_3d_extended_model():
    p = inputs.binary_two_phase(dim=3, n=(67, 21, 13), bc=(1, 1, 1), delta=0.02, undercooling=0.25)
    p.Bt[:2, 0] = (0.3, -0.2)
    p.Ct[:2] = (0.05, 0.0)
    p.G, p.V, p.y0 = 2e-3, 0.3, 6.0
    p.dt = 0.2 * inputs.dt_limit(p)
    phi, mu = inputs.random_multiphase(p, seed=8, amp=1.0)
    _check(p, phi, mu, 2)


def test_after_graph_steps():
    p, phi, mu = inputs.config_c2(n=(200, 128, 1))
    _check(p, phi, mu, 13, lambda s: s.set_graph(4))


def test_antitrapping_and_batch_take_the_separate_pass():
    from paper_2404_01035_amd.solver import BatchSolver

    p, phi, mu = inputs.config_c2(n=(128, 96, 1))
    for mode in (1, 2):
        _check(p, phi, mu, 3, lambda s, m=mode: s.set_antitrapping(m), rel=0.0)
    plist = [inputs.config_c2(n=(96, 64, 1))[0], inputs.binary_two_phase(n=(70, 50, 1), undercooling=0.2)]
    states = [inputs.config_c2(n=(96, 64, 1))[1:], inputs.random_multiphase(plist[1], seed=3, amp=1.0)]
    bs = [BatchSolver(plist) for _ in range(2)]
    try:
        for b in bs:
            for i, (f, m) in enumerate(states):
                b.load(i, f, m)
        d = bs[0].step_diag(3)
        bs[1].step(3)
        e = bs[1].diagnostics()
        assert len(d) == 2
        for x, y in zip(d, e):
            _same_diag(x, y, 0.0)
    finally:
        for b in bs:
            b.close()


def test_nonfinite_reported():
    from paper_2404_01035_amd.solver import Solver

    p, phi, mu = inputs.config_c1()
    mu = mu.copy()
    mu[0, 20, 30] = np.nan
    s = Solver(p)
    try:
        s.load(phi, mu)
        with pytest.raises(abi.MPError) as ei:
            s.step_diag(2)
        assert ei.value.code == abi.MP_E_NONFINITE
        d = s.step_diag(1, allow_nonfinite=True)
        assert d["nonfinite"] > 0 and d["step"] == 3
    finally:
        s.close()


def test_matches_oracle_diagnostics():
    from paper_2404_01035_amd.solver import Solver

    p, phi, mu = inputs.config_c2(n=(160, 120, 1))
    s = Solver(p)
    try:
        s.load(phi, mu)
        d = s.step_diag(6)
    finally:
        s.close()
    ophi, omu = gp.run(phi, mu, 0, 6, p)
    o = gp.diagnostics(ophi, omu, p, 6)
    for k in range(2):
        assert abs(d["mass"][k] - o["mass"][k]) <= 1e-10 * abs(o["mass"][k])
        assert abs(d["min_chi"][k] - o["min_chi"][k]) <= 1e-12
    for a in range(3):
        assert abs(d["volume"][a] - o["volume"][a]) <= 1e-10 * abs(o["volume"][a])
    assert abs(d["max_sum_dev"] - o["max_sum_dev"]) <= 1e-12


def test_more_records_than_the_workspace_holds_takes_the_separate_pass():
    # one-row segments on a 1200 x 4000 grid: 20 strips x 4000 segments = 80,000 wave records,
    # beyond the 65,536 the workspace holds, so the last launch runs plainly and the separate
    # pass reduces: the same numbers as mp_step + mp_diagnostics, sums included
    p, phi, mu = inputs.config_c2(n=(1200, 4000, 1))

    def setup(s):
        s.set_tile(256, 1, 1)

    _check(p, phi, mu, 2, setup, rel=0.0)
