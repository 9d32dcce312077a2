"""GPU parity of the step with the anti-trapping current (Eq. jatr) against the
oracle's ``step_antitrapping``, on the same seeded inputs, through the C ABI.

Sizes span several strips of the 2D kernels (60 columns for the step with the
current folded in, 62 x 12 for the separate correction kernel) with ragged
tails, one strip exactly, one row and a grid smaller than a strip; the cases
mix both potentials, N = 2 and 3, K = 2 and 3, periodic and zero-flux axes and
a temperature gradient.  FP64 is held to 1e-10 (the bar of the plain step),
FP32 to 1e-4.  In 2D the folded kernel (on = 1) and the step followed by the
correction kernel (on = 2) give the same bits.  The switch's interplay with the
launch options (two steps per launch, graphs) and the adjoint's refusal are
checked too.
"""
import zlib

import numpy as np
import pytest

from oracle import gp
from paper_2404_01035_amd import inputs
from test_gpu_parity import errs, nuclei_case, variant

pytestmark = pytest.mark.gpu


def oracle_run_at(phi, mu, n0, nsteps, p):
    for i in range(nsteps):
        phi, mu = gp.step_antitrapping(phi, mu, n0 + i, p)
    return phi, mu


def run_gpu_at(p, phi, mu, nsteps, step0=0, on=True, fuse=None, graph=None):
    from paper_2404_01035_amd.solver import Solver

    s = Solver(p)
    try:
        if fuse:
            s.set_fusion(fuse)
        if graph:
            s.set_graph(graph)
        s.set_antitrapping(on)
        s.load(phi, mu, step0)
        s.step(nsteps)
        return s.fields()
    finally:
        s.close()


CASES = {
    # name: (params kwargs, steps)
    "n2k2_periodic": (dict(dim=2, N=2, K=2, n=(130, 50, 1), bc=(0, 0, 0)), 120),
    "n3k3_ragged_noflux_y_gradient": (dict(dim=2, N=3, K=3, n=(197, 70, 1), bc=(0, 1, 0), G=2e-3), 120),
    "n3k2_noflux": (dict(dim=2, N=3, K=2, n=(77, 66, 1), bc=(1, 1, 0)), 120),
    "n2k3_noflux_x": (dict(dim=2, N=2, K=3, n=(65, 37, 1), bc=(1, 0, 0)), 120),
    "n3k3_obstacle": (dict(dim=2, N=3, K=3, n=(90, 61, 1), bc=(0, 1, 0), potential="obstacle"), 100),
    "n2k2_obstacle_aniso": (dict(dim=2, N=2, K=2, n=(64, 64, 1), bc=(0, 0, 0), potential="obstacle",
                                 delta=0.02), 100),
    "n3k3_aniso": (dict(dim=2, N=3, K=3, n=(150, 40, 1), bc=(0, 0, 0), delta=0.03), 100),
    # one 62-column strip exactly; one row over two strips; a grid smaller than one strip
    "n3k2_one_strip_periodic": (dict(dim=2, N=3, K=2, n=(62, 33, 1), bc=(0, 0, 0)), 60),
    "n2k2_one_row_63": (dict(dim=2, N=2, K=2, n=(63, 1, 1), bc=(1, 0, 0)), 60),
    "n2k3_tiny_3x2_noflux": (dict(dim=2, N=2, K=3, n=(3, 2, 1), bc=(1, 1, 0)), 60),
    # 3D (the correction kernel after each step)
    "3d_n2k2_noflux": (dict(dim=3, N=2, K=2, n=(37, 9, 21), bc=(1, 1, 1)), 40),
    "3d_n3k3_mixed_bc_gradient": (dict(dim=3, N=3, K=3, n=(20, 13, 17), bc=(0, 1, 0), G=1e-3), 40),
    "3d_n2k3_periodic_obstacle_aniso": (dict(dim=3, N=2, K=3, n=(17, 11, 9), bc=(0, 0, 0), potential="obstacle",
                                             delta=0.02), 40),
}


def _case(name, precision="f64"):
    kw, steps = CASES[name]
    p = variant(seed=zlib.crc32(name.encode()) % 1000, precision=precision, **kw)
    phi, mu = nuclei_case(p, seed=9, count=6, radius=min(p.n[:p.dim]) / 4 + 2)
    return p, phi, mu, steps


@pytest.mark.parametrize("name", sorted(CASES))
def test_fp64_with_antitrapping_matches_oracle(name):
    p, phi, mu, steps = _case(name)
    print(f"case {name}: grid {p.n[:2]}, {steps} steps", flush=True)
    f, m = run_gpu_at(p, phi, mu, steps, step0=5)
    of, om = oracle_run_at(phi, mu, 5, steps, p)
    _, pm = gp.run(phi, mu, 5, steps, p)
    print(f"{name}: phi {errs(f, of):.3e} mu {errs(m, om):.3e}; the current moves mu by {errs(om, pm):.3e}")
    assert errs(f, of) <= 1e-10
    assert errs(m, om) <= 1e-10
    assert errs(om, pm) > 1e-6  # the case exercises the current


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_folded_current_is_bitwise_the_separate_correction(precision):
    """Every 2D case: the step with the current formed inside it against the
    step followed by the correction kernel, and the folded path again with a
    segment of 5 rows per wave (segment borders inside the grid) and as graphs."""
    from paper_2404_01035_amd import abi
    from paper_2404_01035_amd.solver import Solver

    for name in sorted(CASES):
        if CASES[name][0]["dim"] != 2:
            continue
        p, phi, mu, _ = _case(name, precision)
        steps = 23
        print(f"case {name} {precision}: folded vs separate, {steps} steps", flush=True)
        sep = run_gpu_at(p, phi, mu, steps, step0=5, on=2)
        f, m = run_gpu_at(p, phi, mu, steps, step0=5, on=1)
        assert np.array_equal(f, sep[0]) and np.array_equal(m, sep[1]), name
        s = Solver(p)
        try:
            s.set_antitrapping(1)
            bx, _, vec = abi.mp_get_tile(s.st)
            abi.mp_set_tile(s.st, bx, 5, vec)
            s.set_graph(6)
            s.load(phi, mu, 5)
            s.step(steps)
            f, m = s.fields()
        finally:
            s.close()
        assert np.array_equal(f, sep[0]) and np.array_equal(m, sep[1]), (name, "seg 5, graphs")


def test_c1_fp64_with_antitrapping_500_steps():
    p, phi, mu = inputs.config_c1(seed=0)
    f, m = run_gpu_at(p, phi, mu, 500)
    of, om = oracle_run_at(phi, mu, 0, 500, p)
    print(f"C1 FP64 500 steps with the current: phi {errs(f, of):.3e} mu {errs(m, om):.3e}")
    assert errs(f, of) <= 1e-10
    assert errs(m, om) <= 1e-10


@pytest.mark.parametrize("name", ["n2k2_periodic", "n3k3_ragged_noflux_y_gradient", "3d_n2k2_noflux",
                                  "3d_n3k3_mixed_bc_gradient"])
def test_fp32_with_antitrapping_matches_oracle(name):
    p, phi, mu, steps = _case(name, precision="f32")
    f, m = run_gpu_at(p, phi, mu, steps, step0=5)
    of, om = oracle_run_at(phi, mu, 5, steps, p)
    print(f"{name} FP32: phi {errs(f, of):.3e} mu {errs(m, om):.3e}")
    assert errs(f, of) <= 1e-4
    assert errs(m, om) <= 1e-4


def test_switch_overrides_fusion_and_graphs_and_switches_back():
    p, phi, mu, _ = _case("n3k2_noflux")
    steps = 37
    ref = run_gpu_at(p, phi, mu, steps)
    for fuse, graph in ((2, None), (1, 8), (2, 4)):
        f, m = run_gpu_at(p, phi, mu, steps, fuse=fuse, graph=graph)
        assert np.array_equal(f, ref[0]) and np.array_equal(m, ref[1]), (fuse, graph)
    # off again: the plain step, bitwise
    from test_gpu_parity import run_gpu

    plain = run_gpu(p, phi, mu, steps, fuse=2)
    f, m = run_gpu_at(p, phi, mu, steps, on=False, fuse=2)
    assert np.array_equal(f, plain[0]) and np.array_equal(m, plain[1])


def test_adjoint_refuses_the_antitrapping_current():
    import torch

    from paper_2404_01035_amd import abi
    from paper_2404_01035_amd.solver import Solver

    p, phi, mu = inputs.config_c1(seed=0)
    s = Solver(p)
    try:
        s.set_antitrapping(True)
        assert abi.mp_get_antitrapping(s.st)
        s.load(phi, mu)
        ckpt = s.checkpoint_buffer(4, 2)
        s.step_ckpt(4, 2, ckpt)
        lam = torch.zeros(p.nfields * p.ncells, dtype=s.dtype).cuda()
        with pytest.raises(Exception, match="anti-trapping"):
            s.adjoint(lam, ckpt, 4, 2, 0)
    finally:
        s.close()


@pytest.mark.parametrize("precision,mass_tol", [("f64", 1e-12), ("f32", 1e-7)])
def test_c2_full_grid_with_current_conserves_solute(precision, mass_tol):
    # At 4096^2 (the benchmark's grid) the current is a divergence, so the solute
    # sum c = sum_a h_a c^a(mu) stays fixed up to rounding, as without it.
    from paper_2404_01035_amd.solver import Solver

    p, phi, mu = inputs.config_c2(precision=precision)
    s = Solver(p)
    try:
        s.set_antitrapping(True)
        s.load(phi, mu)
        del phi, mu
        d0 = s.diagnostics()
        s.step(200)
        d1 = s.diagnostics()
    finally:
        s.close()
    drift = [abs(d1["mass"][k] - d0["mass"][k]) / abs(d0["mass"][k]) for k in range(2)]
    print(f"C2 {precision} with the current, 200 steps: mass drift {drift[0]:.2e} {drift[1]:.2e}")
    assert max(drift) <= mass_tol
    assert d1["nonfinite"] == 0
    assert d1["max_sum_dev"] <= (1e-12 if precision == "f64" else 1e-4)


@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 2e-6)])
def test_c2_full_grid_sampled_step_with_current(precision, tol):
    # The benchmark's grid and launch: one step with the current from the seeded
    # input as loaded, checked window by window against the oracle's windowed step
    # (windows on the correction strips' column and 12-row borders, the grid's
    # edges and across the slab's interface).
    from paper_2404_01035_amd import abi
    from paper_2404_01035_amd.solver import Solver
    from test_gpu_fullsize import _as_loaded, _slab_windows, _windows_2d

    p, phi, mu = inputs.config_c2(precision=precision)
    s = Solver(p)
    try:
        s.set_antitrapping(True)
        seg = abi.mp_get_tile(s.st)[1]
        s.load(phi, mu)
        s.step(1)
        gphi, gmu = s.fields()
    finally:
        s.close()
    phi0, mu0 = _as_loaded(phi, mu, precision)
    del phi, mu
    # the folded kernel's strips: 60 columns by the state's segment of rows
    w = _windows_2d(4096, 4096, np.random.default_rng(11), tile_x=60, seg=seg) + _slab_windows(4096)
    worst = [0.0, 0.0, 0.0]
    for lo, hi in w:
        of, om = gp.step_antitrapping_window(phi0, mu0, 0, p, lo, hi)
        _, pm = gp.step_window(phi0, mu0, 0, p, lo, hi)
        sl = (slice(None),) + tuple(slice(a, b) for a, b in zip(lo, hi))
        ef, em = errs(gphi[sl], of), errs(gmu[sl], om)
        worst = [max(worst[0], ef), max(worst[1], em), max(worst[2], errs(om, pm))]
        assert ef <= tol and em <= tol, (lo, hi, ef, em)
    print(f"C2 {precision} with the current, one step: worst window error phi {worst[0]:.2e} mu {worst[1]:.2e}; "
          f"the current moves mu by up to {worst[2]:.2e} there")
    assert worst[2] > 1e-8  # the windows see the current


def _batch_at(members, nsteps, step0=0, seg=None, vec=0, graph=0):
    from paper_2404_01035_amd.solver import BatchSolver

    b = BatchSolver([m[0] for m in members])
    try:
        if seg or vec:
            b.set_tile(seg or 0, vec)
        if graph:
            b.set_graph(graph)
        b.set_antitrapping(True)
        for i, (_, phi, mu) in enumerate(members):
            b.load(i, phi, mu)
        b.start(step0)
        b.step(nsteps)
        return [b.fields(i) for i in range(len(members))]
    finally:
        b.close()


def test_batch_with_current_matches_oracle_fp64():
    """Four uneven instances (N, K, boundaries and a temperature gradient mixed) in one
    batched launch per step with the current folded in, against the oracle."""
    rng = np.random.default_rng(41)
    members = []
    for (nx, ny, N, K, bc) in [(70, 50, 2, 2, (1, 1, 0)), (130, 64, 3, 3, (0, 1, 0)), (64, 90, 3, 2, (1, 0, 0)),
                               (66, 66, 2, 3, (0, 0, 0))]:
        p, phi, mu = inputs.random_instance(rng, nx, ny, N, K, precision="f64", nuclei=4)
        p.bc = bc
        p.G, p.V, p.y0 = 2e-3, 0.05, ny / 3
        members.append((p, phi, mu))
    steps = 60
    print(f"batch of {len(members)} with the current, {steps} steps", flush=True)
    got = _batch_at(members, steps, step0=5)
    for i, (p, phi, mu) in enumerate(members):
        of, om = oracle_run_at(phi, mu, 5, steps, p)
        _, pm = gp.run(phi, mu, 5, steps, p)
        print(f"  instance {i}: phi {errs(got[i][0], of):.3e} mu {errs(got[i][1], om):.3e}; "
              f"the current moves mu by {errs(om, pm):.3e}")
        assert errs(got[i][0], of) <= 1e-10, i
        assert errs(got[i][1], om) <= 1e-10, i
        assert errs(om, pm) > 1e-6, i


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_batch_with_current_is_bitwise_the_single_grid(precision):
    """Each batched instance against the same instance stepped alone with the current
    folded in; again with 7-row segments and graphs, and with two cells per lane
    (each work item then runs as two strips)."""
    members = inputs.config_c4(ninst=6, seed=23, precision=precision, side=(64, 200))
    steps = 20
    refs = [run_gpu_at(p, phi, mu, steps, step0=3) for (p, phi, mu) in members]
    for seg, vec, graph in [(None, 0, 0), (7, 0, 4), (None, 2, 0)]:
        print(f"batch {precision}: seg {seg} vec {vec} graph {graph}", flush=True)
        got = _batch_at(members, steps, step0=3, seg=seg, vec=vec, graph=graph)
        for i in range(len(members)):
            assert np.array_equal(got[i][0], refs[i][0]), (seg, vec, graph, i)
            assert np.array_equal(got[i][1], refs[i][1]), (seg, vec, graph, i)
