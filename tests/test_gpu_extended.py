"""GPU parity of the extended model's general kernels (through the C ABI) with the
FP64 oracle on the same seeded inputs: temperature-dependent parabolic
coefficients with the dT/dt term (Sec. 3, Eq. Mu_explicit_temperature), the
obstacle with the multiplier over the active phases and per-pair relaxation
constants (Eq. Obstacle, the Tau key of Sec. 5), off-diagonal curvatures and
diffusivities (Eq. free_energy_density, Eq. Mass_conservation), in 2D (one and
two steps per launch, graphs) and 3D, FP64 to 1e-10 and FP32 to 1e-4; the
anti-trapping current of Eq. jatr with the extended model (2D folded into the
step and as a correction kernel, bitwise equal; 3D); and the moving frame (SHIFT): the front row and the shift against the
oracle's, and runs with shifts (with and without the current) against the
oracle's runs in the shifted frame."""
import zlib

import numpy as np
import pytest

from oracle import gp
from paper_2404_01035_amd import abi, inputs

pytestmark = pytest.mark.gpu


def extended(dim, N, K, n, bc, potential="well", delta=0.0, slopes=True, offdiag=True, tau_pairs=True,
             G=4e-3, V=0.5, undercooling=0.1, precision="f64", seed=0):
    rng = np.random.default_rng(300 + seed)
    K1 = K - 1
    p = inputs.Params(dim=dim, n=n, bc=bc, nphases=N, ncomp=K, precision=precision, potential=potential)
    for a in range(N):
        for b in range(a + 1, N):
            p.gamma[a, b] = p.gamma[b, a] = rng.uniform(0.6, 1.6)
            p.delta[a, b] = p.delta[b, a] = delta
            if tau_pairs:
                p.tau_ab[a, b] = p.tau_ab[b, a] = rng.uniform(0.6, 1.8)
    A = rng.uniform(0.6, 2.0, size=(N, K1))
    ceq = rng.uniform(0.1, 0.9, size=(N, K1))
    A01 = rng.uniform(-0.4, 0.4, size=N) if (offdiag and K1 == 2) else np.zeros(N)
    sl = rng.uniform(2.0, 6.0, size=(N, K1)) * rng.choice([-1.0, 1.0], size=(N, K1)) if slopes \
        else np.full((N, K1), np.inf)
    B, Bt, C, s, Ct = inputs.parabolic_coefficients_T(A, ceq, sl, liquid=N - 1, A01=A01)
    p.A[:N, :K1], p.B[:N, :K1], p.C[:N] = A, B, C
    p.Bt[:N, :K1], p.s[:N], p.Ct[:N] = Bt, s, Ct
    p.A01[:N] = A01
    p.D[:N, :K1] = rng.uniform(0.05, 0.3, size=(N, K1))
    p.D[N - 1, :K1] = 1.0
    if offdiag and K1 == 2:
        p.D01[:N] = rng.uniform(-0.5, 0.5, size=N) * np.sqrt(p.D[:N, 0] * p.D[:N, 1])
    p.Te, p.T0, p.G, p.V, p.y0 = 1.0, 1.0 - undercooling, G, V, 0.4 * n[1]
    p.dt = 0.2 * inputs.dt_limit(p)
    return p


def nuclei(p, seed, count=6):
    rng = np.random.default_rng(seed)
    L = [p.n[i] * p.dx for i in range(p.dim)]
    centres = [tuple(rng.uniform(0, L[i]) for i in range(p.dim)) for _ in range(count)]
    phases = [int(rng.integers(0, p.nphases - 1)) for _ in range(count)]
    radius = min(p.n[:p.dim]) / 4 + 2
    phi, mu = inputs.nuclei_initial(p, centres, [radius] * count, phases)
    return phi, mu + rng.uniform(-0.02, 0.02, size=mu.shape)


def run_gpu(p, phi, mu, nsteps, step0=0, fuse=None, graph=0):
    from paper_2404_01035_amd.solver import Solver

    s = Solver(p)
    try:
        if fuse:
            s.set_fusion(fuse)
        if graph:
            s.set_graph(graph)
        s.load(phi, mu, step0)
        s.step(nsteps)
        return s.fields()
    finally:
        s.close()


def errs(a, b):
    return float(np.max(np.abs(a - b)))


CASES = {
    # name: (extended() kwargs, steps)
    "2d_n3k3_all_noflux_y": (dict(dim=2, N=3, K=3, n=(130, 70, 1), bc=(0, 1, 0)), 200),
    "2d_n3k3_slopes_only": (dict(dim=2, N=3, K=3, n=(90, 64, 1), bc=(0, 1, 0), offdiag=False, tau_pairs=False), 200),
    "2d_n3k3_offdiag_only": (dict(dim=2, N=3, K=3, n=(77, 50, 1), bc=(0, 0, 0), slopes=False, tau_pairs=False), 200),
    "2d_n3k2_taupairs_aniso": (dict(dim=2, N=3, K=2, n=(70, 45, 1), bc=(1, 1, 0), delta=0.03, slopes=False), 150),
    "2d_n3k3_active_obstacle": (dict(dim=2, N=3, K=3, n=(90, 60, 1), bc=(0, 1, 0), potential="obstacle_active"), 150),
    "2d_n3k3_clip_obstacle_ext": (dict(dim=2, N=3, K=3, n=(66, 40, 1), bc=(1, 0, 0), potential="obstacle"), 150),
    "2d_n2k3_active_aniso": (dict(dim=2, N=2, K=3, n=(64, 64, 1), bc=(0, 0, 0), potential="obstacle_active",
                                  delta=0.02), 150),
    "3d_n3k3_all_mixed_bc": (dict(dim=3, N=3, K=3, n=(20, 13, 17), bc=(0, 1, 0)), 60),
    "3d_n3k2_active_aniso": (dict(dim=3, N=3, K=2, n=(17, 11, 9), bc=(1, 0, 1), potential="obstacle_active",
                                  delta=0.03), 50),
    "3d_n2k3_offdiag_periodic": (dict(dim=3, N=2, K=3, n=(66, 5, 7), bc=(0, 0, 0)), 50),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_fp64_extended_matches_oracle(name):
    kw, steps = CASES[name]
    p = extended(seed=zlib.crc32(name.encode()) % 1000, **kw)
    phi, mu = nuclei(p, seed=9)
    of, om = gp.run(phi, mu, 7, steps, p)
    fuses = [1, 2] if p.dim == 2 else [1]
    for fuse in fuses:
        print(f"{name}: {steps} steps, {fuse} per launch", flush=True)
        f, m = run_gpu(p, phi, mu, steps, step0=7, fuse=fuse)
        print(f"  phi {errs(f, of):.3e} mu {errs(m, om):.3e}", flush=True)
        assert errs(f, of) <= 1e-10
        assert errs(m, om) <= 1e-10


@pytest.mark.parametrize("name", ["2d_n3k3_all_noflux_y", "2d_n3k3_active_obstacle", "3d_n3k3_all_mixed_bc"])
def test_fp64_extended_random_fields_few_steps(name):
    """Random phase fields (large gradients everywhere) exercise every term at once."""
    kw, _ = CASES[name]
    p = extended(seed=4, **kw)
    phi, mu = inputs.random_multiphase(p, seed=5)
    of, om = gp.run(phi, mu, 3, 5, p)
    for fuse in ([1, 2] if p.dim == 2 else [1]):
        f, m = run_gpu(p, phi, mu, 5, step0=3, fuse=fuse)
        assert errs(f, of) <= 1e-12
        assert errs(m, om) <= 1e-12


@pytest.mark.parametrize("name", ["2d_n3k3_all_noflux_y", "3d_n3k3_all_mixed_bc"])
def test_fp32_extended_within_1e4_of_fp64_oracle(name):
    kw, steps = CASES[name]
    p = extended(seed=zlib.crc32(name.encode()) % 1000, precision="f32", **kw)
    phi, mu = nuclei(p, seed=9)
    f, m = run_gpu(p, phi, mu, steps, step0=7)
    of, om = gp.run(phi, mu, 7, steps, p)
    print(f"{name} FP32: phi {errs(f, of):.3e} mu {errs(m, om):.3e}")
    assert errs(f, of) <= 1e-4
    assert errs(m, om) <= 1e-4


def test_graphs_and_two_steps_are_bitwise_the_single_launch_path():
    p = extended(dim=2, N=3, K=3, n=(100, 80, 1), bc=(0, 1, 0), seed=2)
    phi, mu = nuclei(p, seed=3)
    ref = run_gpu(p, phi, mu, 24, fuse=1)
    for fuse, graph in [(2, 0), (2, 8), (1, 6)]:
        f, m = run_gpu(p, phi, mu, 24, fuse=fuse, graph=graph)
        assert np.array_equal(f, ref[0]) and np.array_equal(m, ref[1]), (fuse, graph)


def test_c2_slopes_conserves_solute_on_gpu():
    """The directional eutectic with temperature-dependent coefficients: the device
    diagnostics' solute mass (with B at each row's T) stays put over 400 steps."""
    from paper_2404_01035_amd.solver import Solver

    p, phi, mu = inputs.config_c2_slopes(precision="f64", n=(256, 192, 1))
    s = Solver(p)
    s.load(phi, mu)
    d0 = s.diagnostics()
    o0 = gp.diagnostics(phi, mu, p, n=0)
    for k in range(2):
        assert abs(d0["mass"][k] - o0["mass"][k]) <= 1e-12 * abs(o0["mass"][k])
    s.step(400)
    d1 = s.diagnostics()
    s.close()
    for k in range(2):
        assert abs(d1["mass"][k] - d0["mass"][k]) <= 1e-12 * abs(d0["mass"][k]), (k, d0, d1)


def test_front_row_and_shift_match_the_oracle():
    from paper_2404_01035_amd.solver import Solver

    for precision in ("f64", "f32"):
        p, phi, mu = inputs.config_c2_slopes(precision=precision, n=(96, 80, 1))
        s = Solver(p)
        s.load(phi, mu)
        s.step(10)
        f, m = s.fields()
        assert s.front_row() == gp.front_row(f)
        melt = [0.013, -0.021]
        assert s.shift(7, melt) == 7
        sf, sm = s.fields()
        of, om = gp.shift(f, m, 7, np.array(melt, dtype=np.float32 if precision == "f32" else np.float64))
        assert np.array_equal(sf, of) and np.array_equal(sm, om)
        assert s.shift(0, melt) == 7
        s.close()


@pytest.mark.parametrize("fuse", [1, 2])
def test_moving_frame_run_matches_oracle(fuse):
    """Steps, shifts whenever the front passes row shiftj, more steps: against the
    oracle stepping the same frames (the temperature law follows the offset)."""
    from paper_2404_01035_amd.solver import Solver

    p, phi, mu = inputs.config_c2_slopes(precision="f64", n=(64, 48, 1))
    p.V = 2.0  # a fast pull so the front moves within the run
    p.dt = 0.2 * inputs.dt_limit(p)
    melt = np.array([0.0, 0.0])
    shiftj, every, nsteps = 5, 20, 120  # the slab's top starts near row 8: the first check shifts
    s = Solver(p)
    s.set_fusion(fuse)
    s.load(phi, mu)
    off = s.step_moving_frame(nsteps, shiftj, every, melt)
    f, m = s.fields()
    s.close()
    of, om, ooff = phi, mu, 0
    for i in range(0, nsteps, every):
        of, om = gp.run(of, om, i, every, p, y_origin=ooff)
        front = gp.front_row(of)
        if front > shiftj:
            of, om = gp.shift(of, om, front - shiftj, melt)
            ooff += front - shiftj
    print(f"moving frame: offset {off}, phi {errs(f, of):.3e} mu {errs(m, om):.3e}")
    assert off == ooff and off > 0
    assert errs(f, of) <= 1e-10 and errs(m, om) <= 1e-10


def test_extended_model_switches():
    p = extended(dim=2, N=3, K=3, n=(32, 24, 1), bc=(0, 0, 0))
    st = abi.mp_create(p)
    try:
        # the anti-trapping current takes the extended model in both of its forms
        for on in (2, 1, 0):
            abi.mp_set_antitrapping(st, on)
            assert abi.mp_get_antitrapping(st) == on
    finally:
        abi.mp_destroy(st)


def run_gpu_at(p, phi, mu, nsteps, step0=0, graph=0, on=1):
    from paper_2404_01035_amd.solver import Solver

    s = Solver(p)
    try:
        if graph:
            s.set_graph(graph)
        s.set_antitrapping(on)
        s.load(phi, mu, step0)
        s.step(nsteps)
        return s.fields()
    finally:
        s.close()


def oracle_run_at(phi, mu, n0, nsteps, p, y_origin=0):
    for i in range(nsteps):
        phi, mu = gp.step_antitrapping(phi, mu, n0 + i, p, y_origin)
    return phi, mu


@pytest.mark.parametrize("name", sorted(CASES))
def test_fp64_extended_with_antitrapping_matches_oracle(name):
    """The anti-trapping current with the general kernels: compositions at each
    row's temperature of time level n, the 2 x 2 susceptibility in the correction;
    in 2D folded into the step and, bit for bit the same, by the step followed by
    the correction kernel; in 3D by the correction kernel."""
    kw, steps = CASES[name]
    steps = min(steps, 120)
    p = extended(seed=zlib.crc32(name.encode()) % 1000, **kw)
    phi, mu = nuclei(p, seed=9)
    print(f"{name} with the current: {steps} steps", flush=True)
    f, m = run_gpu_at(p, phi, mu, steps, step0=7)
    of, om = oracle_run_at(phi, mu, 7, steps, p)
    _, pm = gp.run(phi, mu, 7, steps, p)
    print(f"  phi {errs(f, of):.3e} mu {errs(m, om):.3e}; the current moves mu by {errs(om, pm):.3e}", flush=True)
    assert errs(f, of) <= 1e-10
    assert errs(m, om) <= 1e-10
    assert errs(om, pm) > 1e-6
    if p.dim == 2:
        f2, m2 = run_gpu_at(p, phi, mu, steps, step0=7, on=2)
        assert np.array_equal(f2, f) and np.array_equal(m2, m)


def test_fp32_extended_with_antitrapping_and_graphs():
    kw, steps = CASES["2d_n3k3_all_noflux_y"]
    p = extended(seed=11, precision="f32", **kw)
    phi, mu = nuclei(p, seed=9)
    f, m = run_gpu_at(p, phi, mu, 100, step0=7)
    of, om = oracle_run_at(phi, mu, 7, 100, p)
    print(f"FP32 with the current: phi {errs(f, of):.3e} mu {errs(m, om):.3e}")
    assert errs(f, of) <= 1e-4 and errs(m, om) <= 1e-4
    g = run_gpu_at(p, phi, mu, 100, step0=7, graph=10)
    assert np.array_equal(g[0], f) and np.array_equal(g[1], m)


def test_moving_frame_with_antitrapping_matches_oracle():
    """Shifts of the frame with the current on: the compositions follow the frame's temperature."""
    from paper_2404_01035_amd.solver import Solver

    p, phi, mu = inputs.config_c2_slopes(precision="f64", n=(64, 48, 1))
    p.V = 2.0
    p.dt = 0.2 * inputs.dt_limit(p)
    melt = np.array([0.0, 0.0])
    shiftj, every, nsteps = 5, 20, 80
    s = Solver(p)
    s.set_antitrapping(True)
    s.load(phi, mu)
    off = s.step_moving_frame(nsteps, shiftj, every, melt)
    f, m = s.fields()
    s.close()
    of, om, ooff = phi, mu, 0
    for i in range(0, nsteps, every):
        of, om = oracle_run_at(of, om, i, every, p, y_origin=ooff)
        front = gp.front_row(of)
        if front > shiftj:
            of, om = gp.shift(of, om, front - shiftj, melt)
            ooff += front - shiftj
    print(f"moving frame with the current: offset {off}, phi {errs(f, of):.3e} mu {errs(m, om):.3e}")
    assert off == ooff and off > 0
    assert errs(f, of) <= 1e-10 and errs(m, om) <= 1e-10


# ----------------------------------------------------------------------------
# Batches of the extended model
# ----------------------------------------------------------------------------

def _ext_members(precision="f64"):
    """Uneven 2D instances of the extended model sharing one potential (multi-well)."""
    out = []
    specs = [dict(N=3, K=3, n=(130, 70, 1), bc=(0, 1, 0)),
             dict(N=3, K=3, n=(90, 64, 1), bc=(0, 1, 0), offdiag=False, tau_pairs=False),
             dict(N=3, K=3, n=(77, 50, 1), bc=(0, 0, 0), slopes=False, tau_pairs=False),
             dict(N=3, K=2, n=(70, 45, 1), bc=(1, 1, 0), tau_pairs=False),
             dict(N=2, K=3, n=(66, 61, 1), bc=(1, 0, 0))]
    for i, kw in enumerate(specs):
        p = extended(dim=2, seed=40 + i, precision=precision, **kw)
        phi, mu = nuclei(p, seed=50 + i)
        out.append((p, phi, mu))
    return out


def _batch_ext(members, nsteps, step0=0, on=0, fuse=None, vec=0):
    from paper_2404_01035_amd.solver import BatchSolver

    b = BatchSolver([m[0] for m in members])
    try:
        if fuse:
            abi.mp_set_fusion(b.st, fuse)
        if vec:
            b.set_tile(0, vec)
        if on:
            b.set_antitrapping(on)
        for i, (_, phi, mu) in enumerate(members):
            b.load(i, phi, mu)
        b.start(step0)
        b.step(nsteps)
        return [b.fields(i) for i in range(len(members))]
    finally:
        b.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_batch_of_the_extended_model_is_bitwise_the_single_grid(precision):
    """Each instance of an extended-model batch against the same instance stepped
    alone: two steps per launch, one, two cells per lane (two strips per item),
    and with the anti-trapping current."""
    members = _ext_members(precision)
    steps = 24
    refs = [run_gpu(p, phi, mu, steps, step0=5, fuse=2) for (p, phi, mu) in members]
    for fuse, vec in [(2, 0), (1, 0), (2, 2)]:
        print(f"extended batch {precision}: fuse {fuse} vec {vec}", flush=True)
        got = _batch_ext(members, steps, step0=5, fuse=fuse, vec=vec)
        for i in range(len(members)):
            assert np.array_equal(got[i][0], refs[i][0]), (fuse, vec, i)
            assert np.array_equal(got[i][1], refs[i][1]), (fuse, vec, i)
    refs = [run_gpu_at(p, phi, mu, steps, step0=5) for (p, phi, mu) in members]
    got = _batch_ext(members, steps, step0=5, on=1)
    for i in range(len(members)):
        assert np.array_equal(got[i][0], refs[i][0]), ("current", i)
        assert np.array_equal(got[i][1], refs[i][1]), ("current", i)


def test_batch_of_the_extended_model_matches_oracle_fp64():
    members = _ext_members("f64")
    steps = 60
    got = _batch_ext(members, steps, step0=5)
    got_at = _batch_ext(members, steps, step0=5, on=1)
    for i, (p, phi, mu) in enumerate(members):
        of, om = gp.run(phi, mu, 5, steps, p)
        af, am = oracle_run_at(phi, mu, 5, steps, p)
        print(f"instance {i}: phi {errs(got[i][0], of):.3e} mu {errs(got[i][1], om):.3e}; with the current "
              f"phi {errs(got_at[i][0], af):.3e} mu {errs(got_at[i][1], am):.3e}", flush=True)
        assert errs(got[i][0], of) <= 1e-10 and errs(got[i][1], om) <= 1e-10, i
        assert errs(got_at[i][0], af) <= 1e-10 and errs(got_at[i][1], am) <= 1e-10, i
