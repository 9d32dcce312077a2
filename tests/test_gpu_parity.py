"""GPU (HIP, through the C ABI) against the FP64 oracle on the same seeded inputs.

FP64 bar: max abs error <= 1e-10 on every phi_a and mu_k (1000 steps on C1).
FP32 bar: phi within 1e-4 of the FP64 oracle, relative solute-mass drift <= 1e-7.
"""
import zlib

import numpy as np
import pytest

from oracle import gp
from paper_2404_01035_amd import abi, inputs

pytestmark = pytest.mark.gpu


def run_gpu(p, phi, mu, nsteps, step0=0, tile=None, fuse=None):
    from paper_2404_01035_amd.solver import Solver

    s = Solver(p)
    try:
        if fuse:
            s.set_fusion(fuse)
        if tile:
            s.set_tile(*tile)
        s.load(phi, mu, step0)
        s.step(nsteps)
        return s.fields()
    finally:
        s.close()


def errs(a, b):
    return float(np.max(np.abs(a - b)))


def nuclei_case(p, seed, count=5, radius=6.0):
    rng = np.random.default_rng(seed)
    L = [p.n[i] * p.dx for i in range(p.dim)]
    centres = [tuple(rng.uniform(0, L[i]) for i in range(p.dim)) for _ in range(count)]
    phases = [int(rng.integers(0, p.nphases - 1)) for _ in range(count)]
    phi, mu = inputs.nuclei_initial(p, centres, [radius] * count, phases)
    mu = mu + rng.uniform(-0.02, 0.02, size=mu.shape)
    return phi, mu


def variant(dim, N, K, n, bc, potential="well", delta=0.0, undercooling=0.15, G=0.0,
            precision="f64", seed=0):
    rng = np.random.default_rng(100 + seed)
    p = inputs.Params(dim=dim, n=n, bc=bc, nphases=N, ncomp=K, precision=precision,
                      potential=potential)
    for a in range(N):
        for b in range(a + 1, N):
            p.gamma[a, b] = p.gamma[b, a] = rng.uniform(0.6, 1.6)
            p.delta[a, b] = p.delta[b, a] = delta
    p.gamma3 = 0.0
    K1 = K - 1
    A = rng.uniform(0.5, 2.0, size=(N, K1))
    ceq = rng.uniform(0.1, 0.9, size=(N, K1))
    B, C = inputs.parabolic_coefficients(A, ceq, liquid=N - 1)
    p.A[:N, :K1], p.B[:N, :K1], p.C[:N] = A, B, C
    p.s[:N] = 1.0
    p.s[N - 1] = 0.0
    p.D[:N, :K1] = rng.uniform(0.05, 0.3, size=(N, K1))
    p.D[N - 1, :K1] = 1.0
    p.Te, p.T0, p.G, p.V, p.y0 = 1.0, 1.0 - undercooling, G, 0.02, 0.3 * n[1]
    p.dt = 0.2 * inputs.dt_limit(p)
    return p


@pytest.mark.parametrize("fuse", [1, 2])
def test_c1_fp64_1000_steps_matches_oracle(fuse):
    p, phi, mu = inputs.config_c1(seed=0)
    f, m = run_gpu(p, phi, mu, 1000, fuse=fuse)
    of, om = gp.run(phi, mu, 0, 1000, p)
    print(f"C1 FP64 1000 steps, {fuse} per launch: phi {errs(f, of):.3e} mu {errs(m, om):.3e}")
    assert errs(f, of) <= 1e-10
    assert errs(m, om) <= 1e-10


VARIANTS = {
    # name: (params kwargs, steps)
    "2d_n3k3_ragged_noflux_y": (dict(dim=2, N=3, K=3, n=(300, 70, 1), bc=(0, 1, 0), G=2e-3), 200),
    "2d_n2k3_periodic": (dict(dim=2, N=2, K=3, n=(130, 50, 1), bc=(0, 0, 0)), 200),
    "2d_n3k2_noflux": (dict(dim=2, N=3, K=2, n=(77, 66, 1), bc=(1, 1, 0)), 200),
    "2d_n3k3_aniso": (dict(dim=2, N=3, K=3, n=(150, 40, 1), bc=(0, 0, 0), delta=0.03), 150),
    "2d_n2k2_aniso_noflux": (dict(dim=2, N=2, K=2, n=(70, 45, 1), bc=(1, 1, 0), delta=0.05), 150),
    "2d_n3k3_obstacle": (dict(dim=2, N=3, K=3, n=(90, 60, 1), bc=(0, 1, 0), potential="obstacle"), 150),
    "2d_n2k2_obstacle_aniso": (dict(dim=2, N=2, K=2, n=(64, 64, 1), bc=(0, 0, 0), potential="obstacle", delta=0.02), 150),
    "3d_n2k2_aniso_noflux": (dict(dim=3, N=2, K=2, n=(70, 9, 21), bc=(1, 1, 1), delta=0.02), 80),
    "3d_n3k3_mixed_bc": (dict(dim=3, N=3, K=3, n=(20, 13, 17), bc=(0, 1, 0), G=1e-3), 80),
    "3d_n3k2_obstacle_aniso": (dict(dim=3, N=3, K=2, n=(17, 11, 9), bc=(1, 0, 1), potential="obstacle", delta=0.03), 60),
    "3d_n2k3_periodic": (dict(dim=3, N=2, K=3, n=(66, 5, 7), bc=(0, 0, 0)), 60),
}


@pytest.mark.parametrize("name", sorted(VARIANTS))
def test_fp64_variant_matches_oracle(name):
    kw, steps = VARIANTS[name]
    p = variant(seed=zlib.crc32(name.encode()) % 1000, **kw)
    phi, mu = nuclei_case(p, seed=7, count=6, radius=min(p.n[:p.dim]) / 4 + 2)
    f, m = run_gpu(p, phi, mu, steps, step0=11)
    of, om = gp.run(phi, mu, 11, steps, p)
    print(f"{name}: phi {errs(f, of):.3e} mu {errs(m, om):.3e}")
    assert errs(f, of) <= 1e-10
    assert errs(m, om) <= 1e-10


@pytest.mark.parametrize("name", ["2d_n3k3_ragged_noflux_y", "2d_n3k3_aniso", "3d_n3k2_obstacle_aniso",
                                  "3d_n3k3_mixed_bc"])
def test_fp64_random_fields_few_steps(name):
    """Random phase fields (large gradients everywhere) exercise every term at once."""
    kw, _ = VARIANTS[name]
    p = variant(seed=3, **kw)
    phi, mu = inputs.random_multiphase(p, seed=5)
    f, m = run_gpu(p, phi, mu, 5, step0=2)
    of, om = gp.run(phi, mu, 2, 5, p)
    assert errs(f, of) <= 1e-12
    assert errs(m, om) <= 1e-12


@pytest.mark.parametrize("n", [(1, 5, 1), (2, 3, 1), (3, 1, 1), (1, 1, 1), (5, 1, 1)])
def test_tiny_grids(n):
    p = variant(dim=2, N=3, K=3, n=n, bc=(0, 0, 0))
    phi, mu = inputs.random_multiphase(p, seed=1)
    f, m = run_gpu(p, phi, mu, 20)
    of, om = gp.run(phi, mu, 0, 20, p)
    assert errs(f, of) <= 1e-12 and errs(m, om) <= 1e-12


@pytest.mark.parametrize("n", [(1, 1, 4), (3, 2, 1), (65, 1, 3)])
def test_tiny_grids_3d(n):
    p = variant(dim=3, N=2, K=2, n=n, bc=(0, 1, 0), delta=0.02)
    phi, mu = inputs.random_multiphase(p, seed=2)
    f, m = run_gpu(p, phi, mu, 20)
    of, om = gp.run(phi, mu, 0, 20, p)
    assert errs(f, of) <= 1e-12 and errs(m, om) <= 1e-12


def test_zero_steps_is_identity():
    p, phi, mu = inputs.config_c1()
    f, m = run_gpu(p, phi, mu, 0)
    assert np.array_equal(f, phi) and np.array_equal(m, mu)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_tile_shape_invariance_bitwise(precision):
    p, phi, mu = inputs.config_c2(n=(300, 200, 1), precision=precision)
    ref = None
    for tile in [(256, 32, -1), (128, 7, 1), (64, 1, 2), (64, 500, 1), (256, 3, 2), (128, 9, 4),
                 (64, 64, 4)]:
        if precision == "f64" and tile[2] == 4:
            continue
        f, m = run_gpu(p, phi, mu, 30, tile=tile)
        if ref is None:
            ref = (f, m)
        else:
            assert np.array_equal(f, ref[0]) and np.array_equal(m, ref[1]), tile


@pytest.mark.parametrize("case", ["f64_n3k3", "f32_n2k2_tall", "f32_n3k2_tall"])
def test_tile_shape_invariance_bitwise_3d(case):
    prec, N, K, tall = {"f64_n3k3": ("f64", 3, 3, False), "f32_n2k2_tall": ("f32", 2, 2, True),
                        "f32_n3k2_tall": ("f32", 3, 2, True)}[case]
    p = variant(dim=3, N=N, K=K, n=(70, 13, 40), bc=(0, 1, 1), delta=0.02, precision=prec)
    phi, mu = nuclei_case(p, seed=3)
    tiles = [(256, 16), (256, 1), (256, 5), (256, 64)]
    if tall:  # 64 x 8 tiles exist where their LDS ring is small enough
        tiles += [(512, 3), (512, 16), (512, 64)]
    ref = None
    for tile in tiles:
        f, m = run_gpu(p, phi, mu, 10, tile=tile)
        if ref is None:
            ref = (f, m)
        else:
            assert np.array_equal(f, ref[0]) and np.array_equal(m, ref[1]), tile
    if tall:  # and the tall tile against the oracle
        of, om = gp.run(phi, mu, 0, 10, p)
        assert np.max(np.abs(f - of)) <= 2e-5 and np.max(np.abs(m - om)) <= 2e-5


def test_run_to_run_bitwise():
    p, phi, mu = inputs.config_c2(n=(260, 100, 1))
    a = run_gpu(p, phi, mu, 40)
    b = run_gpu(p, phi, mu, 40)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_steps_split_equals_one_call():
    from paper_2404_01035_amd.solver import Solver

    p, phi, mu = inputs.config_c2(n=(128, 96, 1))
    s = Solver(p)
    s.load(phi, mu)
    s.step(7)
    s.step(0)
    s.step(13)
    f1, m1 = s.fields()
    assert s.time_level == 20
    s.close()
    f2, m2 = run_gpu(p, phi, mu, 20)
    assert np.array_equal(f1, f2) and np.array_equal(m1, m2)


# ----------------------------------------------------------------------------
# FP32 storage and arithmetic (FP64 Lagrange multiplier and reductions)
# ----------------------------------------------------------------------------

def test_c1_fp32_against_fp64_oracle():
    from paper_2404_01035_amd.solver import Solver

    p, phi, mu = inputs.config_c1(seed=0)
    p = p.copy(precision="f32")
    s = Solver(p)
    s.load(phi, mu)
    d0 = s.diagnostics()
    s.step(1000)
    d1 = s.diagnostics()
    f, m = s.fields()
    s.close()
    of, om = gp.run(phi, mu, 0, 1000, p.copy(precision="f64"))
    drift = abs(d1["mass"][0] - d0["mass"][0]) / abs(d0["mass"][0])
    print(f"C1 FP32: phi err {errs(f, of):.3e}, mu err {errs(m, om):.3e}, mass drift {drift:.3e}")
    assert errs(f, of) <= 1e-4
    assert errs(m, om) <= 1e-4
    assert drift <= 1e-7


def test_eutectic_fp32_mass_drift():
    from paper_2404_01035_amd.solver import Solver

    p, phi, mu = inputs.config_c2(n=(512, 256, 1), precision="f32")
    s = Solver(p)
    s.load(phi, mu)
    d0 = s.diagnostics()
    s.step(2000)
    d1 = s.diagnostics()
    s.close()
    for k in range(2):
        # mu starts at 0, so compare the drift to the solute content itself
        drift = abs(d1["mass"][k] - d0["mass"][k]) / abs(d0["mass"][k])
        assert drift <= 1e-7, (k, drift)
    # each FP32 update of phi_a rounds independently: sum phi - 1 random-walks by about
    # 2^-24 sqrt(N steps) per cell; 2e-4 leaves room for the max over 131k cells
    assert d1["max_sum_dev"] < 2e-4


# ----------------------------------------------------------------------------
# Diagnostics reduction
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_diagnostics_match_oracle(precision):
    from paper_2404_01035_amd.solver import Solver

    p, phi, mu = inputs.config_c2(n=(333, 217, 1), precision=precision)
    phi2, mu2 = inputs.random_multiphase(p, seed=4, amp=0.3)
    phi = 0.5 * (phi + phi2)
    mu = mu + mu2
    s = Solver(p)
    s.load(phi, mu)
    g = s.diagnostics()
    s.close()
    # the input as the GPU holds it: rounded to FP32 on the host in that precision
    if precision == "f32":
        hphi, hmu = phi.astype(np.float32).astype(np.float64), mu.astype(np.float32).astype(np.float64)
    else:
        hphi, hmu = phi, mu
    o = gp.diagnostics(hphi, hmu, p)
    assert g["nonfinite"] == 0
    for k in range(2):
        assert abs(g["mass"][k] - o["mass"][k]) <= 1e-12 * abs(o["mass"][k])
        assert abs(g["min_chi"][k] - o["min_chi"][k]) <= 1e-14
    for a in range(3):
        assert abs(g["volume"][a] - o["volume"][a]) <= 1e-12 * abs(o["volume"][a])
    assert abs(g["max_sum_dev"] - o["max_sum_dev"]) <= 1e-15


def test_diagnostics_flag_nonfinite():
    from paper_2404_01035_amd.solver import Solver

    p, phi, mu = inputs.config_c1()
    phi = phi.copy()
    phi[0, 3, 5] = np.nan
    mu = mu.copy()
    mu[0, 60, 1] = np.inf
    s = Solver(p)
    s.load(phi, mu)
    with pytest.raises(abi.MPError) as ei:
        s.diagnostics()
    assert ei.value.code == abi.MP_E_NONFINITE
    d = s.diagnostics(allow_nonfinite=True)
    assert d["nonfinite"] == 2
    s.close()


def test_diagnostics_bitwise_reproducible():
    from paper_2404_01035_amd.solver import Solver

    p, phi, mu = inputs.config_c2(n=(1000, 300, 1))
    s = Solver(p)
    s.load(phi, mu)
    s.step(5)
    a = s.diagnostics()
    b = s.diagnostics()
    s.close()
    assert a == b
