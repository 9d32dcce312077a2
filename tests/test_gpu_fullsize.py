"""Full-size checks in the benchmark's launch configuration.

The oracle cannot step a 4096^2 or 512^3 grid in a test, so one GPU step is
checked on sampled windows (corners, the solidification front, tile and
segment boundaries, random spots) against the oracle's windowed step from the
same GPU state; conservation and the phase-sum constraint are checked on the
whole grid through the diagnostics reduction.
"""
import numpy as np
import pytest

from oracle import gp
from paper_2404_01035_amd import inputs

pytestmark = pytest.mark.gpu


def _windows_2d(ny, nx, rng, tile_x=62, seg=16):
    w = [((0, 0), (8, 70)), ((ny - 8, nx - 70), (ny, nx)), ((56, 1000), (72, 1100)),
         ((0, nx - 40), (6, nx)), ((ny - 5, 0), (ny, 40))]
    for k in (1, 2, 31):  # strip borders (tile_x columns) and segment borders (seg rows)
        x = tile_x * k
        y = seg * k
        w.append(((y - 3, x - 4), (y + 3, x + 4)))
    for _ in range(4):
        y = int(rng.integers(0, ny - 8))
        x = int(rng.integers(0, nx - 64))
        w.append(((y, x), (y + 8, x + 64)))
    return w


def _check_windows(p, phi0, mu0, phi1, mu1, n, windows, tol):
    worst = (0.0, 0.0)
    for lo, hi in windows:
        of, om = gp.step_window(phi0, mu0, n, p, lo, hi)
        sl = (slice(None),) + tuple(slice(a, b) for a, b in zip(lo, hi))
        ef = float(np.max(np.abs(phi1[sl] - of)))
        em = float(np.max(np.abs(mu1[sl] - om)))
        worst = (max(worst[0], ef), max(worst[1], em))
        assert ef <= tol and em <= tol, (lo, hi, ef, em)
    return worst


def _as_loaded(phi, mu, precision):
    """The seeded input as the GPU holds it after ``load``: rounded to FP32 on the host
    in that precision (round to nearest, as the upload's cast), as float64 arrays."""
    if precision == "f32":
        return phi.astype(np.float32).astype(np.float64), mu.astype(np.float32).astype(np.float64)
    return phi, mu


def _slab_windows(nx):
    """Windows across the initial slab's top (y = 64): the solid-melt interface."""
    return [((58, 0), (70, 70)), ((58, 1000), (70, 1130)), ((58, nx - 70), (70, nx))]


def _state(s):
    import torch

    torch.cuda.synchronize()
    a = s.current().cpu().numpy()
    return a[: s.p.nphases], a[s.p.nphases:]


@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 2e-6)])
def test_c2_full_grid_sampled_step(precision, tol):
    from paper_2404_01035_amd.solver import Solver

    p, phi, mu = inputs.config_c2(precision=precision)
    s = Solver(p)
    s.set_fusion(1)
    s.load(phi, mu)
    s.step(1)
    phi1, mu1 = _state(s)
    s.close()
    # the oracle starts from the seeded input itself (as loaded), never from a GPU result
    phi0, mu0 = _as_loaded(phi, mu, precision)
    del phi, mu
    # one step per launch: 62-column strips, the default 31 (FP64) / 14 (FP32) row segments
    w = _windows_2d(4096, 4096, np.random.default_rng(3), seg=31 if precision == "f64" else 14)
    w += _slab_windows(4096)
    worst = _check_windows(p, phi0, mu0, phi1, mu1, 0, w, tol)
    print(f"C2 {precision}: worst window error phi {worst[0]:.2e} mu {worst[1]:.2e}")


@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 4e-6)])
def test_c2_full_grid_sampled_two_step_launch(precision, tol):
    """The launch bench.py times: one two-step launch of the default tile.  The oracle
    takes the first step on the whole grid and the second on the windows."""
    from paper_2404_01035_amd import abi
    from paper_2404_01035_amd.solver import Solver

    p, phi, mu = inputs.config_c2(precision=precision)
    s = Solver(p)
    s.load(phi, mu)
    assert abi.mp_get_fusion(s.st) == 2
    s.step(2)  # one launch of the two-step kernel
    phi2, mu2 = _state(s)
    s.close()
    phi0, mu0 = _as_loaded(phi, mu, precision)
    del phi, mu
    phi1, mu1 = gp.run(phi0, mu0, 0, 1, p)
    # the default two-step tiles: 60-column strips, 31 (FP64) / 14 (FP32) row segments
    w = _windows_2d(4096, 4096, np.random.default_rng(7), tile_x=60, seg=31 if precision == "f64" else 14)
    w += _slab_windows(4096)
    worst = _check_windows(p, phi1, mu1, phi2, mu2, 1, w, tol)
    print(f"C2 {precision} two-step launch: worst window error phi {worst[0]:.2e} mu {worst[1]:.2e}")


@pytest.mark.parametrize("precision,mass_tol", [("f64", 1e-12), ("f32", 1e-7)])
def test_c2_full_grid_conservation(precision, mass_tol):
    from paper_2404_01035_amd.solver import Solver

    p, phi, mu = inputs.config_c2(precision=precision)
    s = Solver(p)
    s.load(phi, mu)
    del phi, mu
    d0 = s.diagnostics()
    s.step(500)
    d1 = s.diagnostics()
    s.close()
    for k in range(2):
        drift = abs(d1["mass"][k] - d0["mass"][k]) / abs(d0["mass"][k])
        assert drift <= mass_tol, (k, drift)
    assert d1["nonfinite"] == 0
    assert d1["max_sum_dev"] <= (1e-12 if precision == "f64" else 1e-4)


def test_c3_full_grid_sampled_step():
    from paper_2404_01035_amd.solver import Solver

    p, phi, mu = inputs.config_c3()
    s = Solver(p)
    s.load(phi, mu)
    s.step(1)
    phi1, mu1 = _state(s)
    s.close()
    phi0, mu0 = _as_loaded(phi, mu, "f32")
    del phi, mu
    n0 = 0
    rng = np.random.default_rng(5)
    w = [((0, 0, 0), (12, 12, 12)),                 # the seeded octant corner
         ((500, 500, 500), (512, 512, 512)),        # far corner (mirror ghosts)
         ((14, 2, 62), (18, 6, 67)),                # x tile border (64)
         ((15, 3, 10), (17, 6, 14)),                # z segment border (16) and y border (4)
         ((0, 0, 0), (3, 3, 40)),
         ((5, 0, 0), (11, 11, 11))]                 # the seed's interface shell
    for _ in range(3):
        z, y, x = (int(v) for v in rng.integers(0, 500, size=3))
        w.append(((z, y, x), (z + 4, y + 4, x + 8)))
    worst = _check_windows(p, phi0, mu0, phi1, mu1, n0, w, 2e-6)
    print(f"C3 f32: worst window error phi {worst[0]:.2e} mu {worst[1]:.2e}")


def test_c4_full_batch_sampled_instances():
    """The full 256-instance ensemble in the benchmark's configuration (default tile, two
    steps per launch, HIP graphs of 50 steps): sampled instances equal the single-grid
    kernels bitwise, and the two smallest match the oracle."""
    from paper_2404_01035_amd import abi
    from paper_2404_01035_amd.solver import BatchSolver, Solver

    members = inputs.config_c4()
    nsteps = 4
    b = BatchSolver([m[0] for m in members])
    try:
        assert abi.mp_get_fusion(b.st) == 2
        b.set_graph(50)
        for i, (_, phi, mu) in enumerate(members):
            b.load(i, phi, mu)
        b.start(0)
        b.step(nsteps)
        rng = np.random.default_rng(9)
        cells = [m[0].ncells for m in members]
        order = np.argsort(cells)
        picks = sorted(set([int(order[0]), int(order[1]), int(order[-1])]
                           + [int(i) for i in rng.choice(len(members), 5, replace=False)]))
        got = {i: b.fields(i) for i in picks}
    finally:
        b.close()
    for i in picks:
        p, phi, mu = members[i]
        s = Solver(p)
        s.load(phi, mu)
        s.step(nsteps)
        ref = s.fields()
        s.close()
        assert np.array_equal(got[i][0], ref[0]) and np.array_equal(got[i][1], ref[1]), i
    for i in (int(order[0]), int(order[1])):
        p, phi, mu = members[i]
        p64 = p.copy(precision="f64")
        of, om = gp.run(phi.astype(np.float64), mu.astype(np.float64), 0, nsteps, p64)
        # FP32 state against the FP64 oracle over four steps
        assert np.max(np.abs(got[i][0] - of)) <= 1e-5, i
        assert np.max(np.abs(got[i][1] - om)) <= 1e-4, i


def _c5_adjoint(precision, target64, nsteps=2000, every=100):
    """The benchmark's C5 configuration: loss 1/2 |phi^N - phi*|^2 at nominal theta,
    checkpoints every 100 steps; returns (lambda^0, gradients, loss)."""
    import torch

    from paper_2404_01035_amd.solver import Solver

    p, phi, mu, _ = inputs.config_c5(precision=precision)
    s = Solver(p)
    try:
        s.load(phi, mu)
        ckpt = s.checkpoint_buffer(nsteps, every)
        s.step_ckpt(nsteps, every, ckpt)
        cur = s.current().double()
        lam = torch.zeros_like(cur)
        lam[: p.nphases] = cur[: p.nphases] - torch.from_numpy(target64).to(cur.device)
        loss = 0.5 * float((lam[: p.nphases] ** 2).sum())
        lam0, g = s.adjoint(lam, ckpt, nsteps, every, 0)
        return lam0.double().cpu().numpy(), g, loss
    finally:
        s.close()


def _c5_loss64(theta, target64, nsteps=2000):
    from paper_2404_01035_amd.solver import Solver

    p, phi, mu, _ = inputs.config_c5(precision="f64")
    s = Solver(inputs.theta_into(p, theta))
    try:
        s.load(phi, mu)
        s.step(nsteps)
        f, _ = s.fields()
        return 0.5 * float(np.sum((f - target64) ** 2))
    finally:
        s.close()


def test_c5_full_size_adjoint():
    """C5 at full size in the benchmark's configuration (512^2, 2000 steps,
    checkpoints every 100), where the oracle cannot go: the FP64 adjoint's tau and
    gamma_01 gradients against central differences of the FP64 loss, and the
    FP32 adjoint (the benchmarked one) against the FP64 adjoint."""
    from paper_2404_01035_amd.solver import Solver

    p, phi, mu, theta_star = inputs.config_c5(precision="f64")
    s = Solver(inputs.theta_into(p, theta_star))
    s.load(phi, mu)
    s.step(2000)
    target64, _ = s.fields()
    s.close()
    lam64, g64, loss64 = _c5_adjoint("f64", target64)
    lam32, g32, loss32 = _c5_adjoint("f32", target64)
    nominal = [1.0] * 6
    for idx, key in ((5, "tau"), (0, "gamma01")):
        h = 1e-4
        up = list(nominal)
        dn = list(nominal)
        up[idx] += h
        dn[idx] -= h
        fd = (_c5_loss64(up, target64) - _c5_loss64(dn, target64)) / (2 * h)
        rel = abs(g64[key] - fd) / abs(fd)
        print(f"C5 FP64 adjoint {key}: {g64[key]:.10g} vs central difference {fd:.10g} (rel {rel:.2e})")
        assert rel <= 1e-6, (key, g64[key], fd)  # measured 2e-8 (tau), 8e-9 (gamma01)
    worst = 0.0
    for key in ("gamma01", "gamma02", "gamma12", "D20", "D21", "tau"):
        rel = abs(g32[key] - g64[key]) / max(abs(g64[key]), 1e-3 * abs(g64["tau"]))
        worst = max(worst, rel)
    lam_rel = float(np.max(np.abs(lam32 - lam64)) / np.max(np.abs(lam64)))
    print(f"C5 FP32 vs FP64 adjoint: worst gradient rel {worst:.2e}, lambda^0 rel {lam_rel:.2e}, "
          f"loss {loss32:.6g} vs {loss64:.6g}")
    assert worst <= 1e-4 and lam_rel <= 1e-3  # measured 2.6e-6 and 7.1e-5


def test_c2_full_grid_fp32_against_fp64():
    """The FP32 path's error per field on the full C2 grid after 2000 steps, against
    the FP64 path (pinned to the oracle): phi within 1e-4."""
    from paper_2404_01035_amd.solver import Solver

    out = {}
    for precision in ("f64", "f32"):
        p, phi, mu = inputs.config_c2(precision=precision)
        s = Solver(p)
        s.load(phi, mu)
        del phi, mu
        s.step(2000)
        out[precision] = s.fields()
        s.close()
    ephi = float(np.max(np.abs(out["f32"][0] - out["f64"][0])))
    emu = float(np.max(np.abs(out["f32"][1] - out["f64"][1])))
    print(f"C2 4096^2, 2000 steps: FP32 - FP64 max |dphi| {ephi:.2e}, max |dmu| {emu:.2e}")
    assert ephi <= 1e-4  # measured 3.5e-5
    assert emu <= 1e-4   # measured 1.2e-5
