"""Two steps per launch (mp_set_fusion(2)) against single steps (bitwise) and the oracle."""
import numpy as np
import pytest

from oracle import gp
from paper_2404_01035_amd import inputs

pytestmark = pytest.mark.gpu


def _run(p, phi, mu, nsteps, fuse, tile=None, graph=0, step0=0, chunks=None):
    from paper_2404_01035_amd.solver import Solver

    s = Solver(p)
    try:
        if tile:
            s.set_tile(*tile)
        s.set_fusion(fuse)
        s.set_graph(graph)
        s.load(phi, mu, step0)
        for n in (chunks or [nsteps]):
            s.step(n)
        assert s.time_level == step0 + nsteps
        return s.fields()
    finally:
        s.close()


def _same(a, b, msg=""):
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), msg


def _case(nx, ny, bc, N=3, K=3, precision="f64", delta=0.0, potential="well", G=2e-3, seed=0):
    from test_gpu_parity import nuclei_case, variant

    p = variant(dim=2, N=N, K=K, n=(nx, ny, 1), bc=bc, potential=potential, delta=delta, G=G,
                precision=precision, seed=seed)
    phi, mu = nuclei_case(p, seed=seed + 7, count=4, radius=5.0)
    return p, phi, mu


CASES = {
    "eutectic_bc_f64": dict(nx=300, ny=200, bc=(0, 1, 0)),
    "eutectic_bc_f32": dict(nx=300, ny=200, bc=(0, 1, 0), precision="f32"),
    "all_periodic": dict(nx=130, ny=70, bc=(0, 0, 0)),
    "all_mirror": dict(nx=130, ny=70, bc=(1, 1, 0)),
    "mirror_x_periodic_y": dict(nx=126, ny=33, bc=(1, 0, 0), N=2, K=2),
    "odd_width_f32": dict(nx=61, ny=47, bc=(1, 1, 0), N=2, K=3, precision="f32"),
    "aniso": dict(nx=124, ny=40, bc=(0, 1, 0), N=3, K=2, delta=0.02),
    "aniso_f32_mirror": dict(nx=250, ny=31, bc=(1, 1, 0), N=2, K=2, delta=0.02, precision="f32"),
    "obstacle": dict(nx=90, ny=64, bc=(0, 1, 0), potential="obstacle"),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_two_steps_per_launch_bitwise(name):
    p, phi, mu = _case(**CASES[name])
    ref = _run(p, phi, mu, 9, 1, step0=3)
    for tile in [None, (64, 1, 1), (128, 3, 2), (256, 8, -1), (64, 64, 4)]:
        if tile and tile[2] == 4 and p.precision == "f64":
            continue
        got = _run(p, phi, mu, 9, 2, tile=tile, step0=3)
        _same(got, ref, (name, tile))


@pytest.mark.parametrize("nx,ny", [(1, 1), (2, 1), (1, 5), (3, 2), (7, 3), (5, 8), (64, 2), (2, 64)])
@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 0), (0, 1, 0), (1, 0, 0)])
def test_two_steps_per_launch_tiny_grids(nx, ny, bc):
    p, phi, mu = _case(nx, ny, bc, N=2, K=2, seed=nx * 31 + ny)
    phi, mu = inputs.random_multiphase(p, seed=nx + 7 * ny, amp=0.3)
    ref = _run(p, phi, mu, 6, 1)
    for tile in [(64, 1, 1), (128, 2, 2), (64, 5, -1)]:
        _same(_run(p, phi, mu, 6, 2, tile=tile), ref, (nx, ny, bc, tile))


def test_two_steps_with_graphs_and_odd_counts():
    p, phi, mu = _case(200, 90, (0, 1, 0), precision="f32")
    ref = _run(p, phi, mu, 23, 1, step0=1)
    _same(_run(p, phi, mu, 23, 2, step0=1), ref, "plain")
    _same(_run(p, phi, mu, 23, 2, graph=4, step0=1, chunks=[5, 8, 3, 7]), ref, "graph 4")
    _same(_run(p, phi, mu, 23, 2, graph=6, step0=1), ref, "graph 6")


def test_two_steps_c1_matches_oracle_1000_steps():
    p, phi, mu = inputs.config_c1(seed=0)
    f, m = _run(p, phi, mu, 1000, 2)
    of, om = gp.run(phi, mu, 0, 1000, p)
    assert np.max(np.abs(f - of)) <= 1e-10 and np.max(np.abs(m - om)) <= 1e-10


def test_two_steps_full_size_eutectic_conserves_and_matches_single():
    p, phi, mu = inputs.config_c2(precision="f64", n=(4096, 4096, 1))
    a = _run(p, phi, mu, 4, 1)
    b = _run(p, phi, mu, 4, 2)
    _same(a, b, "4096^2")


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_batch_two_steps_matches_single_instances(precision):
    from paper_2404_01035_amd.solver import BatchSolver

    members = inputs.config_c4(ninst=6, seed=23, precision=precision, side=(61, 190))
    members[0][0].bc = (1, 1, 0)  # a mirror instance among periodic ones
    members[0][0].dt = 0.2 * inputs.dt_limit(members[0][0])
    for fuse, vec, graph, chunks in [(2, 1, 0, [11]), (2, -1, 0, [4, 7]), (2, 2, 4, [11]), (1, 2, 0, [11])]:
        b = BatchSolver([m[0] for m in members])
        try:
            b.set_tile(5, vec)
            abi_fuse(b, fuse)
            b.set_graph(graph)
            for i, (_, phi, mu) in enumerate(members):
                b.load(i, phi, mu)
            b.start(2)
            for n in chunks:
                b.step(n)
            got = [b.fields(i) for i in range(len(members))]
        finally:
            b.close()
        for i, (p, phi, mu) in enumerate(members):
            _same(got[i], _run(p, phi, mu, 11, 1, step0=2), (fuse, vec, graph, i))


def abi_fuse(b, fuse):
    from paper_2404_01035_amd import abi

    abi.mp_set_fusion(b.st, fuse)
