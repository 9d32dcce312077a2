"""Batched persistent launch and HIP-graph replay, checked against the
single-grid kernel-by-kernel path (bitwise) and against the FP64 oracle."""
import numpy as np
import pytest

from oracle import gp
from paper_2404_01035_amd import inputs

pytestmark = pytest.mark.gpu


def _single(p, phi, mu, nsteps, step0=0, graph=0, tile=None, chunks=None):
    import torch

    from paper_2404_01035_amd.solver import Solver

    s = Solver(p)
    try:
        if tile:
            s.set_tile(*tile)
        s.set_graph(graph)
        s.load(phi, mu, step0)
        if chunks is None:
            s.step(nsteps)
        else:
            scratch = torch.zeros(1 << 20, device="cuda")
            for n in chunks:  # eager work and syncs between replays
                s.step(n)
                scratch.add_(1.0)
                torch.cuda.synchronize()
        assert s.time_level == step0 + nsteps
        return s.fields()
    finally:
        s.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_graph_replay_matches_launch_loop_2d(precision):
    p, phi, mu = inputs.config_c2(n=(300, 200, 1), precision=precision)
    p.G = 3e-3  # time-dependent temperature: every replay must see its own step
    a = _single(p, phi, mu, 31, step0=5)
    b = _single(p, phi, mu, 31, step0=5, graph=4, chunks=[4, 8, 3, 4, 12])
    c = _single(p, phi, mu, 31, step0=5, graph=2)
    for x in (b, c):
        assert np.array_equal(a[0], x[0]) and np.array_equal(a[1], x[1])


def test_graph_replay_matches_launch_loop_3d():
    from test_gpu_parity import nuclei_case, variant

    p = variant(dim=3, N=3, K=3, n=(70, 13, 40), bc=(0, 1, 1), delta=0.02, G=2e-3)
    phi, mu = nuclei_case(p, seed=3)
    a = _single(p, phi, mu, 14)
    b = _single(p, phi, mu, 14, graph=6, chunks=[6, 6, 2])
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def _batch_members(n, seed, precision, side=(64, 200)):
    return inputs.config_c4(ninst=n, seed=seed, precision=precision, side=side)


def _run_batch(members, nsteps, step0=0, seg=None, graph=0):
    from paper_2404_01035_amd.solver import BatchSolver

    b = BatchSolver([m[0] for m in members])
    try:
        if seg:
            b.set_tile(seg)
        b.set_graph(graph)
        for i, (_, phi, mu) in enumerate(members):
            b.load(i, phi, mu)
        b.start(step0)
        b.step(nsteps)
        return [b.fields(i) for i in range(len(members))], b.diagnostics()
    finally:
        b.close()


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_batch_matches_single_instances_bitwise(precision):
    members = _batch_members(7, seed=11, precision=precision)
    got, _ = _run_batch(members, 25, step0=3)
    for i, (p, phi, mu) in enumerate(members):
        ref = _single(p, phi, mu, 25, step0=3)
        assert np.array_equal(got[i][0], ref[0]), i
        assert np.array_equal(got[i][1], ref[1]), i


def test_batch_against_oracle_fp64():
    rng = np.random.default_rng(21)
    members = []
    for (nx, ny, N, K) in [(70, 50, 2, 2), (130, 64, 3, 3), (64, 90, 3, 2), (66, 66, 2, 3)]:
        p, phi, mu = inputs.random_instance(rng, nx, ny, N, K, precision="f64", nuclei=4)
        p.G, p.V, p.y0 = 2e-3, 0.05, ny / 3
        members.append((p, phi, mu))
    got, _ = _run_batch(members, 120, step0=7)
    for i, (p, phi, mu) in enumerate(members):
        of, om = gp.run(phi, mu, 7, 120, p)
        assert np.max(np.abs(got[i][0] - of)) <= 1e-10, i
        assert np.max(np.abs(got[i][1] - om)) <= 1e-10, i


def test_batch_segment_and_graph_invariance():
    members = _batch_members(5, seed=13, precision="f32")
    ref, dref = _run_batch(members, 18)
    for seg, graph in [(1, 0), (7, 0), (64, 6), (16, 2)]:
        got, d = _run_batch(members, 18, seg=seg, graph=graph)
        for i in range(len(members)):
            assert np.array_equal(got[i][0], ref[i][0]), (seg, graph, i)
            assert np.array_equal(got[i][1], ref[i][1]), (seg, graph, i)
        assert d == dref


def test_batch_diagnostics_match_single():
    from paper_2404_01035_amd.solver import Solver

    members = _batch_members(4, seed=17, precision="f64")
    _, dg = _run_batch(members, 10)
    for i, (p, phi, mu) in enumerate(members):
        s = Solver(p)
        s.load(phi, mu)
        s.step(10)
        d = s.diagnostics()
        s.close()
        assert d == dg[i], i


def test_autotuner_keeps_results_and_caches(tmp_path):
    from paper_2404_01035_amd.solver import BatchSolver, Solver

    cache = str(tmp_path / "tiles.json")
    p, phi, mu = inputs.config_c2(n=(300, 200, 1), precision="f64")
    ref = _single(p, phi, mu, 9)
    s = Solver(p)
    try:
        s.load(phi, mu)
        r = s.autotune(reps=2, cache=cache)
        assert r["source"] == "timed" and all(t > 0 for t in r["ms"].values())
        assert abi_tile(s) == (r["bx"], r["seg"], r["vec"])
        assert fusion(s) == r["fuse"]
        assert s.time_level == 0
        s.step(9)
        got = s.fields()
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
    finally:
        s.close()
    s = Solver(p)
    try:
        assert s.autotune(cache=cache)["source"] == "cache"
    finally:
        s.close()
    members = _batch_members(5, seed=19, precision="f32")
    bref, _ = _run_batch(members, 6)
    b = BatchSolver([m[0] for m in members])
    try:
        for i, (_, phi, mu) in enumerate(members):
            b.load(i, phi, mu)
        b.start(0)
        assert b.autotune(reps=2, cache=cache)["source"] == "timed"
        b.step(6)
        for i in range(len(members)):
            f = b.fields(i)
            assert np.array_equal(f[0], bref[i][0]) and np.array_equal(f[1], bref[i][1])
    finally:
        b.close()


def abi_tile(s):
    from paper_2404_01035_amd import abi

    return abi.mp_get_tile(s.st)


def fusion(s):
    from paper_2404_01035_amd import abi

    return abi.mp_get_fusion(s.st)
