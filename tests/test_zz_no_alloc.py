"""mp_diagnostics_static (no workspace; the library's static device scratch)
against mp_diagnostics / mp_diagnostics_batch on the same states, through the
C ABI, and against the oracle's diagnostics: two calls in a row, the second on
a smaller state, then a batch.  The two entry points run the same kernels in
the same order, so the records must agree bitwise; the oracle bounds them to
1e-12 (relative for the sums)."""
import numpy as np
import pytest

from oracle import gp
from paper_2404_01035_amd import abi, inputs

pytestmark = pytest.mark.gpu


def _close(a, b, tol=1e-12):
    return abs(a - b) <= tol * max(1.0, abs(b))


def _check_vs_oracle(d, phi, mu, p):
    o = gp.diagnostics(phi, mu, p)
    for k in range(p.nmu):
        assert _close(d["mass"][k], o["mass"][k])
        assert _close(d["min_chi"][k], o["min_chi"][k])
    for a in range(p.nphases):
        assert _close(d["volume"][a], o["volume"][a])
    assert abs(d["max_sum_dev"] - o["max_sum_dev"]) <= 1e-14
    assert d["nonfinite"] == o["nonfinite"] == 0


def test_static_diagnostics_match_the_workspace_entry_point_twice():
    from paper_2404_01035_amd.solver import Solver

    cases = [inputs.config_c1(seed=0), inputs.config_c2(precision="f64", n=(40, 24, 1))]
    assert cases[1][0].ncells < cases[0][0].ncells  # the second call has the smaller input
    for idx, (p, phi, mu) in enumerate(cases):
        print(f"static diagnostics call {idx + 1}: {p.spatial} N={p.nphases} K={p.ncomp}", flush=True)
        s = Solver(p)
        s.load(phi, mu, step=5 + idx)
        s.step(7)
        ref = s.diagnostics()
        cur = s.current()
        got = abi.mp_diagnostics_static(s.st, cur.data_ptr(), s.time_level, s.stream())
        assert len(got) == 1
        assert got[0] == ref, (got[0], ref)
        assert got[0]["step"] == 12 + idx
        f, m = s.fields()
        _check_vs_oracle(got[0], f, m, p)
        s.close()


def test_static_diagnostics_of_a_batch():
    from paper_2404_01035_amd.solver import BatchSolver

    members = [inputs.config_c2(precision="f32", n=(48, 40, 1)), inputs.config_c1(seed=2),
               inputs.config_c2(precision="f32", n=(30, 20, 1))]
    plist = [m[0] for m in members]
    for q in plist:
        q.precision = "f32"
        q.bc = (inputs.BC_PERIODIC, inputs.BC_PERIODIC, inputs.BC_PERIODIC)
    b = BatchSolver(plist)
    for i, (_, phi, mu) in enumerate(members):
        b.load(i, phi, mu)
    b.start(0)
    b.step(6)
    ref = b.diagnostics()
    w, step = abi.mp_current(b.st)
    got = abi.mp_diagnostics_static(b.st, b.bufs[w].data_ptr(), step, 0)
    assert got == ref
    b.close()


def test_static_diagnostics_refuse_bad_arguments():
    p, _, _ = inputs.config_c1(seed=0)
    st = abi.mp_create(p)
    try:
        with pytest.raises(abi.MPError) as e:
            abi.mp_diagnostics_static(st, 0, 0)
        assert e.value.code == abi.MP_E_NULLPTR
    finally:
        abi.mp_destroy(st)
