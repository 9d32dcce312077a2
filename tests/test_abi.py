"""Host-side checks of the C ABI (no GPU needed: these calls make no HIP call)."""
import math
import os
import re

import numpy as np
import pytest

from paper_2404_01035_amd import abi, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    with open(os.path.join(ROOT, "include", "mp.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(mp_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = abi.lib()
    declared = _header_symbols()
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(abi.EXPORTS) == declared


def test_create_and_query_without_gpu():
    p, _, _ = inputs.config_c1()
    st = abi.mp_create(p)
    try:
        assert abi.mp_state_bytes(st) == p.ncells * p.nfields * 8
        assert abi.mp_workspace_bytes(st) > 0
        assert abi.mp_current(st) == (0, 0)
        abi.mp_set_step(st, 7, 1)
        assert abi.mp_current(st) == (1, 7)
        assert abi.mp_get_tile(st) == (256, 31, 1)
        abi.mp_set_tile(st, 128, 16)
        assert abi.mp_get_tile(st) == (128, 16, 1)
        abi.mp_set_tile(st, 0, 0, -1)
        assert abi.mp_get_tile(st) == (128, 16, -1)
    finally:
        abi.mp_destroy(st)


def test_fp32_state_bytes():
    p, _, _ = inputs.config_c2(n=(96, 80, 1), precision="f32")
    st = abi.mp_create(p)
    assert abi.mp_state_bytes(st) == p.ncells * 5 * 4
    abi.mp_destroy(st)


def test_dt_limit_matches_input_formula():
    for p in [inputs.config_c1()[0], inputs.config_c2(n=(64, 64, 1))[0],
              inputs.dendrite_params(n=(16, 16, 16))]:
        assert math.isclose(abi.mp_dt_limit(p), inputs.dt_limit(p), rel_tol=1e-14)


def test_dt_limit_matches_input_formula_extended_model():
    """Per-pair tau and off-diagonal A/D enter the limit the same way on both sides."""
    rng = np.random.default_rng(4)
    p = inputs.config_c2(n=(64, 64, 1))[0]
    for q in range(3):
        a, b = [(0, 1), (0, 2), (1, 2)][q]
        p.tau_ab[a, b] = p.tau_ab[b, a] = rng.uniform(0.4, 1.5)
    assert math.isclose(abi.mp_dt_limit(p), inputs.dt_limit(p), rel_tol=1e-14)
    p.A01[:3] = rng.uniform(-0.4, 0.4, size=3)
    p.D[:3, :2] = rng.uniform(0.1, 1.0, size=(3, 2))
    p.D01[:3] = 0.3 * np.sqrt(p.D[:3, 0] * p.D[:3, 1])
    assert math.isclose(abi.mp_dt_limit(p), inputs.dt_limit(p), rel_tol=1e-13)
    p.dt = 0.5 * inputs.dt_limit(p)
    abi.mp_destroy(abi.mp_create(p))


def test_create_rejects_bad_extended_coefficients():
    p = inputs.config_c2_slopes(n=(32, 32, 1))[0]
    abi.mp_destroy(abi.mp_create(p))
    q = p.copy()
    q.tau_ab[0, 1] = q.tau_ab[1, 0] = 1.0  # one pair only
    _expect(abi.MP_E_PARAM, q, "every pair")
    q = p.copy()
    q.tau_ab[0, 1], q.tau_ab[1, 0] = 1.0, 2.0
    _expect(abi.MP_E_PARAM, q, "symmetric")
    q = p.copy()
    q.A01[1] = 2.0 * np.sqrt(q.A[1, 0] * q.A[1, 1]) + 0.1  # curvature matrix not positive definite
    _expect(abi.MP_E_PARAM, q, "positive definite")
    q = p.copy()
    q.D[2, :2] = (1.0, 1.0)
    q.D01[2] = 1.5
    _expect(abi.MP_E_PARAM, q, "semidefinite")
    q = p.copy()
    q.Bt[0, 1] = float("inf")
    _expect(abi.MP_E_PARAM, q, "Bt")
    import ctypes as C
    g, c = abi.to_grid(p), abi.to_params(p)
    c.potential = 3
    h = C.c_void_p()
    assert abi.lib().mp_create(C.byref(g), 3, 3, C.byref(c), C.byref(h)) == abi.MP_E_PARAM


def _expect(code, p, match=None):
    with pytest.raises(abi.MPError) as ei:
        abi.mp_create(p)
    assert ei.value.code == code, str(ei.value)
    if match:
        assert re.search(match, str(ei.value)), str(ei.value)


def test_create_rejects_bad_input():
    p, _, _ = inputs.config_c1()
    _expect(abi.MP_E_UNSTABLE, p.copy(dt=1.01 * inputs.dt_limit(p)), "stability")
    _expect(abi.MP_E_PARAM, p.copy(nphases=4), "nphases")
    _expect(abi.MP_E_PARAM, p.copy(ncomp=4), "ncomp")
    _expect(abi.MP_E_PARAM, p.copy(dim=4), "dim")
    _expect(abi.MP_E_PARAM, p.copy(n=(0, 64, 1)), "n\\[0\\]")
    _expect(abi.MP_E_PARAM, p.copy(n=(8, 8, 2)), "2D grid")
    _expect(abi.MP_E_PARAM, p.copy(bc=(2, 0, 0)), "bc")
    _expect(abi.MP_E_PARAM, p.copy(dx=-1.0), "dx")
    _expect(abi.MP_E_PARAM, p.copy(eps=0.0), "eps")
    _expect(abi.MP_E_PARAM, p.copy(tau=-1.0), "tau")
    q = p.copy()
    q.A[0, 0] = 0.0
    _expect(abi.MP_E_PARAM, q, "A\\[0\\]\\[0\\]")
    q = p.copy()
    q.D[1, 0] = -1.0
    _expect(abi.MP_E_PARAM, q, "D\\[1\\]\\[0\\]")
    q = p.copy()
    q.gamma[0, 1] = 2.0  # asymmetric
    _expect(abi.MP_E_PARAM, q, "symmetric")
    q = p.copy()
    q.delta[0, 1] = q.delta[1, 0] = 0.5
    _expect(abi.MP_E_PARAM, q, "delta")
    q = p.copy()
    q.C[0] = float("nan")
    _expect(abi.MP_E_PARAM, q, "finite")
    import ctypes as C
    g, c = abi.to_grid(p), abi.to_params(p)
    h = C.c_void_p()
    for field in ("precision", "potential"):
        c2 = abi.to_params(p)
        setattr(c2, field, 7)
        assert abi.lib().mp_create(C.byref(g), 2, 2, C.byref(c2), C.byref(h)) == abi.MP_E_PARAM
        assert field in abi.mp_last_error()
    assert abi.lib().mp_create(C.byref(g), 2, 2, C.byref(c), C.byref(h)) == abi.MP_OK
    abi.mp_destroy(h.value)


def test_calls_reject_null_and_unbound():
    L = abi.lib()
    assert L.mp_bind(None, None, None, None) == abi.MP_E_NULLPTR
    assert L.mp_step(None, 1, None) == abi.MP_E_NULLPTR
    p, _, _ = inputs.config_c1()
    st = abi.mp_create(p)
    try:
        assert L.mp_step(st, 1, None) == abi.MP_E_UNBOUND
        assert "before mp_bind" in abi.mp_last_error()
        assert L.mp_bind(st, None, None, None) == abi.MP_E_NULLPTR
        assert L.mp_bind(st, 256, 256, 512) == abi.MP_E_PARAM      # same buffer twice
        assert L.mp_bind(st, 256, 520, 1024) == abi.MP_E_PARAM     # misaligned
        assert L.mp_set_step(st, -1, 0) == abi.MP_E_PARAM
        assert L.mp_set_step(st, 0, 2) == abi.MP_E_PARAM
        assert L.mp_set_tile(st, 100, 0, 0) == abi.MP_E_PARAM
        assert L.mp_set_tile(st, 0, -3, 0) == abi.MP_E_PARAM
        assert L.mp_set_tile(st, 0, 0, 4) == abi.MP_E_PARAM   # FP64: at most 2 cells per lane
        assert L.mp_set_tile(st, 0, 0, 3) == abi.MP_E_PARAM
    finally:
        abi.mp_destroy(st)
    abi.mp_destroy(None)


def test_create_rejects_null_pointers():
    import ctypes as C
    L = abi.lib()
    h = C.c_void_p()
    assert L.mp_create(None, 2, 2, None, C.byref(h)) == abi.MP_E_NULLPTR
    p, _, _ = inputs.config_c1()
    g = abi.to_grid(p)
    assert L.mp_create(C.byref(g), 2, 2, None, C.byref(h)) == abi.MP_E_NULLPTR
    assert L.mp_create(C.byref(g), 2, 2, C.byref(abi.to_params(p)), None) == abi.MP_E_NULLPTR


def test_batch_create_validation_and_layout_without_gpu():
    members = inputs.config_c4(ninst=5, seed=2, side=(64, 96))
    plist = [m[0] for m in members]
    st = abi.mp_create_batch(plist)
    try:
        assert abi.mp_instance_count(st) == 5
        prev_end = 0
        for i, p in enumerate(plist):
            off, nb = abi.mp_instance_offset(st, i)
            assert off % 256 == 0 and off >= prev_end
            assert nb == p.ncells * p.nfields * 4
            prev_end = off + nb
        assert abi.mp_state_bytes(st) >= prev_end
        with pytest.raises(abi.MPError):
            abi.mp_instance_offset(st, 5)
    finally:
        abi.mp_destroy(st)
    bad = [p.copy() for p in plist]
    bad[2] = bad[2].copy(dt=2 * inputs.dt_limit(bad[2]))
    with pytest.raises(abi.MPError) as ei:
        abi.mp_create_batch(bad)
    assert ei.value.code == abi.MP_E_UNSTABLE and "instance 2" in str(ei.value)
    mixed = [p.copy() for p in plist]
    mixed[1] = mixed[1].copy(precision="f64")
    with pytest.raises(abi.MPError) as ei:
        abi.mp_create_batch(mixed)
    assert ei.value.code == abi.MP_E_PARAM and "precision" in str(ei.value)
    d3 = [inputs.dendrite_params(n=(8, 8, 8))]
    with pytest.raises(abi.MPError) as ei:
        abi.mp_create_batch(d3)
    assert "2D" in str(ei.value)
    assert abi.lib().mp_create_batch(0, None, None, None, None, None) == abi.MP_E_NULLPTR


def test_graph_chunk_validation_without_gpu():
    p, _, _ = inputs.config_c1()
    st = abi.mp_create(p)
    try:
        for bad in (-2, 1, 3, 7):
            assert abi.lib().mp_set_graph(st, bad) == abi.MP_E_PARAM
        for good in (0, 2, 8, 100):
            abi.mp_set_graph(st, good)
        assert abi.mp_instance_count(st) == 1
        assert abi.mp_instance_offset(st, 0) == (0, abi.mp_state_bytes(st))
    finally:
        abi.mp_destroy(st)


def test_adjoint_rejects_unsupported_variants_without_gpu():
    import ctypes as C
    L = abi.lib()
    cases = []
    p, _, _ = inputs.config_c1()
    cases.append((p.copy(potential="obstacle"), abi.MP_E_PARAM, "obstacle"))
    q = p.copy()
    q.delta[0, 1] = q.delta[1, 0] = 0.02
    q.dt = 0.2 * inputs.dt_limit(q)
    cases.append((q, abi.MP_E_PARAM, "anisotropic"))
    cases.append((inputs.dendrite_params(n=(8, 8, 8), delta=0.0), abi.MP_E_PARAM, "2D"))
    cases.append((inputs.kks_from(p), abi.MP_E_PARAM, "KKS"))
    buf = C.c_void_p(256)
    g = (C.c_double * 10)()
    for prm, code, word in cases:
        st = abi.mp_create(prm)
        try:
            rc = L.mp_adjoint(st, buf, 10, 5, 0, buf, buf, g, buf, None)
            assert rc == code and word in abi.mp_last_error(), (rc, abi.mp_last_error())
        finally:
            abi.mp_destroy(st)
    st = abi.mp_create(p)
    try:
        assert L.mp_adjoint(st, None, 10, 5, 0, buf, buf, g, buf, None) == abi.MP_E_NULLPTR
        assert L.mp_adjoint(st, buf, 10, 5, 0, buf, buf, g, buf, None) == abi.MP_E_UNBOUND
        assert abi.mp_adjoint_work_bytes(st, 0) == 0
        assert abi.mp_adjoint_work_bytes(st, 10) > 10 * abi.mp_state_bytes(st)
    finally:
        abi.mp_destroy(st)
    members = inputs.config_c4(ninst=2, side=(64, 70))
    bst = abi.mp_create_batch([m[0] for m in members])
    try:
        assert L.mp_adjoint(bst, buf, 10, 5, 0, buf, buf, g, buf, None) == abi.MP_E_STATE
        assert abi.mp_adjoint_work_bytes(bst, 5) == 0
    finally:
        abi.mp_destroy(bst)


def test_tune_candidates_and_errors_without_gpu():
    import ctypes as C
    p, _, _ = inputs.config_c1()
    st = abi.mp_create(p)
    try:
        cand = abi.mp_tune_candidates(st)
        assert len(cand) >= 4 and all(b in (64, 128, 256) and s >= 1 and v in (1, 2) and f in (1, 2)
                                      for b, s, v, f in cand)
        for b, s, v, f in cand:  # every candidate is one the state accepts
            abi.mp_set_fusion(st, f)
            abi.mp_set_tile(st, b, s, v)
        L = abi.lib()
        buf = (C.c_int32 * 4)(64, 16, 1, 1)
        ms = (C.c_double * 1)()
        best = C.c_int()
        assert L.mp_tune(st, buf, 1, 3, ms, C.byref(best), None) == abi.MP_E_UNBOUND
        assert L.mp_tune(st, None, 1, 3, ms, C.byref(best), None) == abi.MP_E_NULLPTR
    finally:
        abi.mp_destroy(st)
    st = abi.mp_create(inputs.dendrite_params(n=(8, 8, 8)))
    try:
        assert {(b, v, f) for b, _, v, f in abi.mp_tune_candidates(st)} == {(256, 1, 1), (512, 1, 1)}
        assert abi.lib().mp_set_tile(st, 0, 0, 2) == abi.MP_E_PARAM
    finally:
        abi.mp_destroy(st)


def test_autotune_signature_distinguishes_workloads():
    from paper_2404_01035_amd import autotune
    p, _, _ = inputs.config_c1()
    q = p.copy(precision="f32")
    a = autotune.signature([p], "dev")
    assert a == autotune.signature([p.copy()], "dev")
    assert a != autotune.signature([q], "dev") and a != autotune.signature([p], "other")
    members = [m[0] for m in inputs.config_c4(ninst=3, side=(64, 80))]
    assert autotune.signature(members, "dev") != autotune.signature(members[:2], "dev")
    # the anti-trapping current's form and the extended model select other kernels
    assert a != autotune.signature([p], "dev", antitrapping=1)
    assert autotune.signature([p], "dev", 1) != autotune.signature([p], "dev", 2)
    e = p.copy()
    e.Bt[0, 0] = 0.1
    assert a != autotune.signature([e], "dev")
    e = p.copy(potential="obstacle_active")
    assert autotune.signature([e], "dev") != autotune.signature([p.copy(potential="obstacle")], "dev")


def test_fusion_setting_validation_without_gpu():
    p, _, _ = inputs.config_c1()
    st = abi.mp_create(p)
    try:
        assert abi.mp_get_fusion(st) == 2  # the default for a single 2D grid
        abi.mp_set_fusion(st, 1)
        assert abi.mp_get_fusion(st) == 1
        for bad in (0, 3, -1):
            with pytest.raises(abi.MPError):
                abi.mp_set_fusion(st, bad)
    finally:
        abi.mp_destroy(st)
    st = abi.mp_create(inputs.dendrite_params(n=(8, 8, 8)))
    try:
        with pytest.raises(abi.MPError, match="2D"):
            abi.mp_set_fusion(st, 2)
    finally:
        abi.mp_destroy(st)
    bst = abi.mp_create_batch([m[0] for m in inputs.config_c4(ninst=2, side=(64, 70))])
    try:
        abi.mp_set_fusion(bst, 2)  # batches of 2D grids take either
        assert abi.mp_get_fusion(bst) == 2
    finally:
        abi.mp_destroy(bst)


def test_antitrapping_switch_validation_without_gpu():
    import ctypes as C
    L = abi.lib()
    p, _, _ = inputs.config_c1()
    st = abi.mp_create(p)
    try:
        assert abi.mp_get_antitrapping(st) == 0  # off by default
        abi.mp_set_antitrapping(st, 2)  # the separate correction kernel
        assert abi.mp_get_antitrapping(st) == 2
        abi.mp_set_antitrapping(st, True)  # folded into the step
        assert abi.mp_get_antitrapping(st) == 1
        for bad in (-1, 3):
            assert L.mp_set_antitrapping(st, bad) == abi.MP_E_PARAM
        assert abi.mp_get_antitrapping(st) == 1
        # the adjoint refuses it before looking at its buffers
        g = (C.c_double * 10)()
        rc = L.mp_adjoint(st, None, 10, 5, 0, None, None, g, None, None)
        assert rc == abi.MP_E_STATE and "anti-trapping" in abi.mp_last_error()
        abi.mp_set_antitrapping(st, False)
        assert abi.mp_get_antitrapping(st) == 0
    finally:
        abi.mp_destroy(st)
    assert L.mp_set_antitrapping(None, 1) == abi.MP_E_NULLPTR
    assert L.mp_get_antitrapping(None, None) == abi.MP_E_NULLPTR
    st = abi.mp_create(inputs.dendrite_params(n=(8, 8, 8)))
    try:
        abi.mp_set_antitrapping(st, True)  # 3D grids take it too
        assert abi.mp_get_antitrapping(st) == 1
    finally:
        abi.mp_destroy(st)
    bst = abi.mp_create_batch([m[0] for m in inputs.config_c4(ninst=2, side=(64, 70))])
    try:
        # a batch takes the current folded into the step only
        with pytest.raises(abi.MPError) as ei:
            abi.mp_set_antitrapping(bst, 2)
        assert ei.value.code == abi.MP_E_STATE
        abi.mp_set_antitrapping(bst, True)
        assert abi.mp_get_antitrapping(bst) == 1
    finally:
        abi.mp_destroy(bst)


def _in_subprocess(code, env):
    import subprocess
    import sys

    e = dict(os.environ)
    e.update(env)
    return subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=e, cwd=ROOT,
                          timeout=120)


def test_mp_tile_environment_sets_the_tile_of_new_states():
    code = ("from paper_2404_01035_amd import abi, inputs\n"
            "p = inputs.config_c2(n=(64, 64, 1))[0]\n"
            "st = abi.mp_create(p); print(abi.mp_get_tile(st)); abi.mp_destroy(st)\n")
    r = _in_subprocess(code, {"MP_TILE": "128,16,2"})
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "(128, 16, 2)"
    bad = _in_subprocess(code, {"MP_TILE": "100,16,1"})
    assert bad.returncode != 0 and "MP_TILE" in bad.stderr


def test_mp_log_echoes_failures_to_stderr():
    code = ("from paper_2404_01035_amd import abi, inputs\n"
            "p = inputs.config_c1()[0]\n"
            "try:\n    abi.mp_create(p.copy(nphases=4))\nexcept abi.MPError:\n    pass\n")
    r = _in_subprocess(code, {"MP_LOG": "1"})
    assert r.returncode == 0, r.stderr
    assert "[mpstep] error -1: nphases must be 2 or 3" in r.stderr
    quiet = _in_subprocess(code, {"MP_LOG": "0"})
    assert "[mpstep]" not in quiet.stderr


def _kks_base(potential="well"):
    p, _, _ = inputs.config_c2(n=(64, 48, 1))
    return inputs.kks_from(p, potential=potential, theta=[0.2, 0.3, 0.1], theta3=0.5)


@pytest.mark.parametrize("potential", ["well", "theta"])
def test_kks_dt_limit_matches_input_formula(potential):
    p = _kks_base(potential)
    assert math.isclose(abi.mp_dt_limit(p), inputs.dt_limit(p), rel_tol=1e-14)
    if potential == "theta":
        # a stiff potential takes over from the gradient term
        q = p.copy()
        q.theta[0] = 400.0
        assert inputs.dt_limit(q) < inputs.dt_limit(p)
        assert math.isclose(abi.mp_dt_limit(q), inputs.dt_limit(q), rel_tol=1e-14)
    st = abi.mp_create(p)
    abi.mp_destroy(st)


def test_kks_validation_without_gpu():
    p = _kks_base("theta")
    _expect(abi.MP_E_PARAM, p.copy(Mphi=0.0), "Mphi")
    _expect(abi.MP_E_PARAM, p.copy(potential="obstacle"), "KKS")
    q = p.copy()
    q.theta[1] = -1.0
    _expect(abi.MP_E_PARAM, q, "theta\\[1\\]")
    q = p.copy()
    q.theta_ab[0, 1] = 2.0  # asymmetric
    _expect(abi.MP_E_PARAM, q, "theta_ab")
    q = p.copy()
    q.tau_ab[0, 1] = q.tau_ab[1, 0] = 1.0
    _expect(abi.MP_E_PARAM, q, "tau_ab")
    # Eq. Well1 is a KKS potential
    g, _, _ = inputs.config_c2(n=(64, 48, 1))
    _expect(abi.MP_E_PARAM, g.copy(potential="theta"), "potential")
    import ctypes as C
    c = abi.to_params(p)
    c.model = 5
    h = C.c_void_p()
    assert abi.lib().mp_create(C.byref(abi.to_grid(p)), 3, 3, C.byref(c), C.byref(h)) == abi.MP_E_PARAM
    assert "model" in abi.mp_last_error()
    # KKS does not read tau
    st = abi.mp_create(p.copy(tau=-1.0))
    abi.mp_destroy(st)


def test_kks_refuses_the_current_without_gpu():
    st = abi.mp_create(_kks_base("well"))
    try:
        assert abi.lib().mp_set_antitrapping(st, 1) == abi.MP_E_STATE
        assert "grand-potential" in abi.mp_last_error()
        assert abi.lib().mp_set_antitrapping(st, 0) == abi.MP_OK
    finally:
        abi.mp_destroy(st)
