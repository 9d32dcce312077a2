"""Pins of the oracle's hand-written discrete adjoint.

The adjoint is checked against the forward step itself, never against a second
copy of its own formulas: the dot-product identity <J v, w> = <v, J^T w> with
J v taken by complex step through ``step``, parameter gradients against complex
steps in the parameter, and a multi-step loss against central differences.
"""
import numpy as np
import pytest

from oracle import gp
from paper_2404_01035_amd import inputs
from test_oracle_pins import random_state, small_params

CS = 1e-30

CASES = [
    dict(N=2, n=(5, 4, 1), bc=(0, 0, 0)),
    dict(N=3, n=(4, 5, 1), bc=(0, 1, 0), gamma3=0.3, G=0.05),
    dict(N=3, n=(6, 3, 1), bc=(1, 1, 0)),
    dict(N=2, dim=3, n=(3, 4, 3), bc=(1, 0, 1)),
    dict(N=3, dim=3, n=(3, 3, 4), bc=(0, 1, 0), G=0.1),
    dict(N=3, n=(1, 4, 1), bc=(0, 1, 0)),
    dict(N=2, n=(2, 1, 1), bc=(0, 0, 0)),
]


def _case(case, seed=3):
    p = small_params(**case)
    phi, mu = random_state(p, seed=seed, simplex=True)
    return p, phi, mu


@pytest.mark.parametrize("case", CASES)
def test_adjoint_dot_product_one_step(case):
    p, phi, mu = _case(case)
    rng = np.random.default_rng(1)
    v = rng.normal(size=phi.shape), rng.normal(size=mu.shape)
    w = rng.normal(size=phi.shape), rng.normal(size=mu.shape)
    fc, mc = gp.step(phi + 1j * CS * v[0], mu + 1j * CS * v[1], 2, p)
    lhs = np.sum(fc.imag / CS * w[0]) + np.sum(mc.imag / CS * w[1])
    lp, lm, _ = gp.adjoint_step(phi, mu, 2, p, w[0], w[1])
    rhs = np.sum(lp * v[0]) + np.sum(lm * v[1])
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def _perturbed(p, name, idx, h):
    q = p.copy()
    dtype = complex if isinstance(h, complex) else float
    q.gamma = np.array(q.gamma, dtype=dtype)
    q.D = np.array(q.D, dtype=dtype)
    if name == "gamma":
        a, b = gp.PAIRS[idx]
        q.gamma[a, b] += h
        q.gamma[b, a] += h
    elif name == "D":
        q.D[idx] += h
    else:
        q.tau = q.tau + h
    return q


@pytest.mark.parametrize("case", CASES[:5])
def test_adjoint_parameter_gradients_one_step(case):
    p, phi, mu = _case(case, seed=5)
    rng = np.random.default_rng(2)
    w = rng.normal(size=phi.shape), rng.normal(size=mu.shape)
    _, _, g = gp.adjoint_step(phi, mu, 2, p, w[0], w[1])
    N, K1 = p.nphases, p.nmu
    checks = [("tau", None, g["tau"])]
    for q, (a, b) in enumerate(gp.PAIRS):
        if b < N:
            checks.append(("gamma", q, g["gamma"][q]))
    for a in range(N):
        for k in range(K1):
            checks.append(("D", (a, k), g["D"][a, k]))
    for name, idx, got in checks:
        q = _perturbed(p, name, idx, 1j * CS)
        fc, mc = gp.step(phi.astype(complex), mu.astype(complex), 2, q)
        num = (np.sum(fc.imag * w[0]) + np.sum(mc.imag * w[1])) / CS
        assert abs(got - num) <= 1e-11 * max(1.0, abs(num)), (name, idx, got, num)


def test_adjoint_multi_step_dot_product_and_zero_blocks():
    p, phi, mu = _case(dict(N=3, n=(6, 5, 1), bc=(0, 1, 0), G=0.02), seed=7)
    rng = np.random.default_rng(3)
    v = rng.normal(size=phi.shape), rng.normal(size=mu.shape)
    w = rng.normal(size=phi.shape), rng.normal(size=mu.shape)
    fc, mc = gp.run(phi + 1j * CS * v[0], mu + 1j * CS * v[1], 4, 8, p)
    lhs = np.sum(fc.imag / CS * w[0]) + np.sum(mc.imag / CS * w[1])
    lp, lm, _ = gp.adjoint_run(phi, mu, 4, 8, p, w[0], w[1])
    rhs = np.sum(lp * v[0]) + np.sum(lm * v[1])
    assert abs(lhs - rhs) <= 1e-11 * max(1.0, abs(lhs))
    # a zero cotangent stays zero
    lp0, lm0, g0 = gp.adjoint_run(phi, mu, 4, 3, p, 0 * w[0], 0 * w[1])
    assert not np.any(lp0) and not np.any(lm0) and not np.any(g0["gamma"]) and g0["tau"] == 0.0


def test_adjoint_loss_gradient_central_differences():
    """L = 1/2 sum (phi^N - phi*)^2 over 10 steps: gradients in gamma, D_liq and tau
    against central differences of the forward run (step 1e-5, FP64)."""
    rng = np.random.default_rng(9)
    p, phi, mu = inputs.random_instance(rng, 12, 10, 3, 3, precision="f64", nuclei=3)
    target = gp.run(phi, mu, 0, 10, p)[0] + 0.01 * rng.normal(size=phi.shape)

    def loss(q):
        f, _ = gp.run(phi, mu, 0, 10, q)
        return 0.5 * float(np.sum((f - target) ** 2))

    fN, _ = gp.run(phi, mu, 0, 10, p)
    _, _, g = gp.adjoint_run(phi, mu, 0, 10, p, fN - target, np.zeros_like(mu))
    h = 1e-5
    for name, idx, got in [("gamma", 0, g["gamma"][0]), ("gamma", 2, g["gamma"][2]),
                           ("D", (2, 0), g["D"][2, 0]), ("D", (2, 1), g["D"][2, 1]),
                           ("tau", None, g["tau"])]:
        lp = loss(_perturbed(p, name, idx, h))
        lm = loss(_perturbed(p, name, idx, -h))
        num = (lp - lm) / (2 * h)
        assert abs(got - num) <= 1e-6 * max(1e-8, abs(num)) + 1e-12, (name, idx, got, num)


def test_adjoint_refuses_nondifferentiable_variants():
    p, phi, mu = _case(dict(N=2, n=(4, 4, 1), bc=(0, 0, 0)))
    with pytest.raises(ValueError):
        gp.adjoint_step(phi, mu, 0, p.copy(potential="obstacle"), phi, mu)
    q = p.copy()
    q.delta[0, 1] = q.delta[1, 0] = 0.02
    with pytest.raises(ValueError):
        gp.adjoint_step(phi, mu, 0, q, phi, mu)
