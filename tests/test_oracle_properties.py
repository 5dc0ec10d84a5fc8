"""Identities of the model (Section 2.1) checked on the FP64 oracle at randomly drawn parameters and event
sets (hypothesis), beside the fixed-input pins: each holds at every theta, so a mistake that happens to
cancel at the default parameters still fails here.

* lambda_n and Lambda are linear in (mu, xi) jointly: mu dl/dmu + xi dl/dxi = N - Lambda.
* Both spatial kernels are 2-D densities: l(c x, c tau_x, c h0) = l - 2 N log c, Lambda unchanged.
* Both temporal kernels are densities in t: l(c t, c tau_t, omega / c) = l - N log c, Lambda unchanged.
* The gradient is the derivative of the value (central differences, Richardson-extrapolated).
* Rows are independent terms: l over [0, k) plus l over [k, N) is l over [0, N).

Against the planted mistakes of test_oracle_mutations.py these identities alone catch 10 of 19 (every
derivative mistake, the time-density normalisation, the compensator sign and limits); the structural
ones (the target's bandwidth for the source's, tie handling, a transposed coordinate, a constant factor)
leave them intact and are caught by the closed forms of test_oracle_pins.py.
"""

import math

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle

SETTINGS = settings(max_examples=25, deadline=None, suppress_health_check=[HealthCheck.too_slow])


@st.composite
def problems(draw):
    n = draw(st.integers(2, 40))
    seed = draw(st.integers(0, 2**31 - 1))
    # log-uniform parameters around the workloads' values
    mu = math.exp(draw(st.floats(math.log(0.05), math.log(5.0))))
    tau_x = math.exp(draw(st.floats(math.log(2.0), math.log(40.0))))
    tau_t = math.exp(draw(st.floats(math.log(1.0), math.log(30.0))))
    xi = math.exp(draw(st.floats(math.log(0.05), math.log(2.0))))
    h0 = math.exp(draw(st.floats(math.log(0.5), math.log(20.0))))
    omega = math.exp(draw(st.floats(math.log(0.02), math.log(2.0))))
    rng = np.random.default_rng(seed)
    t = np.sort(rng.uniform(0.0, 30.0, n))
    x = rng.normal(0.0, 10.0, n)
    y = rng.normal(0.0, 10.0, n)
    s = rng.lognormal(0.0, 0.5, n)
    return t, x, y, s, np.array([mu, tau_x, tau_t, xi, h0, omega])


def _unfloored(lam):
    return bool((lam > 1e-40).all())


@SETTINGS
@given(problems())
def test_euler_identity_at_any_theta(p):
    t, x, y, s, th = p
    ll, g, lam, Lam, _ = oracle.loglik(t, x, y, s, th, per_row=True)
    if not _unfloored(lam):
        return
    assert th[0] * g[0] + th[3] * g[3] == pytest.approx(len(t) - Lam.sum(), rel=1e-11, abs=1e-11)


@SETTINGS
@given(problems(), st.floats(0.1, 10.0))
def test_space_scaling_at_any_theta(p, c):
    t, x, y, s, th = p
    ll, _, lam, Lam, _ = oracle.loglik(t, x, y, s, th, per_row=True)
    th2 = th.copy()
    th2[1] *= c
    th2[4] *= c
    ll2, _, lam2, Lam2, _ = oracle.loglik(t, c * x, c * y, s, th2, per_row=True)
    if not (_unfloored(lam) and _unfloored(lam2)):
        return
    assert ll2 == pytest.approx(ll - 2 * len(t) * math.log(c), rel=1e-11, abs=1e-9)
    assert Lam2.sum() == pytest.approx(Lam.sum(), rel=1e-12)


@SETTINGS
@given(problems(), st.floats(0.1, 10.0))
def test_time_scaling_at_any_theta(p, c):
    t, x, y, s, th = p
    ll, _, lam, Lam, _ = oracle.loglik(t, x, y, s, th, per_row=True)
    th2 = th.copy()
    th2[2] *= c
    th2[5] /= c
    ll2, _, lam2, Lam2, _ = oracle.loglik(c * t, x, y, s, th2, per_row=True)
    if not (_unfloored(lam) and _unfloored(lam2)):
        return
    assert ll2 == pytest.approx(ll - len(t) * math.log(c), rel=1e-11, abs=1e-9)
    assert Lam2.sum() == pytest.approx(Lam.sum(), rel=1e-12)


@SETTINGS
@given(problems())
def test_gradient_is_the_derivative_at_any_theta(p):
    t, x, y, s, th = p
    ll, g, lam, _, _ = oracle.loglik(t, x, y, s, th, per_row=True)
    if not _unfloored(lam):
        return
    for k in range(6):
        h = 1e-4 * th[k]

        def d(step):
            hi, lo = th.copy(), th.copy()
            hi[k] += step
            lo[k] -= step
            return (oracle.loglik(t, x, y, s, hi)[0] - oracle.loglik(t, x, y, s, lo)[0]) / (2 * step)

        rich = (4 * d(h / 2) - d(h)) / 3
        assert g[k] == pytest.approx(rich, rel=1e-6, abs=1e-8 * (abs(ll) + 1.0) / th[k])


@SETTINGS
@given(problems(), st.data())
def test_rows_add_up_at_any_theta(p, data):
    t, x, y, s, th = p
    n = len(t)
    k = data.draw(st.integers(0, n))
    ll, g = oracle.loglik(t, x, y, s, th)
    ll_a, g_a = oracle.loglik(t, x, y, s, th, rows=(0, k))
    ll_b, g_b = oracle.loglik(t, x, y, s, th, rows=(k, n))
    assert ll_a + ll_b == pytest.approx(ll, rel=1e-13, abs=1e-12)
    np.testing.assert_allclose(g_a + g_b, g, rtol=1e-12, atol=1e-12 * np.abs(g).max())
