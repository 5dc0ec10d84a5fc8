"""GPU parity of the paper's spatially uniform background (equation "fixed": mu0 / A(X) times
the temporal Gaussian), selected by a domain area > 0 in the event set, against the FP64
oracle with the same area.  Same tolerances as the Gaussian-background model."""

import math

import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2407_11349_amd as hk

pytestmark = pytest.mark.gpu

AREA = 1.0e6  # km^2: the 1000 x 1000 km box of the workloads
TOL = {"fp64": (1e-12, 1e-10, 1e-12), "fp32": (1e-9, 1e-6, 5e-6), "fp32_skip": (1e-9, 1e-6, 5e-6)}


def _say(msg):
    print(msg, flush=True)


def _run(dev, th, prec, rows=None):
    ll, g = hk.loglik_grad(dev, th, precision=prec, rows=rows)
    torch.cuda.synchronize()
    return float(ll.item()), g.cpu().numpy()


def _check(ll, g, ll_ref, g_ref, prec, what):
    tl, tg, _ = TOL[prec]
    rel_l = abs(ll - ll_ref) / abs(ll_ref)
    nz = g_ref != 0.0
    rel_g = np.abs(g[nz] - g_ref[nz]) / np.abs(g_ref[nz])
    _say(f"{what} {prec}: loglik rel err {rel_l:.2e}, grad rel err max {rel_g.max():.2e}")
    assert rel_l <= tl and rel_g.max() <= tg
    assert np.all(g[~nz] == 0.0)  # d/d tau_x


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_skip"])
def test_uniform_background_n2000(prec):
    ev = synth.generate(synth.N2K)
    th = synth.theta_default()
    ll_ref, g_ref, lam_ref, _, _ = oracle.loglik(ev.t, ev.x, ev.y, ev.s, th, per_row=True, area=AREA)
    dev = hk.DeviceEvents.from_arrays(ev.t, ev.x, ev.y, ev.s, area=AREA)
    ll, g = _run(dev, th, prec)
    _check(ll, g, ll_ref, g_ref, prec, "uniform n2000")
    lam, _ = hk.event_terms(dev, th, precision=prec)
    np.testing.assert_allclose(lam.cpu().numpy(), lam_ref, rtol=TOL[prec][2])


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_uniform_background_n20000_model1_and_model2(prec):
    """1000 days, 3000 counties: the paper's model 2 (density-scaled bandwidths) and model 1 (s = 1)."""
    ev = synth.generate(synth.N100K, n=20000, seed=23)
    th = synth.theta_default()
    for s, name in ((ev.s, "model2"), (np.ones(ev.n), "model1")):
        ll_ref, g_ref = oracle.loglik(ev.t, ev.x, ev.y, s, th, area=AREA)
        dev = hk.DeviceEvents.from_arrays(ev.t, ev.x, ev.y, s, area=AREA)
        ll, g = _run(dev, th, prec)
        _check(ll, g, ll_ref, g_ref, prec, f"uniform n20000 {name}")


@pytest.mark.parametrize("prec", ["fp32", "fp32_skip"])
def test_uniform_background_integer_day_ties(prec):
    """Integer-day times: the background depends on the time gap alone, so every pair with the same
    gap shares one exponent; the hi/lo split of that exponent keeps the FP32 sum unbiased."""
    ev = synth.generate(synth.N100K, n=20000, seed=29)
    t = np.floor(ev.t)
    th = synth.theta_default()
    ll_ref, g_ref, lam_ref, _, _ = oracle.loglik(t, ev.x, ev.y, ev.s, th, per_row=True, area=AREA)
    dev = hk.DeviceEvents.from_arrays(t, ev.x, ev.y, ev.s, area=AREA)
    lam, _ = hk.event_terms(dev, th, precision=prec)
    rel = lam.cpu().numpy() / lam_ref - 1.0
    _say(f"uniform ties {prec} per-event lambda: mean rel {rel.mean():.3e} rms {np.sqrt((rel ** 2).mean()):.3e}")
    ll, g = _run(dev, th, prec)
    _check(ll, g, ll_ref, g_ref, prec, "uniform ties")


def test_uniform_background_rows_of_n100k_and_additivity():
    ev = synth.generate(synth.N100K)
    th = synth.theta_default()
    dev = hk.DeviceEvents.from_arrays(ev.t, ev.x, ev.y, ev.s, area=AREA)
    ll, g = _run(dev, th, "fp32")
    cuts = [0, 33333, 50000, 100000]
    parts = [_run(dev, th, "fp32", rows=(a, b)) for a, b in zip(cuts[:-1], cuts[1:])]
    assert sum(p[0] for p in parts) == pytest.approx(ll, rel=1e-9)
    rng = np.random.default_rng(31)
    for a in np.sort(rng.choice(ev.n - 500, 4, replace=False)):
        a = int(a)
        ref, gref = oracle.loglik(ev.t, ev.x, ev.y, ev.s, th, rows=(a, a + 500), area=AREA)
        got, gg = _run(dev, th, "fp32", rows=(a, a + 500))
        assert abs(got - ref) <= 1e-9 * abs(ref) + 5e-7 * math.sqrt(500)
