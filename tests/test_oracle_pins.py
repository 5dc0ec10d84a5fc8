"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test checks the oracle against a closed form, an independent numerical
computation, a library routine, or an invariant that the paper's model
(Section 2.1: equations "fixed", "varying", "model" and the compensator) fixes.
Together they are chosen so that a dropped term, a wrong sign, a wrong index
(for instance the target's bandwidth used in place of the source's) or a wrong
normalisation fails at least one of them.
"""

import math

import mpmath
import numpy as np
import pytest
from scipy import stats

import oracle
import synth

LOG_FLOOR = math.log(1e-40)


def _theta(mu=0.5, tau_x=10.0, tau_t=7.0, xi=0.3, h0=2.0, omega=0.2):
    return np.array([mu, tau_x, tau_t, xi, h0, omega])


def _small_events(n, seed, t_max=30.0, box=40.0):
    rng = np.random.default_rng(seed)
    t = np.sort(rng.uniform(0.0, t_max, n))
    x = rng.normal(0.0, box / 4, n)
    y = rng.normal(0.0, box / 4, n)
    s = rng.lognormal(0.0, 0.5, n)
    return t, x, y, s


# ---------------------------------------------------------------- closed forms

def test_single_event_closed_form():
    """N = 1: lambda_1 = 0 is floored and the triggering part of Lambda vanishes (t_N = t_1)."""
    th = _theta()
    for t1 in (0.3, 5.0, 40.0):
        ll, g = oracle.loglik([t1], [3.0], [-2.0], [1.7], th)
        phi = stats.norm.cdf
        expect = LOG_FLOOR - th[0] * (phi(0.0) - phi(-t1 / th[2]))
        assert ll == pytest.approx(expect, rel=1e-15, abs=1e-13)
        # floored: the gradient is minus that of the compensator only
        assert g[0] == pytest.approx(-(0.5 - phi(-t1 / th[2])), rel=1e-14)
        assert g[1] == 0.0 and g[4] == 0.0
        assert g[3] == 0.0 and g[5] == 0.0


def test_two_event_closed_form_with_library_densities():
    """N = 2 with distinct bandwidth scales: pins self exclusion, causality direction,
    the source (earlier event's) bandwidth and every normalisation constant."""
    mu, tau_x, tau_t, xi, h0, omega = th = _theta(0.7, 3.0, 2.0, 0.4, 1.5, 0.3)
    t = np.array([1.0, 2.2])
    x = np.array([0.5, 1.7])
    y = np.array([-0.3, 0.9])
    s = np.array([0.6, 2.5])
    dt = t[1] - t[0]
    mvn = stats.multivariate_normal
    kb = mvn.pdf([x[1], y[1]], mean=[x[0], y[0]], cov=tau_x**2 * np.eye(2)) * stats.norm.pdf(dt, scale=tau_t)
    h1 = h0 * s[0]
    kt = mvn.pdf([x[1], y[1]], mean=[x[0], y[0]], cov=h1**2 * np.eye(2)) * stats.expon.pdf(dt, scale=1 / omega)
    lam1 = mu * kb
    lam2 = mu * kb + xi * kt
    phi = stats.norm.cdf
    big = t[1]
    comp = sum(mu * (phi((big - tm) / tau_t) - phi(-tm / tau_t)) + xi * (1 - math.exp(-omega * (big - tm)))
               for tm in t)
    ll, _, lam, Lam, _ = oracle.loglik(t, x, y, s, th, per_row=True)
    assert lam[0] == pytest.approx(lam1, rel=1e-13)
    assert lam[1] == pytest.approx(lam2, rel=1e-13)
    assert Lam.sum() == pytest.approx(comp, rel=1e-13)
    assert ll == pytest.approx(math.log(lam1) + math.log(lam2) - comp, rel=1e-13)


def test_rates_against_library_densities_random():
    """Every lambda_n of a random event set equals the library-density sum."""
    t, x, y, s = _small_events(40, 1)
    th = _theta(0.9, 6.0, 4.0, 0.5, 3.0, 0.4)
    bg, tr = oracle.rate_parts(t, x, y, s, th)
    mvn = stats.multivariate_normal
    for n in range(len(t)):
        b = 0.0
        g = 0.0
        for m in range(len(t)):
            if t[m] == t[n]:
                continue
            b += mvn.pdf([x[n], y[n]], mean=[x[m], y[m]], cov=th[1] ** 2 * np.eye(2)) * \
                stats.norm.pdf(t[n] - t[m], scale=th[2])
            if t[m] < t[n]:
                g += mvn.pdf([x[n], y[n]], mean=[x[m], y[m]], cov=(th[4] * s[m]) ** 2 * np.eye(2)) * \
                    stats.expon.pdf(t[n] - t[m], scale=1 / th[5])
        assert bg[n] == pytest.approx(b, rel=1e-12, abs=1e-300)
        assert tr[n] == pytest.approx(g, rel=1e-12, abs=1e-300)


# ----------------------------------------------------------- the compensator

def _gauss_legendre(a, b, k):
    z, w = np.polynomial.legendre.leggauss(k)
    return 0.5 * (b - a) * z + 0.5 * (b + a), 0.5 * (b - a) * w


def test_compensator_against_numerical_integration_of_the_rate():
    """Lambda = integral of lambda(x, t) over R^2 x (0, t_N] (paper, eq. likelihood and the
    R^2 approximation), done by brute-force quadrature of the pointwise rate function."""
    mu, tau_x, tau_t, xi, h0, omega = th = _theta(0.8, 1.5, 2.0, 0.6, 0.8, 0.7)
    t = np.array([1.0, 2.5, 4.0])
    x = np.array([0.0, 0.7, -0.4])
    y = np.array([0.2, -0.5, 0.6])
    s = np.array([1.0, 0.7, 1.5])
    tN = t[-1]

    # spatial rule: wide box, Gauss-Legendre (integrand is smooth and decays like a Gaussian)
    L = 14.0
    gx, wx = _gauss_legendre(-L, L, 160)
    X, Y = np.meshgrid(gx, gx, indexing="ij")
    W2 = np.outer(wx, wx)

    def rate(tt):
        lam = np.zeros_like(X)
        for m in range(3):
            if tt != t[m]:
                lam += mu * stats.multivariate_normal(mean=[x[m], y[m]], cov=tau_x**2 * np.eye(2)).pdf(
                    np.dstack([X, Y])) * stats.norm.pdf(tt - t[m], scale=tau_t)
            if t[m] < tt:
                lam += xi * stats.multivariate_normal(mean=[x[m], y[m]], cov=(h0 * s[m]) ** 2 * np.eye(2)).pdf(
                    np.dstack([X, Y])) * omega * math.exp(-omega * (tt - t[m]))
        return float((lam * W2).sum())

    total = 0.0
    edges = [0.0, *t]
    for a, b in zip(edges[:-1], edges[1:]):
        tt, wt = _gauss_legendre(a, b, 40)
        total += sum(w * rate(v) for v, w in zip(tt, wt))
    _, _, _, Lam, _ = oracle.loglik(t, x, y, s, th, per_row=True)
    assert Lam.sum() == pytest.approx(total, rel=1e-10)


# ------------------------------------------------------------------ gradient

def test_gradient_against_richardson_finite_differences():
    ev = synth.generate(synth.N2K, n=300, seed=7)
    th = synth.theta_default()
    _, g = oracle.loglik(ev.t, ev.x, ev.y, ev.s, th)

    def f(v):
        return oracle.loglik(ev.t, ev.x, ev.y, ev.s, v)[0]

    for k in range(6):
        h = 1e-4 * th[k]

        def d(hh):
            e = np.zeros(6)
            e[k] = hh
            return (f(th + e) - f(th - e)) / (2 * hh)

        rich = (4 * d(h / 2) - d(h)) / 3
        assert g[k] == pytest.approx(rich, rel=2e-7, abs=1e-7 * abs(g).max())


def test_euler_identity_mu_xi():
    """lambda_n is linear in (mu, xi) and Lambda too, so mu*dl/dmu + xi*dl/dxi = N - Lambda."""
    ev = synth.generate(synth.N2K, n=500, seed=3)
    th = synth.theta_default()
    ll, g, lam, Lam, _ = oracle.loglik(ev.t, ev.x, ev.y, ev.s, th, per_row=True)
    assert (lam > 1e-40).all()
    assert th[0] * g[0] + th[3] * g[3] == pytest.approx(len(ev.t) - Lam.sum(), rel=1e-12)


# ---------------------------------------------------------------- invariants

def test_space_scaling_identity():
    """l(c x, c tau_x, c h0) = l - 2 N log c: both spatial densities are 2-D."""
    ev = synth.generate(synth.N2K, n=400, seed=11)
    th = synth.theta_default()
    ll, _ = oracle.loglik(ev.t, ev.x, ev.y, ev.s, th)
    for c in (0.37, 3.0):
        th2 = th.copy()
        th2[1] *= c
        th2[4] *= c
        ll2, _ = oracle.loglik(ev.t, c * ev.x, c * ev.y, ev.s, th2)
        assert ll2 == pytest.approx(ll - 2 * len(ev.t) * math.log(c), rel=1e-12)


def test_time_scaling_identity():
    """l(c t, c tau_t, omega / c) = l - N log c, Lambda unchanged: both time kernels are densities."""
    ev = synth.generate(synth.N2K, n=400, seed=12)
    th = synth.theta_default()
    ll, _, _, Lam, _ = oracle.loglik(ev.t, ev.x, ev.y, ev.s, th, per_row=True)
    for c in (0.5, 4.0):
        th2 = th.copy()
        th2[2] *= c
        th2[5] /= c
        ll2, _, _, Lam2, _ = oracle.loglik(c * ev.t, ev.x, ev.y, ev.s, th2, per_row=True)
        assert ll2 == pytest.approx(ll - len(ev.t) * math.log(c), rel=1e-12)
        assert Lam2.sum() == pytest.approx(Lam.sum(), rel=1e-13)


def test_translation_rotation_and_permutation_invariance():
    ev = synth.generate(synth.N2K, n=300, seed=13)
    th = synth.theta_default()
    ll, g = oracle.loglik(ev.t, ev.x, ev.y, ev.s, th)
    a = 0.7
    xr = math.cos(a) * ev.x - math.sin(a) * ev.y + 123.0
    yr = math.sin(a) * ev.x + math.cos(a) * ev.y - 45.0
    ll2, g2 = oracle.loglik(ev.t, xr, yr, ev.s, th)
    assert ll2 == pytest.approx(ll, rel=1e-12)
    np.testing.assert_allclose(g2, g, rtol=1e-10)
    perm = np.random.default_rng(0).permutation(len(ev.t))
    ll3, g3 = oracle.loglik(ev.t[perm], ev.x[perm], ev.y[perm], ev.s[perm], th)
    assert ll3 == pytest.approx(ll, rel=1e-12)
    np.testing.assert_allclose(g3, g, rtol=1e-10)


def test_triggering_sum_matches_ozaki_recursion():
    """All events at one place and s = 1: the triggering sum of event n is
    omega/(2 pi h0^2) * A_n with A_1 = 0, A_n = exp(-omega (t_n - t_{n-1})) (1 + A_{n-1})
    (Ozaki 1979), an O(N) computation independent of the double sum."""
    rng = np.random.default_rng(5)
    n = 200
    t = np.sort(rng.uniform(0, 50, n))
    z = np.zeros(n)
    th = _theta(0.5, 3.0, 2.0, 0.4, 1.3, 0.35)
    _, tr = oracle.rate_parts(t, z, z, np.ones(n), th)
    A = np.zeros(n)
    for i in range(1, n):
        A[i] = math.exp(-th[5] * (t[i] - t[i - 1])) * (1.0 + A[i - 1])
    np.testing.assert_allclose(tr, th[5] / (2 * math.pi * th[4] ** 2) * A, rtol=1e-12, atol=1e-300)


def test_background_sum_matches_library_kde():
    """All events at one place: the background sum is a 1-D Gaussian kernel sum over other
    times, scaled by the bivariate density at 0."""
    rng = np.random.default_rng(6)
    n = 150
    t = np.sort(rng.uniform(0, 50, n))
    z = np.zeros(n)
    th = _theta(0.5, 3.0, 2.0, 0.4, 1.3, 0.35)
    bg, _ = oracle.rate_parts(t, z, z, np.ones(n), th)
    for i in range(n):
        others = np.delete(t, i)
        expect = stats.norm.pdf(t[i], loc=others, scale=th[2]).sum() / (2 * math.pi * th[1] ** 2)
        assert bg[i] == pytest.approx(expect, rel=1e-12)


def test_tie_semantics():
    """An event tied in time with event A adds nothing to A's rate (and A nothing to it),
    but still excites later events."""
    t = np.array([1.0, 2.0, 3.5])
    x = np.array([0.0, 0.5, 0.2])
    y = np.array([0.0, -0.3, 0.4])
    s = np.array([1.0, 1.2, 0.8])
    th = _theta(0.6, 2.0, 1.5, 0.5, 1.0, 0.4)
    _, _, lam, _, _ = oracle.loglik(t, x, y, s, th, per_row=True)
    t2 = np.array([1.0, 2.0, 2.0, 3.5])
    x2 = np.array([0.0, 0.5, 0.1, 0.2])
    y2 = np.array([0.0, -0.3, 0.1, 0.4])
    s2 = np.array([1.0, 1.2, 0.9, 0.8])
    _, _, lam2, _, _ = oracle.loglik(t2, x2, y2, s2, th, per_row=True)
    assert lam2[1] == pytest.approx(lam[1], rel=1e-15)
    # the tied partner sees exactly the events the other one sees (besides itself)
    t3 = np.array([1.0, 2.0, 3.5])
    x3 = np.array([0.0, 0.1, 0.2])
    y3 = np.array([0.0, 0.1, 0.4])
    _, _, lam3, _, _ = oracle.loglik(t3, x3, y3, np.array([1.0, 0.9, 0.8]), th, per_row=True)
    assert lam2[2] == pytest.approx(lam3[1], rel=1e-15)
    assert lam2[3] > lam[2]


def test_floor_of_tiny_rates():
    """Two events far apart: both rates underflow, are floored at 1e-40, and contribute
    no gradient through the log term (the gradient is minus that of the compensator)."""
    t = np.array([1.0, 900.0])
    x = np.array([0.0, 5000.0])
    y = np.array([0.0, 0.0])
    s = np.array([1.0, 1.0])
    th = _theta()
    ll, g, lam, Lam, ell = oracle.loglik(t, x, y, s, th, per_row=True)
    assert (lam < 1e-40).all()
    np.testing.assert_allclose(ell, LOG_FLOOR - Lam, rtol=1e-15)

    def comp(v):
        return oracle.loglik(t, x, y, s, v, per_row=True)[3].sum()

    for k in range(6):
        e = np.zeros(6)
        e[k] = 1e-6 * th[k]
        fd = -(comp(th + e) - comp(th - e)) / (2 * e[k])
        assert g[k] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_row_range_additivity():
    ev = synth.generate(synth.N2K, n=257, seed=21)
    th = synth.theta_default()
    ll, g = oracle.loglik(ev.t, ev.x, ev.y, ev.s, th)
    cuts = [0, 1, 64, 200, 257]
    parts = [oracle.loglik(ev.t, ev.x, ev.y, ev.s, th, rows=(a, b)) for a, b in zip(cuts[:-1], cuts[1:])]
    assert sum(p[0] for p in parts) == pytest.approx(ll, rel=1e-13)
    np.testing.assert_allclose(sum(p[1] for p in parts), g, rtol=1e-12)
    assert oracle.loglik(ev.t, ev.x, ev.y, ev.s, th, rows=(5, 5))[0] == 0.0


def test_fifty_digit_brute_force():
    """The FP64 oracle against a 50-digit evaluation of the same sums (rounding pin)."""
    mpmath.mp.dps = 50
    t, x, y, s = _small_events(7, 9, t_max=10.0, box=8.0)
    th = _theta(0.6, 2.0, 1.5, 0.5, 1.0, 0.4)
    mu, tau_x, tau_t, xi, h0, om = [mpmath.mpf(float(v)) for v in th]
    T = [mpmath.mpf(float(v)) for v in t]
    X = [mpmath.mpf(float(v)) for v in x]
    Y = [mpmath.mpf(float(v)) for v in y]
    S = [mpmath.mpf(float(v)) for v in s]
    tot = mpmath.mpf(0)
    for n in range(7):
        lam = mpmath.mpf(0)
        for m in range(7):
            if T[m] == T[n]:
                continue
            d2 = (X[n] - X[m]) ** 2 + (Y[n] - Y[m]) ** 2
            dt = T[n] - T[m]
            lam += mu * mpmath.exp(-d2 / (2 * tau_x**2)) / (2 * mpmath.pi * tau_x**2) * \
                mpmath.npdf(dt, 0, tau_t)
            if T[m] < T[n]:
                h = h0 * S[m]
                lam += xi * mpmath.exp(-d2 / (2 * h**2)) / (2 * mpmath.pi * h**2) * om * mpmath.exp(-om * dt)
        a = T[-1] - T[n]
        Lam = mu * (mpmath.ncdf(a / tau_t) - mpmath.ncdf(-T[n] / tau_t)) + xi * (1 - mpmath.exp(-om * a))
        tot += mpmath.log(lam) - Lam
    ll, _ = oracle.loglik(t, x, y, s, th)
    assert ll == pytest.approx(float(tot), rel=1e-14)


# ------------------------------------------------------------- philox, X draw

def test_philox_known_answer_vectors():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x64_10_kat.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(w, 16) for w in r]
        assert oracle.philox4x64_10(v[0:4], v[4:6]) == v[6:10]


def test_philox_matches_numpy_bit_generator():
    """numpy.random.Philox is Philox4x64-10; it increments the counter before each block."""
    rng = np.random.default_rng(17)
    M = 2**64 - 1
    for _ in range(20):
        c = [int(v) for v in rng.integers(0, 2**63, 4)]
        k = [int(v) for v in rng.integers(0, 2**63, 2)]
        prev = list(c)
        prev[0] = (prev[0] - 1) & M
        bg = np.random.Philox(counter=prev, key=k)
        assert [int(v) for v in bg.random_raw(4)] == oracle.philox4x64_10(c, k)


def test_resample_uniform_inside_counties():
    ev = synth.generate(synth.N2K, n=20000, seed=31)
    x, y = oracle.resample(ev.county, ev.rect, seed=2000, iteration=3)
    r = ev.rect[ev.county]
    assert ((x >= r[:, 0]) & (x < r[:, 2]) & (y >= r[:, 1]) & (y < r[:, 3])).all()
    ux = (x - r[:, 0]) / (r[:, 2] - r[:, 0])
    uy = (y - r[:, 1]) / (r[:, 3] - r[:, 1])
    assert stats.kstest(ux, "uniform").pvalue > 1e-3
    assert stats.kstest(uy, "uniform").pvalue > 1e-3
    assert abs(np.corrcoef(ux, uy)[0, 1]) < 0.05
    x2, _ = oracle.resample(ev.county, ev.rect, seed=2000, iteration=4)
    assert abs(np.corrcoef(ux, (x2 - r[:, 0]) / (r[:, 2] - r[:, 0]))[0, 1]) < 0.05
    # deterministic in (seed, iteration, n)
    x3, _ = oracle.resample(ev.county, ev.rect, seed=2000, iteration=3)
    assert np.array_equal(x, x3)


# ------------------------------------------- the paper's uniform background

AREA = 1.0e6  # km^2: a 1000 x 1000 km domain


def test_uniform_background_two_event_closed_form():
    """The paper's own background mu0 / A(X) times the temporal Gaussian (equation "fixed"), N = 2:
    library densities, the source bandwidth of model 2 and the unchanged compensator."""
    mu, tau_x, tau_t, xi, h0, omega = th = _theta(0.7, 3.0, 2.0, 0.4, 1.5, 0.3)
    t = np.array([1.0, 2.2])
    x = np.array([0.5, 1.7])
    y = np.array([-0.3, 0.9])
    s = np.array([0.6, 2.5])
    dt = t[1] - t[0]
    kb = stats.norm.pdf(dt, scale=tau_t) / AREA
    kt = stats.multivariate_normal.pdf([x[1], y[1]], mean=[x[0], y[0]], cov=(h0 * s[0]) ** 2 * np.eye(2)) * \
        stats.expon.pdf(dt, scale=1 / omega)
    lam1, lam2 = mu * kb, mu * kb + xi * kt
    phi = stats.norm.cdf
    comp = sum(mu * (phi((t[1] - tm) / tau_t) - phi(-tm / tau_t)) + xi * (1 - math.exp(-omega * (t[1] - tm)))
               for tm in t)
    ll, g, lam, Lam, _ = oracle.loglik(t, x, y, s, th, per_row=True, area=AREA)
    assert lam[0] == pytest.approx(lam1, rel=1e-13)
    assert lam[1] == pytest.approx(lam2, rel=1e-13)
    assert Lam.sum() == pytest.approx(comp, rel=1e-13)
    assert ll == pytest.approx(math.log(lam1) + math.log(lam2) - comp, rel=1e-13)
    assert g[1] == 0.0  # tau_x plays no part


def test_uniform_background_sum_is_a_temporal_kde():
    t, x, y, s = _small_events(40, 5)
    th = _theta(0.9, 6.0, 4.0, 0.5, 3.0, 0.4)
    bg, _ = oracle.rate_parts(t, x, y, s, th, area=AREA)
    for n in range(len(t)):
        other = t[t != t[n]]
        assert bg[n] == pytest.approx(stats.norm.pdf(t[n] - other, scale=th[2]).sum() / AREA, rel=1e-12)


def test_uniform_background_gradient_against_richardson_finite_differences():
    ev = synth.generate(synth.N2K, n=300, seed=17)
    th = synth.theta_default()
    _, g = oracle.loglik(ev.t, ev.x, ev.y, ev.s, th, area=AREA)

    def f(v):
        return oracle.loglik(ev.t, ev.x, ev.y, ev.s, v, area=AREA)[0]

    for k in range(6):
        h = 1e-4 * th[k]
        e = np.zeros(6)

        def d(hh):
            e[:] = 0.0
            e[k] = hh
            return (f(th + e) - f(th - e)) / (2 * hh)

        rich = (4 * d(h / 2) - d(h)) / 3
        assert g[k] == pytest.approx(rich, rel=2e-7, abs=1e-7 * abs(g).max())


def test_uniform_background_scaling_identities():
    """Space: l(c x, c h0; area c^2 A) = l - 2 N log c.  Time: l(c t, c tau_t, omega / c) = l - N log c.
    Euler: mu dl/dmu + xi dl/dxi = N - Lambda."""
    ev = synth.generate(synth.N2K, n=400, seed=19)
    th = synth.theta_default()
    ll, g, lam, Lam, _ = oracle.loglik(ev.t, ev.x, ev.y, ev.s, th, per_row=True, area=AREA)
    assert (lam > 1e-40).all()
    n = len(ev.t)
    assert th[0] * g[0] + th[3] * g[3] == pytest.approx(n - Lam.sum(), rel=1e-12)
    for c in (0.37, 3.0):
        th2 = th.copy()
        th2[4] *= c
        ll2, _ = oracle.loglik(ev.t, c * ev.x, c * ev.y, ev.s, th2, area=c * c * AREA)
        assert ll2 == pytest.approx(ll - 2 * n * math.log(c), rel=1e-12)
        th3 = th.copy()
        th3[2] *= c
        th3[5] /= c
        ll3, _ = oracle.loglik(c * ev.t, ev.x, ev.y, ev.s, th3, area=AREA)
        assert ll3 == pytest.approx(ll - n * math.log(c), rel=1e-12)
    # tau_x plays no part
    th4 = th.copy()
    th4[1] *= 5.0
    assert oracle.loglik(ev.t, ev.x, ev.y, ev.s, th4, area=AREA)[0] == ll
