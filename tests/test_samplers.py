"""CPU tests of the sampler layer on analytic targets (no GPU)."""

import numpy as np
import pytest

from paper_2407_11349_amd.mcmc import DelayedAcceptanceHMC, HMC, bulk_ess, ess, mcse_mean, split_rhat


def _ar1(rho, n, chains, seed):
    rng = np.random.default_rng(seed)
    x = np.zeros((chains, n))
    e = rng.normal(size=(chains, n)) * np.sqrt(1 - rho**2)
    x[:, 0] = rng.normal(size=chains)
    for t in range(1, n):
        x[:, t] = rho * x[:, t - 1] + e[:, t]
    return x


@pytest.mark.parametrize("rho", [0.0, 0.5, 0.9])
def test_ess_matches_ar1_closed_form(rho):
    """ESS of an AR(1) series is n (1 - rho) / (1 + rho)."""
    x = _ar1(rho, 20000, 4, seed=int(rho * 10))
    expect = x.size * (1 - rho) / (1 + rho)
    assert ess(x) == pytest.approx(expect, rel=0.1)
    assert bulk_ess(x) == pytest.approx(expect, rel=0.1)
    assert split_rhat(x) < 1.01


def test_rhat_flags_chains_that_disagree():
    x = _ar1(0.5, 2000, 4, seed=3)
    x[0] += 1.0
    assert split_rhat(x) > 1.1


class Gauss:
    def __init__(self, mu, Q):
        self.mu, self.Q = np.asarray(mu), np.asarray(Q)
        self.calls = 0

    def logp(self, z):
        d = z - self.mu
        self.calls += 1
        return -0.5 * d @ self.Q @ d

    def logp_and_grad(self, z):
        d = z - self.mu
        self.calls += 1
        return -0.5 * d @ self.Q @ d, -(self.Q @ d)


def _target(seed=0):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(6, 6))
    C = A @ A.T / 6 + 0.2 * np.eye(6)
    mu = rng.normal(size=6)
    return Gauss(mu, np.linalg.inv(C)), mu, C


def _check_moments(draws, mu, C, k=4.5):
    for i in range(6):
        se = mcse_mean(draws[:, i][None, :])
        assert abs(draws[:, i].mean() - mu[i]) < k * se + 1e-3, (i, draws[:, i].mean(), mu[i], se)
    np.testing.assert_allclose(np.cov(draws.T).diagonal(), C.diagonal(), rtol=0.25)


def test_hmc_recovers_gaussian_moments():
    tgt, mu, C = _target(0)
    hmc = HMC(tgt, n_leapfrog=20, step_size=0.1, rng=np.random.default_rng(1))
    s = hmc.init_state(np.zeros(6))
    s = hmc.warmup(s, 400)
    draws, acc = [], 0
    for _ in range(3000):
        s, a, _ = hmc.step(s)
        acc += a
        draws.append(s.z)
    draws = np.array(draws)
    assert 0.5 < acc / 3000 <= 1.0
    _check_moments(draws, mu, C)


def test_delayed_acceptance_is_exact_with_a_wrong_surrogate():
    """The surrogate is a Gaussian with a shifted mean and inflated covariance; the DA kernel
    must still sample the exact target."""
    tgt, mu, C = _target(1)
    bad = Gauss(mu + 0.3 * np.sqrt(C.diagonal()), np.linalg.inv(1.5 * C))
    hmc = HMC(tgt, n_leapfrog=20, step_size=0.1, rng=np.random.default_rng(2))
    s = hmc.warmup(hmc.init_state(np.zeros(6)), 400)
    da = DelayedAcceptanceHMC(tgt, bad.logp_and_grad, n_leapfrog=20, step_size=hmc.eps, inv_mass=hmc.inv_mass,
                              rng=np.random.default_rng(3), fallback_below=0.0)
    st = da.init_state(s.z)
    draws = []
    for _ in range(6000):
        st, _, _ = da.step(st)
        draws.append(st.z)
    draws = np.array(draws)
    assert da.stats["stage1_accept"] > da.stats["stage2_accept"] > 0
    _check_moments(draws, mu, C)


def test_fallback_to_exact_hmc_when_acceptance_collapses():
    """A surrogate pointing far away makes stage 2 reject; the windowed acceptance drops below
    0.5 and exact HMC steps take over, still sampling the target."""
    tgt, mu, C = _target(2)
    awful = Gauss(mu + 8.0, np.linalg.inv(0.05 * C))
    hmc = HMC(tgt, n_leapfrog=20, step_size=0.1, rng=np.random.default_rng(4))
    s = hmc.warmup(hmc.init_state(np.zeros(6)), 400)
    da = DelayedAcceptanceHMC(tgt, awful.logp_and_grad, n_leapfrog=20, step_size=hmc.eps, inv_mass=hmc.inv_mass,
                              rng=np.random.default_rng(5), window=20, fallback_below=0.5)
    st = da.init_state(s.z)
    draws = []
    for _ in range(3000):
        st, _, _ = da.step(st)
        draws.append(st.z)
    assert da.stats["fallback"] > 1000
    _check_moments(np.array(draws), mu, C)


def test_good_surrogate_needs_few_exact_evaluations():
    """With the exact density as its own surrogate, stage 2 always accepts and each iteration costs
    one exact log-density evaluation instead of n_leapfrog gradients."""
    tgt, mu, C = _target(3)
    sur = Gauss(mu, tgt.Q)
    da = DelayedAcceptanceHMC(tgt, sur.logp_and_grad, n_leapfrog=20, step_size=0.1, rng=np.random.default_rng(6))
    st = da.init_state(np.zeros(6))
    tgt.calls = 0
    for _ in range(500):
        st, _, _ = da.step(st)
    assert da.stats["stage2_accept"] == da.stats["stage1_accept"]
    assert tgt.calls == da.stats["stage1_accept"] <= 500


def test_univariate_mh_recovers_gaussian_moments_and_adapts():
    """The paper's sampler: one-coordinate random-walk updates reach the Gaussian's moments, and
    warm-up adaptation brings every coordinate's acceptance near 0.44."""
    from paper_2407_11349_amd.mcmc.mh import UnivariateMH

    tgt, mu, C = _target(2)
    mh = UnivariateMH(tgt, scales=np.full(6, 0.05), rng=np.random.default_rng(4))
    z = np.zeros(6)
    lp = tgt.logp(z)
    for it in range(3000):
        z, lp = mh.sweep(z, lp, adapt_rate=0.5 / np.sqrt(it + 1.0))
    mh.accepts[:] = 0
    mh.tries[:] = 0
    draws = []
    for it in range(20000):
        z, lp = mh.sweep(z, lp)
        draws.append(z.copy())
    draws = np.array(draws)
    assert np.all(np.abs(mh.acceptance() - 0.44) < 0.1)
    _check_moments(draws, mu, C)
    assert lp == pytest.approx(tgt.logp(z))


class DrawTarget(Gauss):
    """A Gaussian whose mean moves with every latent-location draw (as l(theta; X) does), with a
    batched log density that records how many vectors each call carries."""

    def __init__(self, mu, Q):
        super().__init__(mu, Q)
        self.mu0 = self.mu.copy()
        self.batches = []

    def resample(self, it):
        self.mu = self.mu0 + 0.05 * np.random.default_rng([7, it]).normal(size=6)

    def logp_batch(self, zs):
        self.batches.append(len(zs))
        return np.array([Gauss.logp(self, z) for z in zs])


def test_delayed_acceptance_lazy_refresh_pairs_exact_values():
    """After each draw the current point's exact value is recomputed only when a proposal reaches
    stage 2, in one two-vector call; the chain equals the one that recomputes it eagerly."""
    from paper_2407_11349_amd.mcmc.da_hmc import DAState

    _, mu, C = _target(4)
    chains = []
    for lazy in (True, False):
        tgt = DrawTarget(mu, np.linalg.inv(C))
        sur = Gauss(mu + 0.1, np.linalg.inv(1.2 * C))
        da = DelayedAcceptanceHMC(tgt, sur.logp_and_grad, n_leapfrog=10, step_size=0.15,
                                  rng=np.random.default_rng(8), fallback_below=0.0)
        tgt.resample(0)
        st = da.init_state(np.zeros(6))
        zs = []
        for it in range(400):
            st, _, _ = da.step(st)
            zs.append(st.z.copy())
            tgt.resample(it + 1)
            st = da.refresh_exact(st) if lazy else DAState(st.z, Gauss.logp(tgt, st.z), st.s, st.s_grad)
        chains.append(np.array(zs))
        if lazy:
            # every stage-2 correction after the first draw change takes the paired call
            assert da.stats["stage1_accept"] - 1 <= da.stats["paired_exact"] <= da.stats["stage1_accept"]
            assert da.stats["paired_exact"] > 100
            assert tgt.batches and set(tgt.batches) == {2}
    np.testing.assert_allclose(chains[0], chains[1], rtol=0, atol=1e-12)


def test_univariate_mh_pairs_the_refreshed_density_with_the_first_proposal():
    """After a new draw the current point's density and the first proposal's come from one
    two-vector call; the chain equals the one that evaluates them one at a time."""
    from paper_2407_11349_amd.mcmc.mh import UnivariateMH

    _, mu, C = _target(5)
    chains = []
    for paired in (True, False):
        tgt = DrawTarget(mu, np.linalg.inv(C))
        if not paired:
            tgt.logp_batch = None  # the sampler then calls logp twice
        mh = UnivariateMH(tgt, scales=np.full(6, 0.3), rng=np.random.default_rng(9))
        z = np.zeros(6)
        zs = []
        for it in range(300):
            tgt.resample(it)
            z, _ = mh.sweep(z)
            zs.append(z.copy())
        chains.append(np.array(zs))
        if paired:
            assert tgt.batches == [2] * 300
    np.testing.assert_allclose(chains[0], chains[1], rtol=0, atol=0)


def test_step_size_jitter_breaks_a_resonant_trajectory_length():
    """On a standard normal a trajectory of one full period (20 steps of 2 pi / 20) returns close to
    its start, so fixed-length HMC barely mixes; jittering the step size per iteration (+-20%) mixes,
    and still samples the target."""
    from paper_2407_11349_amd.mcmc.hmc import HMC

    tgt = Gauss(np.zeros(6), np.eye(6))
    out = {}
    for jitter in (0.0, 0.2):
        hmc = HMC(tgt, n_leapfrog=20, step_size=2 * np.pi / 20, rng=np.random.default_rng(10), jitter=jitter)
        s = hmc.init_state(np.full(6, 0.5))
        draws = []
        for _ in range(3000):
            s, _, _ = hmc.step(s)
            draws.append(s.z)
        out[jitter] = np.array(draws)
    stuck, mixed = out[0.0], out[0.2]
    assert bulk_ess(stuck[:, 0].reshape(1, -1)) < 20  # creeps along with the leapfrog's period error
    assert bulk_ess(mixed[:, 0].reshape(1, -1)) > 300
    _check_moments(mixed, np.zeros(6), np.eye(6))


def test_windowed_fallback_follows_the_state_and_biases_a_fixed_mixture_does_not():
    """The exact-HMC fallback chosen by recent acceptance depends on where the chain is: with a
    surrogate that is exact for z0 < 0 and far too narrow in z0 for z0 >= 0, acceptance drops on the
    right, exact HMC takes over there, and the chain under-visits the right half (a biased mean and
    a shrunken variance of z0 under a standard normal target).  An exact-HMC step taken with a fixed
    probability each iteration is a fixed mixture of invariant kernels and samples the target."""

    class Std:
        prior_var = 1e4

        def logp(self, z):
            return -0.5 * float(z @ z)

        def logp_and_grad(self, z):
            return -0.5 * float(z @ z), -z

    def sur(z):
        if z[0] < 0:
            return -0.5 * float(z @ z), -z.copy()
        g = -z.copy()
        g[0] -= 4.0 * z[0]
        return -0.5 * float(z @ z) - 2.0 * z[0] ** 2, g

    def run(**kw):
        da = DelayedAcceptanceHMC(Std(), sur, dim=2, n_leapfrog=8, step_size=0.25, rng=np.random.default_rng(11),
                                  window=50, **kw)
        st = da.init_state(np.zeros(2))
        d = np.empty((20000, 2))
        for i in range(d.shape[0]):
            st, _, _ = da.step(st)
            d[i] = st.z
        return d[:, 0], da.stats

    z0, stats = run(fallback_below=0.5)
    assert stats["fallback"] > 0
    assert z0.mean() < -8 * mcse_mean(z0[None, :]) and z0.var() < 0.8
    z0, stats = run(fallback_below=0.5, fallback_prob=0.2)
    assert stats["fallback"] > 0
    assert abs(z0.mean()) < 4 * mcse_mean(z0[None, :]) and abs(z0.var() - 1.0) < 0.1
    with pytest.raises(ValueError):
        DelayedAcceptanceHMC(Std(), sur, dim=2, fallback_prob=1.0)
