"""Failure handling of the sampler layer (CPU): a likelihood or surrogate that returns NaN.

The paper's rewrite of its GPU kernel was motivated by NaNs the earlier kernel produced at large N
(Section 2.3).  A Metropolis-type kernel stays exact only if a proposal whose density cannot be
evaluated is rejected; a NaN must never turn into an acceptance (Python's min(0.0, nan) is 0.0, which a
plain min(1, exp(r)) rule would read as probability 1).  A chain whose current point has no finite density
cannot continue and stops with an error."""

import numpy as np
import pytest

from paper_2407_11349_amd.mcmc import DelayedAcceptanceHMC, HMC, NonFiniteStateError, UnivariateMH, accept_prob


class NaNRegionGauss:
    """Standard normal in 6 dimensions whose density and gradient are NaN where z[0] > cut (a fake
    likelihood that fails on part of the space), counting the NaN values it handed out."""

    def __init__(self, cut=0.3):
        self.cut = cut
        self.nan_calls = 0

    def _bad(self, z):
        bad = bool(z[0] > self.cut)
        self.nan_calls += bad
        return bad

    def logp(self, z):
        z = np.asarray(z, dtype=np.float64)
        return np.nan if self._bad(z) else -0.5 * float(z @ z)

    def logp_and_grad(self, z):
        z = np.asarray(z, dtype=np.float64)
        if self._bad(z):
            return np.nan, np.full(6, np.nan)
        return -0.5 * float(z @ z), -z


class NaNEveryKth:
    """Standard normal whose k-th, 2k-th, ... density evaluation returns NaN wherever it is asked."""

    def __init__(self, k):
        self.k, self.calls, self.nan_calls = k, 0, 0

    def _bad(self):
        self.calls += 1
        bad = self.calls % self.k == 0
        self.nan_calls += bad
        return bad

    def logp(self, z):
        z = np.asarray(z, dtype=np.float64)
        return np.nan if self._bad() else -0.5 * float(z @ z)

    def logp_and_grad(self, z):
        z = np.asarray(z, dtype=np.float64)
        if self._bad():
            return np.nan, np.full(6, np.nan)
        return -0.5 * float(z @ z), -z


def test_accept_prob_rejects_non_finite_ratios():
    assert accept_prob(np.nan) == 0.0
    assert accept_prob(np.inf) == 0.0
    assert accept_prob(-np.inf) == 0.0
    assert accept_prob(0.3) == 1.0
    assert accept_prob(-1.0) == pytest.approx(np.exp(-1.0))


def test_hmc_rejects_every_proposal_whose_density_is_nan():
    tgt = NaNRegionGauss(cut=0.3)
    hmc = HMC(tgt, n_leapfrog=10, step_size=0.3, rng=np.random.default_rng(4))
    s = hmc.init_state(np.full(6, -0.2))
    draws = []
    for _ in range(600):
        s, _, _ = hmc.step(s)
        draws.append(s.z.copy())
        assert np.isfinite(s.logp) and np.all(np.isfinite(s.grad))
    draws = np.array(draws)
    assert tgt.nan_calls > 0, "the test must reach the NaN region"
    assert np.all(draws[:, 0] <= tgt.cut), "a proposal with a NaN density was accepted"


def test_hmc_rejects_a_trajectory_with_a_nan_midway():
    tgt = NaNEveryKth(7)
    hmc = HMC(tgt, n_leapfrog=10, step_size=0.2, rng=np.random.default_rng(5))
    s = hmc.init_state(np.zeros(6))
    for _ in range(200):
        s, acc, a = hmc.step(s)
        assert np.isfinite(s.logp)
    assert tgt.nan_calls > 0


def test_chain_cannot_start_where_the_density_is_nan():
    tgt = NaNRegionGauss(cut=0.3)
    with pytest.raises(NonFiniteStateError):
        HMC(tgt).init_state(np.full(6, 1.0))
    with pytest.raises(NonFiniteStateError):
        DelayedAcceptanceHMC(tgt, lambda z: (-0.5 * float(z @ z), -z)).init_state(np.full(6, 1.0))
    mh = UnivariateMH(tgt, rng=np.random.default_rng(0))
    with pytest.raises(NonFiniteStateError):
        mh.sweep(np.full(6, 1.0), None)


def test_delayed_acceptance_rejects_nan_exact_values_and_nan_surrogate_proposals():
    tgt = NaNRegionGauss(cut=0.3)
    sur_nan = [0]

    def sur(z):
        # a surrogate that is itself NaN in a second region (z[1] > 0.4)
        z = np.asarray(z)
        if z[1] > 0.4:
            sur_nan[0] += 1
            return np.nan, np.full(6, np.nan)
        return -0.5 * float(z @ z) * 1.05, -1.05 * z

    da = DelayedAcceptanceHMC(tgt, sur, n_leapfrog=10, step_size=0.3, rng=np.random.default_rng(6), window=10**9)
    st = da.init_state(np.full(6, -0.2))
    zs = []
    for _ in range(600):
        st, _, _ = da.step(st)
        zs.append(st.z.copy())
        assert np.isfinite(st.s)
    zs = np.array(zs)
    assert tgt.nan_calls > 0 and sur_nan[0] > 0
    assert np.all(zs[:, 0] <= 0.3), "stage 2 accepted a proposal whose exact density is NaN"
    assert np.all(zs[:, 1] <= 0.4), "stage 1 accepted a proposal whose surrogate density is NaN"


def test_delayed_acceptance_stops_when_the_current_points_exact_value_is_nan():
    """Under the cut posterior the current point's exact value is recomputed after each latent draw; if the
    likelihood then fails there, the chain stops rather than rejecting forever against a NaN."""

    class FailsAfter:
        def __init__(self):
            self.broken = False

        def logp(self, z):
            return np.nan if self.broken else -0.5 * float(np.dot(z, z))

        def logp_batch(self, zs):
            return np.array([self.logp(z) for z in zs])

        def logp_and_grad(self, z):
            z = np.asarray(z)
            return (np.nan, np.full(6, np.nan)) if self.broken else (-0.5 * float(z @ z), -z)

    tgt = FailsAfter()
    da = DelayedAcceptanceHMC(tgt, lambda z: (-0.5 * float(np.dot(z, z)), -np.asarray(z)), n_leapfrog=5,
                              step_size=0.2, rng=np.random.default_rng(7))
    st = da.init_state(np.zeros(6))
    tgt.broken = True
    st = da.refresh_exact(st)
    with pytest.raises(NonFiniteStateError):
        for _ in range(50):  # the first proposal that survives stage 1 needs the current exact value
            st, _, _ = da.step(st)


def test_univariate_mh_rejects_nan_proposals():
    tgt = NaNRegionGauss(cut=0.3)
    mh = UnivariateMH(tgt, scales=np.full(6, 0.8), rng=np.random.default_rng(8))
    z, lp = np.full(6, -0.2), None
    for _ in range(300):
        z, lp = mh.sweep(z, lp)
        assert z[0] <= tgt.cut and np.isfinite(lp)
    assert tgt.nan_calls > 0
