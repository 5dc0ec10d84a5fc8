"""CPU test of the cut-posterior experiment driver with a fake target whose density
moves a little with every latent-location draw (as l(theta; X) does), and a fixed
surrogate of the X-averaged log-likelihood."""

import numpy as np

from paper_2407_11349_amd.mcmc import experiment as ex


class FakeCutTarget:
    prior_var = 100.0

    def __init__(self, mu, Q, jitter=0.05, seed=0):
        self.mu0, self.Q = np.asarray(mu), np.asarray(Q)
        self.mu = self.mu0.copy()
        self.jitter = jitter
        self.seed = seed
        self.n_loglik = 0
        self.n_grad = 0

    def resample(self, iteration):
        rng = np.random.default_rng([self.seed, iteration])
        self.mu = self.mu0 + self.jitter * rng.normal(size=self.mu0.shape)

    def _prior(self, z):
        return -0.5 * float(z @ z) / self.prior_var, -z / self.prior_var

    def _ll(self, z):
        d = z - self.mu
        return -0.5 * d @ self.Q @ d, -(self.Q @ d)

    def logp(self, z):
        self.n_loglik += 1
        return self._ll(z)[0] + self._prior(z)[0]

    def logp_and_grad(self, z):
        self.n_grad += 1
        ll, g = self._ll(z)
        lp, gp = self._prior(z)
        return ll + lp, g + gp


class FakeSurrogate:
    def __init__(self, mu, Q):
        self.mu, self.Q = mu, Q

    def value_and_grad(self, z):
        z = np.atleast_2d(z)
        d = z - self.mu
        return -0.5 * np.einsum("bi,ij,bj->b", d, self.Q, d), -(d @ self.Q)


def test_burn_in_records_tuples_and_chains_agree():
    rng = np.random.default_rng(0)
    A = rng.normal(size=(6, 6))
    C = (A @ A.T / 6 + 0.3 * np.eye(6)) * 0.01
    mu = rng.normal(size=6) * 0.1
    Q = np.linalg.inv(C)
    tgt = FakeCutTarget(mu, Q)
    n0 = tgt.n_grad
    hmc, st, rec, _ = ex.burn_in(tgt, mu + 3.0, 300, n_leapfrog=10, seed=1, n_warmup=200)
    # the mode search reaches the posterior from a distant start
    assert np.all(np.abs(st.z - mu) < 1.0)
    # after warm-up, every gradient evaluation is recorded with the prior removed:
    # 10 leapfrog points and one start-of-iteration evaluation per iteration, plus the first
    assert len(rec.z) == 300 * 11 + 1 and tgt.n_grad - n0 > len(rec.z)
    plain = ex.run_plain_hmc(tgt, hmc, st.z, 1500, it0=1000)
    da = ex.run_da_hmc(tgt, FakeSurrogate(mu, Q), hmc, st.z, 1500, it0=5000, prior_var=tgt.prior_var)
    # cost: plain HMC needs n_leapfrog + 1 gradients per iteration; DA one or two log-densities,
    # except in fallback iterations (exact HMC: 1 + n_leapfrog gradients)
    assert plain.n_grad == 1500 * 11 + 1
    assert da.n_grad == 11 * da.stats["fallback"]
    assert da.n_loglik <= 2 * 1500 + 1
    assert da.stats["fallback"] < 0.2 * 1500
    sp, sd = ex._summary(plain.draws), ex._summary(da.draws)
    se = np.sqrt(np.array(sp["mcse"]) ** 2 + np.array(sd["mcse"]) ** 2)
    assert np.all(np.abs(np.array(sp["mean"]) - np.array(sd["mean"])) < 4.5 * se + 1e-4)


def test_univariate_mh_chain_on_the_cut_target():
    """The paper's univariate MH under per-iteration latent draws: 7 log-densities per sweep
    (one after the draw, six proposals), no gradients, and means that agree with plain HMC."""
    rng = np.random.default_rng(1)
    A = rng.normal(size=(6, 6))
    C = (A @ A.T / 6 + 0.3 * np.eye(6)) * 0.01
    mu = rng.normal(size=6) * 0.1
    Q = np.linalg.inv(C)
    tgt = FakeCutTarget(mu, Q)
    hmc, st, _, _ = ex.burn_in(tgt, mu, 200, n_leapfrog=10, seed=2, n_warmup=200)
    mh = ex.run_mh(tgt, st.z, hmc.inv_mass, 3000, it0=20000)
    assert mh.n_grad == 0 and mh.n_loglik == 3000 * 7
    acc = np.array(mh.stats["acceptance"])
    assert np.all((acc > 0.2) & (acc < 0.7))
    plain = ex.run_plain_hmc(tgt, hmc, st.z, 3000, it0=40000)
    sp, sm = ex._summary(plain.draws), ex._summary(mh.draws)
    se = np.sqrt(np.array(sp["mcse"]) ** 2 + np.array(sm["mcse"]) ** 2)
    assert np.all(np.abs(np.array(sp["mean"]) - np.array(sm["mean"])) < 4.5 * se + 1e-4)
