"""An oracle-backed cut-posterior target for sampler parity tests (test infrastructure).

OracleCutTarget has the interface of paper_2407_11349_amd.mcmc.cut.HawkesCutTarget (resample,
logp, logp_batch, logp_and_grad, _prior, n_loglik / n_grad counters), with every value from the
FP64 CPU oracle and every latent-location draw from the oracle's Philox4x64-10 draw, so that a
sampler run over it and one over the HIP library with the same seeds must take the same steps.
QuadraticSurrogate is a fixed surrogate (a Gaussian approximation of the log-likelihood around a
point) with the interface of surrogate.Surrogate.value_and_grad, identical for both runs."""

from __future__ import annotations

import numpy as np

import oracle


class OracleCutTarget:
    def __init__(self, t, s, county, rect, seed: int, prior_sd: float = 10.0):
        self.t = np.ascontiguousarray(t, dtype=np.float64)
        self.s = np.ascontiguousarray(s, dtype=np.float64)
        self.county = np.ascontiguousarray(county, dtype=np.int32)
        self.rect = np.ascontiguousarray(rect, dtype=np.float64)
        self.seed = seed
        self.prior_var = prior_sd ** 2
        self.x = self.y = None
        self.n_loglik = 0
        self.n_grad = 0

    def resample(self, iteration: int) -> None:
        self.x, self.y = oracle.resample(self.county, self.rect, self.seed, iteration)

    def _prior(self, z):
        return -0.5 * float(np.dot(z, z)) / self.prior_var, -z / self.prior_var

    @staticmethod
    def _ok(z):
        return np.all(np.isfinite(z)) and not np.any(np.abs(z) > 50)

    def logp(self, z) -> float:
        z = np.asarray(z, dtype=np.float64)
        if not self._ok(z):
            return -np.inf
        ll, _ = oracle.loglik(self.t, self.x, self.y, self.s, np.exp(z))
        self.n_loglik += 1
        return ll + self._prior(z)[0]

    def logp_batch(self, zs) -> np.ndarray:
        return np.array([self.logp(z) for z in zs])

    def logp_and_grad(self, z):
        z = np.asarray(z, dtype=np.float64)
        if not self._ok(z):
            return -np.inf, np.zeros_like(z)
        th = np.exp(z)
        ll, g = oracle.loglik(self.t, self.x, self.y, self.s, th)
        self.n_grad += 1
        lp, gp = self._prior(z)
        return ll + lp, th * g + gp


class QuadraticSurrogate:
    """lhat(z) = c - (z - m)' P (z - m) / 2 with a fixed diagonal precision P."""

    def __init__(self, m, prec, c=0.0):
        self.m = np.asarray(m, dtype=np.float64)
        self.p = np.asarray(prec, dtype=np.float64)
        self.c = float(c)

    def value_and_grad(self, z):
        z = np.atleast_2d(np.asarray(z, dtype=np.float64))
        d = z - self.m
        return self.c - 0.5 * np.sum(self.p * d * d, axis=1), -self.p * d
