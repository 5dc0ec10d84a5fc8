"""Hamiltonian Monte Carlo over the log-parameters z = log theta.

Targets expose ``logp_and_grad(z) -> (float, ndarray)`` and ``logp(z) -> float``.
The step size is tuned during warm-up by dual averaging (Hoffman and Gelman,
2014, Section 3.2) towards a target acceptance rate, and a diagonal inverse
mass matrix is set from the warm-up draws at mid warm-up.  After warm-up the
step size can be jittered per iteration, uniformly within +-jitter of its
value (Neal, 2011, Section 4.2), so that no fixed trajectory length resonates
with a period of the target.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class DualAveraging:
    log_eps0: float
    target: float = 0.8
    gamma: float = 0.05
    t0: float = 10.0
    kappa: float = 0.75
    mu: float = field(init=False)
    hbar: float = 0.0
    log_eps_bar: float = 0.0
    t: int = 0

    def __post_init__(self):
        self.mu = np.log(10.0) + self.log_eps0

    def update(self, accept_prob: float) -> float:
        self.t += 1
        w = 1.0 / (self.t + self.t0)
        self.hbar = (1.0 - w) * self.hbar + w * (self.target - accept_prob)
        log_eps = self.mu - np.sqrt(self.t) / self.gamma * self.hbar
        eta = self.t ** (-self.kappa)
        self.log_eps_bar = eta * log_eps + (1.0 - eta) * self.log_eps_bar
        return float(np.exp(log_eps))

    def final(self) -> float:
        return float(np.exp(self.log_eps_bar))


def leapfrog(z, p, grad, eps, inv_mass, n_steps, grad_fn):
    """n_steps leapfrog steps of H(z, p) = -logp(z) + p' M^-1 p / 2.  grad is d logp/dz at z.
    Returns (z, p, logp, grad) at the end point; grad_fn(z) -> (logp, grad)."""
    z = z.copy()
    p = p + 0.5 * eps * grad
    logp = None
    for i in range(n_steps):
        z = z + eps * inv_mass * p
        logp, grad = grad_fn(z)
        if not np.isfinite(logp) or not np.all(np.isfinite(grad)):
            return z, p, -np.inf, grad
        if i + 1 < n_steps:
            p = p + eps * grad
    p = p + 0.5 * eps * grad
    return z, p, logp, grad


def kinetic(p, inv_mass):
    return 0.5 * float(np.sum(inv_mass * p * p))


def accept_prob(log_ratio) -> float:
    """Metropolis acceptance probability min(1, exp(log_ratio)); a log ratio that is not finite (NaN from a
    failed density evaluation, or +-inf) rejects.  (Python's min(0.0, nan) is 0.0, so the plain rule would
    accept a NaN.)"""
    r = float(log_ratio)
    return float(np.exp(min(0.0, r))) if np.isfinite(r) else 0.0


class NonFiniteStateError(RuntimeError):
    """A chain's current point has a log density or gradient that is not finite: no valid Markov chain
    continues from there, so the sampler stops instead of rejecting every proposal against it."""


def check_state(z, logp, grad=None, what="log density"):
    if not np.isfinite(logp) or (grad is not None and not np.all(np.isfinite(grad))):
        raise NonFiniteStateError(f"{what} at the current point z = {np.asarray(z).tolist()} is not finite "
                                  f"(value {logp}, gradient {None if grad is None else np.asarray(grad).tolist()})")


@dataclass
class HMCState:
    z: np.ndarray
    logp: float
    grad: np.ndarray


class HMC:
    """Plain HMC with exact gradients (n_leapfrog gradient evaluations per iteration)."""

    def __init__(self, target, dim=6, n_leapfrog=20, step_size=0.05, inv_mass=None, rng=None, jitter=0.0):
        self.target = target
        self.dim = dim
        self.n_leapfrog = n_leapfrog
        self.eps = step_size
        self.jitter = jitter
        self.inv_mass = np.ones(dim) if inv_mass is None else np.asarray(inv_mass, dtype=np.float64)
        self.rng = np.random.default_rng(0) if rng is None else rng

    def init_state(self, z) -> HMCState:
        z = np.asarray(z, dtype=np.float64)
        logp, grad = self.target.logp_and_grad(z)
        check_state(z, logp, grad)
        return HMCState(z, logp, grad)

    def jittered_eps(self) -> float:
        """The step size of one iteration: eps, or eps (1 + jitter U(-1, 1)) with jitter > 0."""
        if self.jitter <= 0.0:
            return self.eps
        return self.eps * (1.0 + self.jitter * (2.0 * self.rng.uniform() - 1.0))

    def step(self, s: HMCState, eps=None):
        eps = self.jittered_eps() if eps is None else eps
        p0 = self.rng.normal(size=self.dim) / np.sqrt(self.inv_mass)
        z1, p1, logp1, grad1 = leapfrog(s.z, p0, s.grad, eps, self.inv_mass, self.n_leapfrog,
                                        self.target.logp_and_grad)
        h0 = -s.logp + kinetic(p0, self.inv_mass)
        h1 = -logp1 + kinetic(p1, self.inv_mass)
        a = accept_prob(h0 - h1)
        if self.rng.uniform() < a:
            return HMCState(z1, logp1, grad1), True, a
        return s, False, a

    def warmup(self, s: HMCState, n_warmup: int, target_accept=0.8, on_step=None):
        """Tune the step size (dual averaging) and a diagonal mass from the warm-up draws."""
        da = DualAveraging(np.log(self.eps), target=target_accept)
        draws = []
        half = n_warmup // 2
        for it in range(n_warmup):
            s, acc, a = self.step(s, self.eps)
            if on_step:
                on_step(it, s, acc)
            self.eps = da.update(a)
            draws.append(s.z.copy())
            if it + 1 == half and half >= 20:
                w = np.array(draws[half // 2:])
                var = w.var(axis=0)
                if np.all(var > 0):
                    self.inv_mass = var
                da = DualAveraging(np.log(self.eps), target=target_accept)
        self.eps = da.final()
        return s
