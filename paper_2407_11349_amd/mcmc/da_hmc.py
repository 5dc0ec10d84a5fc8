"""Delayed-acceptance HMC with a surrogate log-likelihood (Christen and Fox,
2005, applied to HMC proposals), with an exact-HMC fallback.

Stage 1: a leapfrog trajectory driven by the surrogate posterior
s(z) = lhat(z) + log prior(z) is accepted with min(1, exp(H_s(z, p) - H_s(z', p'))),
H_s = -s + kinetic.  Stage 2: the exact log posterior corrects it with
min(1, exp([logp(z') - s(z')] - [logp(z) - s(z)])).  The composite kernel
leaves the exact posterior invariant whatever the surrogate's error; the
surrogate only changes how often proposals survive.

Exact-HMC fallback, two rules:
  window   (fallback_prob = 0) when the acceptance rate over the last `window`
           iterations falls below `fallback_below`, iterations are exact HMC
           (exact gradients) until it recovers.  The choice of kernel then
           depends on the chain's recent past, and through it on where the
           chain is: where the surrogate is poor, acceptance drops and exact
           HMC takes over.  Each kernel leaves the posterior invariant, but a
           choice that follows the state does not in general: with a surrogate
           that is poor in one half-space the chain under-visits that half
           (tests/test_samplers.py).
  mixture  (fallback_prob = q > 0) each iteration is an exact-HMC step with the
           fixed probability q and a delayed-acceptance step otherwise; a fixed
           mixture of invariant kernels is invariant.

Under the cut posterior the target changes with every latent-location draw, so
the exact value at the current point is needed afresh each iteration, but only
when a proposal reaches stage 2.  It is computed then, together with the
proposal's value in one two-vector evaluation when the target offers
`logp_batch` (the FP32 sweep forms each pair's geometry once for both).
"""

from __future__ import annotations

from collections import deque
from dataclasses import dataclass

import numpy as np

from .hmc import HMC, accept_prob, check_state, kinetic, leapfrog


@dataclass
class DAState:
    z: np.ndarray
    logp: float | None   # exact log posterior at z under the current target (None: not yet computed)
    s: float             # surrogate log posterior at z
    s_grad: np.ndarray   # its gradient


class DelayedAcceptanceHMC:
    def __init__(self, target, surrogate_logp_and_grad, dim=6, n_leapfrog=20, step_size=0.05, inv_mass=None,
                 rng=None, window=50, fallback_below=0.5, trajectory=None, jitter=0.0, fallback_prob=0.0):
        """trajectory(z, p, grad, eps, inv_mass, n_steps) -> (z, p, s, grad), if given, runs the whole stage-1
        leapfrog trajectory on the surrogate at once (e.g. on the GPU) instead of step by step here.
        fallback_prob > 0 selects the mixture fallback rule (module docstring) instead of the window rule."""
        if not (0.0 <= fallback_prob < 1.0):
            raise ValueError("fallback_prob must be in [0, 1)")
        self.fallback_prob = float(fallback_prob)
        self.target = target
        self.sur = surrogate_logp_and_grad
        self.trajectory = trajectory
        self.dim = dim
        self.n_leapfrog = n_leapfrog
        self.eps = step_size
        self.inv_mass = np.ones(dim) if inv_mass is None else np.asarray(inv_mass, dtype=np.float64)
        self.rng = np.random.default_rng(0) if rng is None else rng
        self.window = deque(maxlen=window)
        self.fallback_below = fallback_below
        self.exact = HMC(target, dim=dim, n_leapfrog=n_leapfrog, step_size=step_size, inv_mass=self.inv_mass,
                         rng=self.rng, jitter=jitter)
        self.stats = {"iterations": 0, "stage1_accept": 0, "stage2_accept": 0, "fallback": 0, "accept": 0,
                      "paired_exact": 0}

    def init_state(self, z) -> DAState:
        z = np.asarray(z, dtype=np.float64)
        s, sg = self.sur(z)
        check_state(z, s, sg, "surrogate log density")
        lp = self.target.logp(z)
        check_state(z, lp)
        return DAState(z, lp, s, sg)

    def refresh_exact(self, st: DAState) -> DAState:
        """The target changed (a new latent-location draw): the exact value at the current point is
        stale and is recomputed when a stage-2 correction next needs it."""
        return DAState(st.z, None, st.s, st.s_grad)

    def _exact_pair(self, z0, z1):
        """Exact log posteriors at the current point and the proposal under the same target."""
        batch = getattr(self.target, "logp_batch", None)
        self.stats["paired_exact"] += 1
        if batch is not None:
            v = batch([z0, z1])
            return float(v[0]), float(v[1])
        return self.target.logp(z0), self.target.logp(z1)

    def in_fallback(self) -> bool:
        return len(self.window) == self.window.maxlen and np.mean(self.window) < self.fallback_below

    def step(self, st: DAState):
        self.stats["iterations"] += 1
        use_exact = (self.rng.uniform() < self.fallback_prob) if self.fallback_prob > 0.0 else self.in_fallback()
        if use_exact:
            self.stats["fallback"] += 1
            self.exact.eps = self.eps
            self.exact.inv_mass = self.inv_mass
            hs = self.exact.init_state(st.z)
            new, acc, _ = self.exact.step(hs)
            self.window.append(1.0 if acc else 0.0)
            if acc:
                self.stats["accept"] += 1
                s, sg = self.sur(new.z)
                check_state(new.z, s, sg, "surrogate log density")
                return DAState(new.z, new.logp, s, sg), acc, "fallback"
            return st, acc, "fallback"
        self.exact.eps = self.eps
        eps = self.exact.jittered_eps()
        p0 = self.rng.normal(size=self.dim) / np.sqrt(self.inv_mass)
        if self.trajectory is not None:
            z1, p1, s1, sg1 = self.trajectory(st.z, p0, st.s_grad, eps, self.inv_mass, self.n_leapfrog)
        else:
            z1, p1, s1, sg1 = leapfrog(st.z, p0, st.s_grad, eps, self.inv_mass, self.n_leapfrog, self.sur)
        h0 = -st.s + kinetic(p0, self.inv_mass)
        h1 = -s1 + kinetic(p1, self.inv_mass)
        a1 = accept_prob(h0 - h1)
        if not (self.rng.uniform() < a1):
            self.window.append(0.0)
            return st, False, "stage1"
        self.stats["stage1_accept"] += 1
        if st.logp is None:
            lp0, logp1 = self._exact_pair(st.z, z1)
            check_state(st.z, lp0)
            st = DAState(st.z, lp0, st.s, st.s_grad)
        else:
            logp1 = self.target.logp(z1)
        log_a2 = (logp1 - s1) - (st.logp - st.s)
        a2 = accept_prob(log_a2)
        if self.rng.uniform() < a2:
            self.stats["stage2_accept"] += 1
            self.stats["accept"] += 1
            self.window.append(1.0)
            return DAState(z1, logp1, s1, sg1), True, "accept"
        self.window.append(0.0)
        return st, False, "stage2"
