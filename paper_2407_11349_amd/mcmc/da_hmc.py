"""Delayed-acceptance HMC with a surrogate log-likelihood (Christen and Fox,
2005, applied to HMC proposals), with an exact-HMC fallback.

Stage 1: a leapfrog trajectory driven by the surrogate posterior
s(z) = lhat(z) + log prior(z) is accepted with min(1, exp(H_s(z, p) - H_s(z', p'))),
H_s = -s + kinetic.  Stage 2: the exact log posterior corrects it with
min(1, exp([logp(z') - s(z')] - [logp(z) - s(z)])).  The composite kernel
leaves the exact posterior invariant whatever the surrogate's error; the
surrogate only changes how often proposals survive.  When the acceptance rate
over the last `window` iterations falls below `fallback_below`, iterations are
exact HMC (exact gradients) until it recovers.
"""

from __future__ import annotations

from collections import deque
from dataclasses import dataclass

import numpy as np

from .hmc import HMC, HMCState, kinetic, leapfrog


@dataclass
class DAState:
    z: np.ndarray
    logp: float          # exact log posterior at z (under the current target)
    s: float             # surrogate log posterior at z
    s_grad: np.ndarray   # its gradient


class DelayedAcceptanceHMC:
    def __init__(self, target, surrogate_logp_and_grad, dim=6, n_leapfrog=20, step_size=0.05, inv_mass=None,
                 rng=None, window=50, fallback_below=0.5):
        self.target = target
        self.sur = surrogate_logp_and_grad
        self.dim = dim
        self.n_leapfrog = n_leapfrog
        self.eps = step_size
        self.inv_mass = np.ones(dim) if inv_mass is None else np.asarray(inv_mass, dtype=np.float64)
        self.rng = np.random.default_rng(0) if rng is None else rng
        self.window = deque(maxlen=window)
        self.fallback_below = fallback_below
        self.exact = HMC(target, dim=dim, n_leapfrog=n_leapfrog, step_size=step_size, inv_mass=self.inv_mass,
                         rng=self.rng)
        self.stats = {"iterations": 0, "stage1_accept": 0, "stage2_accept": 0, "fallback": 0, "accept": 0}

    def init_state(self, z) -> DAState:
        z = np.asarray(z, dtype=np.float64)
        s, sg = self.sur(z)
        return DAState(z, self.target.logp(z), s, sg)

    def refresh_exact(self, st: DAState) -> DAState:
        """Recompute the exact log posterior at the current point (after the target changed)."""
        return DAState(st.z, self.target.logp(st.z), st.s, st.s_grad)

    def in_fallback(self) -> bool:
        return len(self.window) == self.window.maxlen and np.mean(self.window) < self.fallback_below

    def step(self, st: DAState):
        self.stats["iterations"] += 1
        if self.in_fallback():
            self.stats["fallback"] += 1
            self.exact.eps = self.eps
            self.exact.inv_mass = self.inv_mass
            hs = self.exact.init_state(st.z)
            new, acc, _ = self.exact.step(hs)
            self.window.append(1.0 if acc else 0.0)
            if acc:
                self.stats["accept"] += 1
                s, sg = self.sur(new.z)
                return DAState(new.z, new.logp, s, sg), acc, "fallback"
            return st, acc, "fallback"
        p0 = self.rng.normal(size=self.dim) / np.sqrt(self.inv_mass)
        z1, p1, s1, sg1 = leapfrog(st.z, p0, st.s_grad, self.eps, self.inv_mass, self.n_leapfrog, self.sur)
        h0 = -st.s + kinetic(p0, self.inv_mass)
        h1 = -s1 + kinetic(p1, self.inv_mass)
        a1 = float(np.exp(min(0.0, h0 - h1))) if np.isfinite(h1) else 0.0
        if not (self.rng.uniform() < a1):
            self.window.append(0.0)
            return st, False, "stage1"
        self.stats["stage1_accept"] += 1
        logp1 = self.target.logp(z1)
        log_a2 = (logp1 - s1) - (st.logp - st.s)
        a2 = float(np.exp(min(0.0, log_a2))) if np.isfinite(logp1) else 0.0
        if self.rng.uniform() < a2:
            self.stats["stage2_accept"] += 1
            self.stats["accept"] += 1
            self.window.append(1.0)
            return DAState(z1, logp1, s1, sg1), True, "accept"
        self.window.append(0.0)
        return st, False, "stage2"
