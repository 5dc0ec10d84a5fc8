"""The paper's own parameter kernel: random-walk Metropolis-Hastings with univariate
updates (Section 2.3.2, run inside the cut-posterior scheme of Section 2.2).

Each sweep updates the log-parameters z = log theta one coordinate at a time with a
Gaussian random-walk proposal; every proposal costs one exact log-density (the
forward-only sweep, no gradient).  The proposal scales adapt during warm-up
towards the acceptance rate 0.44 that suits one-dimensional random walks, and are
fixed afterwards.
"""

from __future__ import annotations

import numpy as np


class UnivariateMH:
    def __init__(self, target, dim=6, scales=None, rng=None, target_accept=0.44):
        self.target = target
        self.dim = dim
        self.scales = np.full(dim, 0.01) if scales is None else np.asarray(scales, dtype=np.float64).copy()
        self.rng = np.random.default_rng(0) if rng is None else rng
        self.target_accept = target_accept
        self.accepts = np.zeros(dim)
        self.tries = np.zeros(dim)

    def sweep(self, z, logp: float, adapt_rate: float = 0.0):
        """One pass over the coordinates from (z, logp = log density at z); returns the new pair.
        With adapt_rate > 0 each coordinate's log scale moves by adapt_rate * (accepted - target)."""
        z = np.asarray(z, dtype=np.float64).copy()
        for i in range(self.dim):
            prop = z.copy()
            prop[i] += self.scales[i] * self.rng.normal()
            lp = self.target.logp(prop)
            acc = bool(np.isfinite(lp) and np.log(self.rng.uniform()) < lp - logp)
            if acc:
                z, logp = prop, lp
            self.tries[i] += 1
            self.accepts[i] += acc
            if adapt_rate > 0.0:
                self.scales[i] *= np.exp(adapt_rate * ((1.0 if acc else 0.0) - self.target_accept))
        return z, logp

    def acceptance(self) -> np.ndarray:
        return self.accepts / np.maximum(self.tries, 1)
