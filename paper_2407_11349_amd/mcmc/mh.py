"""The paper's own parameter kernel: random-walk Metropolis-Hastings with univariate
updates (Section 2.3.2, run inside the cut-posterior scheme of Section 2.2).

Each sweep updates the log-parameters z = log theta one coordinate at a time with a
Gaussian random-walk proposal; every proposal costs one exact log-density (the
forward-only sweep, no gradient).  The proposal scales adapt during warm-up
towards the acceptance rate 0.44 that suits one-dimensional random walks, and are
fixed afterwards.  Under the cut posterior each sweep starts after a new
latent-location draw, so the current point's density is recomputed; with a target
that offers `logp_batch` it is evaluated together with the first proposal.
"""

from __future__ import annotations

import numpy as np

from .hmc import accept_prob, check_state


class UnivariateMH:
    def __init__(self, target, dim=6, scales=None, rng=None, target_accept=0.44):
        self.target = target
        self.dim = dim
        self.scales = np.full(dim, 0.01) if scales is None else np.asarray(scales, dtype=np.float64).copy()
        self.rng = np.random.default_rng(0) if rng is None else rng
        self.target_accept = target_accept
        self.accepts = np.zeros(dim)
        self.tries = np.zeros(dim)

    def sweep(self, z, logp: float | None = None, adapt_rate: float = 0.0):
        """One pass over the coordinates from (z, logp = log density at z, or None to compute it);
        returns the new pair.  With adapt_rate > 0 each coordinate's log scale moves by
        adapt_rate * (accepted - target)."""
        z = np.asarray(z, dtype=np.float64).copy()
        batch = getattr(self.target, "logp_batch", None)
        for i in range(self.dim):
            prop = z.copy()
            prop[i] += self.scales[i] * self.rng.normal()
            if logp is None:
                if batch is not None:
                    logp, lp = (float(v) for v in batch([z, prop]))
                else:
                    logp, lp = self.target.logp(z), self.target.logp(prop)
            else:
                lp = self.target.logp(prop)
            check_state(z, logp)
            acc = bool(self.rng.uniform() < accept_prob(lp - logp))
            if acc:
                z, logp = prop, lp
            self.tries[i] += 1
            self.accepts[i] += acc
            if adapt_rate > 0.0:
                self.scales[i] *= np.exp(adapt_rate * ((1.0 if acc else 0.0) - self.target_accept))
        return z, logp

    def acceptance(self) -> np.ndarray:
        return self.accepts / np.maximum(self.tries, 1)
