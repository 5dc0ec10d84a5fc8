"""The paper's cut-posterior scheme (Section 2.2) on the GPU likelihood.

Each iteration first redraws every latent location uniformly inside its
county (p(X | coarsened data), O(N), GPU), then applies a parameter kernel
that leaves p(theta | X, t) invariant.  Parameters are sampled as
z = log theta with independent N(0, prior_sd^2) priors on each z_i.
"""

from __future__ import annotations

import numpy as np
import torch

from .. import likelihood as lk


class HawkesCutTarget:
    """log p(z | X, t) = l(exp z; X) + sum_i log N(z_i; 0, prior_sd^2) (up to a constant)."""

    def __init__(self, events: lk.DeviceEvents, county: torch.Tensor | None = None, rect: torch.Tensor | None = None,
                 seed: int = 0, precision: str = "fp32", prior_sd: float = 10.0, workspace_bytes: int | None = None):
        """workspace_bytes: the likelihood workspace (default: hawkes_workspace_bytes); a larger one lets the
        pair sweep run in fewer passes, with the same results."""
        self.ev = events
        self.county = county
        self.rect = rect
        self.seed = seed
        self.precision = precision
        self.prior_var = prior_sd ** 2
        self.ws = lk.Workspace(events.n, precision, events.t.device, nbytes=workspace_bytes)
        self.out = torch.empty(1, dtype=torch.float64, device=events.t.device)
        self.grad = torch.empty(6, dtype=torch.float64, device=events.t.device)
        self.out_batch = None
        self.n_loglik = 0
        self.n_grad = 0

    def resample(self, iteration: int) -> None:
        if self.county is None:
            return
        lk.resample_locations(self.county, self.rect, self.seed, iteration, self.ev.x, self.ev.y)

    def _prior(self, z):
        return -0.5 * float(np.dot(z, z)) / self.prior_var, -z / self.prior_var

    def logp(self, z) -> float:
        z = np.asarray(z, dtype=np.float64)
        if not np.all(np.isfinite(z)) or np.any(np.abs(z) > 50):
            return -np.inf
        lk.loglik(self.ev, np.exp(z), precision=self.precision, ws=self.ws, out=self.out)
        self.n_loglik += 1
        lp, _ = self._prior(z)
        return float(self.out.item()) + lp

    def logp_batch(self, zs) -> np.ndarray:
        """log p(z_k | X, t) for several points under the current draw, the likelihoods from one
        batched call (two parameter vectors per FP32 pair sweep)."""
        zs = [np.asarray(z, dtype=np.float64) for z in zs]
        out = np.full(len(zs), -np.inf)
        ok = [k for k, z in enumerate(zs) if np.all(np.isfinite(z)) and not np.any(np.abs(z) > 50)]
        if not ok:
            return out
        if self.out_batch is None or self.out_batch.numel() < len(ok):
            self.out_batch = torch.empty(len(ok), dtype=torch.float64, device=self.ev.t.device)
        th = np.exp(np.stack([zs[k] for k in ok]))
        lk.loglik_batch(self.ev, th, precision=self.precision, ws=self.ws, out=self.out_batch)
        vals = self.out_batch[:len(ok)].cpu().numpy()
        self.n_loglik += len(ok)
        for j, k in enumerate(ok):
            out[k] = float(vals[j]) + self._prior(zs[k])[0]
        return out

    def logp_and_grad(self, z):
        z = np.asarray(z, dtype=np.float64)
        if not np.all(np.isfinite(z)) or np.any(np.abs(z) > 50):
            return -np.inf, np.zeros_like(z)
        th = np.exp(z)
        lk.loglik_grad(self.ev, th, precision=self.precision, ws=self.ws, out=self.out, grad=self.grad)
        self.n_grad += 1
        g = self.grad.cpu().numpy()
        lp, gp = self._prior(z)
        return float(self.out.item()) + lp, th * g + gp

    def loglik_and_grad_logtheta(self, z):
        """(l, d l / d log theta) without the prior: the tuples the surrogate learns."""
        th = np.exp(np.asarray(z, dtype=np.float64))
        lk.loglik_grad(self.ev, th, precision=self.precision, ws=self.ws, out=self.out, grad=self.grad)
        self.n_grad += 1
        return float(self.out.item()), th * self.grad.cpu().numpy()
