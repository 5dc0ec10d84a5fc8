"""BF16 surrogate of the log-likelihood, trained and evaluated by the HIP
kernels of libhawkes (include/hawkes_mlp.h).

The network sees standardised inputs z = (log theta - m_z) / s_z and predicts
a standardised log-likelihood y = (l - m_y) / s_y; its input gradient is the
standardised gradient g = s_z * (theta . dl/dtheta) / s_y.  Standardisation is
needed because near the posterior mode the spread of log theta is ~1e-3,
far below BF16 resolution of raw inputs.  The data tuples (theta, l, grad)
come from the exact GPU likelihood.
"""

from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib

P = _lib.MLP_PARAMS


def _aligned_buffer(nbytes: int, device) -> tuple[torch.Tensor, int]:
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    base = buf.data_ptr()
    return buf, base + ((-base) % 256)


class SurrogateNet:
    """Network state on the GPU: FP32 master weights, Adam moments, BF16 copies."""

    def __init__(self, params, device="cuda"):
        lib = _lib.load()
        self.device = torch.device(device)
        self._state_buf, self.state = _aligned_buffer(int(lib.hawkes_mlp_state_bytes()), self.device)
        self._ws = None
        self._ws_batch = 0
        self.load(params)

    def load(self, params) -> None:
        p = torch.as_tensor(np.asarray(params, dtype=np.float32)).to(self.device).contiguous()
        if p.numel() != P:
            raise ValueError(f"expected {P} parameters")
        lib = _lib.load()
        _lib.check(lib.hawkes_mlp_load(self.state, p.data_ptr(), _lib.stream_handle()), "hawkes_mlp_load")
        torch.cuda.current_stream().synchronize()

    def params(self) -> torch.Tensor:
        out = torch.empty(P, dtype=torch.float32, device=self.device)
        _lib.check(_lib.load().hawkes_mlp_store(self.state, out.data_ptr(), _lib.stream_handle()), "hawkes_mlp_store")
        return out

    def forward(self, z: torch.Tensor, want_grad: bool = True):
        z = z.to(self.device, torch.float32).contiguous()
        B = z.shape[0]
        f = torch.empty(B, dtype=torch.float32, device=self.device)
        gz = torch.empty(B, 6, dtype=torch.float32, device=self.device) if want_grad else None
        _lib.check(_lib.load().hawkes_mlp_forward(self.state, z.data_ptr(), B, f.data_ptr(),
                                                  gz.data_ptr() if gz is not None else None, _lib.stream_handle()),
                   "hawkes_mlp_forward")
        return f, gz

    def leapfrog(self, z, p, grad, eps: float, inv_mass, n_steps: int, std: "Standardiser", prior_var: float):
        """A whole leapfrog trajectory on the surrogate log posterior
        s(z) = s_y f((z - m_z)/s_z) + m_y - z.z/(2 prior_var) in one kernel (hawkes_mlp_leapfrog);
        returns (z, p, s, grad) at the end point as host arrays (s = -inf if a step was not finite)."""
        L = _lib.LEAPFROG_IO_DOUBLES
        if getattr(self, "_lf_host", None) is None:
            self._lf_host = torch.empty(L, dtype=torch.float64).pin_memory()
            self._lf_dev = torch.empty(L, dtype=torch.float64, device=self.device)
        h = self._lf_host.numpy()
        h[0:6], h[6:12], h[12:18], h[18:24] = z, p, grad, inv_mass
        h[24:30], h[30:36] = std.m_z, std.s_z
        h[36], h[37], h[38], h[39], h[40], h[41] = std.m_y, std.s_y, prior_var, eps, 0.0, 0.0
        self._lf_dev.copy_(self._lf_host, non_blocking=True)
        _lib.check(_lib.load().hawkes_mlp_leapfrog(self.state, self._lf_dev.data_ptr(), int(n_steps),
                                                   _lib.stream_handle()), "hawkes_mlp_leapfrog")
        out = self._lf_dev.cpu().numpy()
        return out[0:6].copy(), out[6:12].copy(), float(out[40]), out[12:18].copy()

    def _workspace(self, B: int) -> int:
        if self._ws is None or self._ws_batch < B:
            nbytes = int(_lib.load().hawkes_mlp_workspace_bytes(B))
            self._ws_tensor, self._ws = _aligned_buffer(nbytes, self.device)
            self._ws_bytes = nbytes
            self._ws_batch = B
        return self._ws

    def loss_grad(self, z, y, g, lam: float, grad: torch.Tensor | None = None):
        z = z.to(self.device, torch.float32).contiguous()
        y = y.to(self.device, torch.float32).contiguous()
        g = g.to(self.device, torch.float32).contiguous()
        B = z.shape[0]
        ws = self._workspace(B)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        grad = torch.empty(P, dtype=torch.float32, device=self.device) if grad is None else grad
        _lib.check(_lib.load().hawkes_mlp_loss_grad(self.state, z.data_ptr(), y.data_ptr(), g.data_ptr(), B,
                                                    ctypes.c_float(lam), ws, self._ws_bytes, loss.data_ptr(),
                                                    grad.data_ptr(), _lib.stream_handle()), "hawkes_mlp_loss_grad")
        return loss, grad

    def adam_step(self, grad: torch.Tensor, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8) -> None:
        _lib.check(_lib.load().hawkes_mlp_adam_step(self.state, grad.data_ptr(), int(step), ctypes.c_float(lr),
                                                    ctypes.c_float(beta1), ctypes.c_float(beta2),
                                                    ctypes.c_float(eps), _lib.stream_handle()),
                   "hawkes_mlp_adam_step")


def group_means(v: np.ndarray, groups: np.ndarray) -> np.ndarray:
    """Mean of v over each group id 0..max(groups)."""
    n = int(groups.max()) + 1
    return np.bincount(groups, weights=v, minlength=n) / np.maximum(np.bincount(groups, minlength=n), 1)


@dataclass
class Standardiser:
    """Affine maps between log theta / l / gradient and the network's units."""

    m_z: np.ndarray
    s_z: np.ndarray
    m_y: float
    s_y: float

    @classmethod
    def fit(cls, logtheta: np.ndarray, ll: np.ndarray, groups: np.ndarray | None = None) -> "Standardiser":
        """With ``groups`` (tuples that share one latent-location draw), the value scale is the
        spread of l within the groups: the offset a draw adds to l is not part of the fit."""
        s_z = np.maximum(logtheta.std(axis=0), 1e-12)
        spread = ll if groups is None else ll - group_means(ll, groups)[groups]
        return cls(logtheta.mean(axis=0), s_z, float(ll.mean()), float(max(spread.std(), 1e-12)))

    def z(self, logtheta):
        return (np.asarray(logtheta) - self.m_z) / self.s_z

    def y(self, ll):
        return (np.asarray(ll) - self.m_y) / self.s_y

    def g(self, grad_logtheta):
        return np.asarray(grad_logtheta) * self.s_z / self.s_y

    def ll_from_y(self, y):
        return np.asarray(y, dtype=np.float64) * self.s_y + self.m_y

    def grad_from_g(self, g):
        return np.asarray(g, dtype=np.float64) * self.s_y / self.s_z


class Surrogate:
    """l(log theta) ~ s_y f((log theta - m_z)/s_z) + m_y with its gradient."""

    def __init__(self, net: SurrogateNet, std: Standardiser):
        self.net = net
        self.std = std

    def leapfrog(self, z, p, grad, eps, inv_mass, n_steps, prior_var):
        """Leapfrog trajectory on the surrogate posterior (value + N(0, prior_var) priors), on the GPU."""
        return self.net.leapfrog(z, p, grad, eps, inv_mass, n_steps, self.std, prior_var)

    def value_and_grad(self, logtheta: np.ndarray):
        z = torch.tensor(self.std.z(np.atleast_2d(logtheta)), dtype=torch.float32)
        f, gz = self.net.forward(z)
        f = f.cpu().numpy().astype(np.float64)
        gz = gz.cpu().numpy().astype(np.float64)
        return self.std.ll_from_y(f), self.std.grad_from_g(gz)


def train(net: SurrogateNet, std: Standardiser, logtheta, ll, grad_logtheta, *, lam=1.0, epochs=40, batch=256,
          lr=1e-3, seed=0, lr_decay=0.98, log=None, groups: np.ndarray | None = None):
    """Adam on the Sobolev loss over the tuples; returns the per-epoch mean loss.

    With ``groups`` (one id per tuple: the latent-location draw it was computed under, ids
    0..G-1), the value term fits l only up to one offset per group: each epoch the targets are
    l - mean_group(l) + mean_group(f) with f the current network, so that the value residual of
    a tuple is its residual minus its group's mean residual.  The gradient term is unchanged."""
    Z = torch.tensor(std.z(logtheta), dtype=torch.float32, device=net.device)
    Y = torch.tensor(std.y(ll), dtype=torch.float32, device=net.device)
    G = torch.tensor(std.g(grad_logtheta), dtype=torch.float32, device=net.device)
    n = Z.shape[0]
    if groups is not None:
        groups = np.asarray(groups, dtype=np.int64)
        yc = std.y(ll)
        yc = yc - group_means(yc, groups)[groups]
    rng = np.random.default_rng(seed)
    grad = torch.empty(P, dtype=torch.float32, device=net.device)
    step = 0
    history = []
    for ep in range(epochs):
        if groups is not None:
            f = np.concatenate([net.forward(Z[i:i + 4096], want_grad=False)[0].cpu().numpy()
                                for i in range(0, n, 4096)]).astype(np.float64)
            Y = torch.tensor(yc + group_means(f, groups)[groups], dtype=torch.float32, device=net.device)
        perm = torch.from_numpy(rng.permutation(n)).to(net.device)
        tot = torch.zeros(1, dtype=torch.float32, device=net.device)
        nb = 0
        for s in range(0, n - batch + 1, batch):
            idx = perm[s:s + batch]
            loss, _ = net.loss_grad(Z[idx], Y[idx], G[idx], lam, grad=grad)
            step += 1
            net.adam_step(grad, step, lr * (lr_decay ** ep))
            tot += loss
            nb += 1
        history.append(float(tot.item()) / max(nb, 1))
        if log:
            log(f"epoch {ep}: loss {history[-1]:.4e}")
    return history
