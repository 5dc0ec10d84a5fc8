"""Pins of the FP64 surrogate-network reference (oracle/mlp.py): finite differences,
PyTorch's CPU double-backward (a library pin of the Sobolev-loss gradient), the
Adam update against its closed form on a single step, and the BF16 rounding rule."""

import numpy as np
import pytest
import torch

from oracle import mlp
from synth.mlp_init import init_params


def _data(B, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(B, 6)), rng.normal(size=B), rng.normal(size=(B, 6))


def test_input_gradient_finite_differences():
    th = init_params(3).astype(np.float64)
    z, _, _ = _data(7, 1)
    f, gz = mlp.forward(th, z)
    for i in range(6):
        e = np.zeros(6)
        e[i] = 1e-5
        fd = (mlp.forward(th, z + e)[0] - mlp.forward(th, z - e)[0]) / 2e-5
        np.testing.assert_allclose(gz[:, i], fd, rtol=1e-7, atol=1e-9)


def test_sobolev_parameter_gradient_finite_differences():
    th = init_params(4).astype(np.float64) * 3.0  # larger weights exercise the curvature terms
    z, y, g = _data(5, 2)
    lam = 0.7
    _, grad = mlp.sobolev_loss_and_grad(th, z, y, g, lam)
    rng = np.random.default_rng(0)
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 40, replace=False), [0, 1536, mlp.N_PARAMS - 1,
                                                                        mlp.N_PARAMS - 100]])
    for k in idx:
        e = np.zeros(mlp.N_PARAMS)
        e[k] = 1e-6
        lp = mlp.sobolev_loss_and_grad(th + e, z, y, g, lam)[0]
        lm = mlp.sobolev_loss_and_grad(th - e, z, y, g, lam)[0]
        fd = (lp - lm) / 2e-6
        assert grad[k] == pytest.approx(fd, rel=1e-5, abs=1e-8), k


def test_sobolev_gradient_matches_torch_double_backward():
    """Library pin: PyTorch autograd (CPU, float64, create_graph) on the same network."""
    th = init_params(5).astype(np.float64)
    z, y, g = _data(9, 3)
    lam = 0.25
    loss, grad = mlp.sobolev_loss_and_grad(th, z, y, g, lam)
    P = torch.tensor(th, dtype=torch.float64, requires_grad=True)
    blocks = {}
    for name, shp, off in mlp.layout():
        blocks[name] = P[off:off + int(np.prod(shp))].reshape(shp)
    Z = torch.tensor(z, dtype=torch.float64, requires_grad=True)
    act = torch.nn.functional.gelu
    h = act(Z @ blocks["W1"].T + blocks["b1"])
    h = act(h @ blocks["W2"].T + blocks["b2"])
    h = act(h @ blocks["W3"].T + blocks["b3"])
    f = h @ blocks["w4"] + blocks["b4"][0]
    (gz,) = torch.autograd.grad(f.sum(), Z, create_graph=True)
    L = ((f - torch.tensor(y)) ** 2 + lam * ((gz - torch.tensor(g)) ** 2).sum(dim=1)).mean()
    L.backward()
    assert float(L.detach()) == pytest.approx(loss, rel=1e-12)
    np.testing.assert_allclose(P.grad.numpy(), grad, rtol=1e-9, atol=1e-12)


def test_adam_first_step_is_sign_times_lr():
    """With bias correction, the first Adam step moves each coordinate by lr * g/(|g| + eps')."""
    rng = np.random.default_rng(1)
    th = rng.normal(size=50)
    gr = rng.normal(size=50)
    new, m, v = mlp.adam_step(th, np.zeros(50), np.zeros(50), gr, 1, 1e-3)
    np.testing.assert_allclose(new - th, -1e-3 * gr / (np.abs(gr) + 1e-8), rtol=1e-12)


def test_bf16_rounding_rule():
    vals = np.array([1.0, 1.0 + 2**-8, 1.0 + 3 * 2**-9, 1.0 + 2**-9, 1.0 + 3 * 2**-8, -3.14159, 65504.0, 1e-30],
                    dtype=np.float32)
    r = mlp.to_bf16(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0  # tie between 1 and 1 + 2^-7 (BF16 spacing at 1): goes to the even mantissa
    assert r[2] == 1.0 + 2**-7
    assert r[3] == 1.0
    assert r[4] == 1.0 + 2**-6  # tie between 1 + 2^-7 (odd) and 1 + 2^-6 (even)
    ref = torch.tensor(vals).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(r, ref)
