"""Pins of the FP64 surrogate-network reference (oracle/mlp.py): finite differences,
PyTorch's CPU double-backward (a library pin of the Sobolev-loss gradient), the
Adam update against closed forms over several steps (a constant gradient and an
alternating one), and the BF16 rounding rule."""

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


def _adam_run(grads, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    th = np.zeros_like(grads[0])
    m, v = np.zeros_like(th), np.zeros_like(th)
    steps = []
    for k, gr in enumerate(grads, start=1):
        new, m, v = mlp.adam_step(th, m, v, gr, k, lr, beta1=beta1, beta2=beta2, eps=eps)
        steps.append(new - th)
        th = new
    return steps, m, v


def test_adam_constant_gradient_closed_form():
    """With g_t = g for every t: m_t = g (1 - beta1^t), v_t = g^2 (1 - beta2^t), so after bias correction
    every step moves each coordinate by -lr g / (|g| + eps) (Kingma and Ba, 2015, Algorithm 1)."""
    rng = np.random.default_rng(2)
    g = rng.normal(size=40) * np.logspace(-3, 2, 40)
    b1, b2, lr = 0.8, 0.95, 1e-3  # far from the defaults, so the two decay rates cannot stand in for each other
    steps, m, v = _adam_run([g] * 6, lr, b1, b2)
    np.testing.assert_allclose(m, g * (1.0 - b1 ** 6), rtol=1e-13)
    np.testing.assert_allclose(v, g * g * (1.0 - b2 ** 6), rtol=1e-13)
    for st in steps:
        np.testing.assert_allclose(st, -lr * g / (np.abs(g) + 1e-8), rtol=1e-11)


def test_adam_alternating_gradient_closed_form():
    """With g_t = (-1)^(t+1) g: m_t = (1 - beta1) g (-1)^(t+1) (1 - (-beta1)^t) / (1 + beta1) (a geometric
    series) and v_t = g^2 (1 - beta2^t), so step t moves by -lr m_t / (1 - beta1^t) / (|g| + eps)."""
    rng = np.random.default_rng(3)
    g = rng.normal(size=30)
    b1, b2, lr = 0.7, 0.9, 2e-3
    T = 5
    steps, m, v = _adam_run([g * (-1.0) ** t for t in range(T)], lr, b1, b2)
    for t in range(1, T + 1):
        mt = (1.0 - b1) * g * (-1.0) ** (t + 1) * (1.0 - (-b1) ** t) / (1.0 + b1)
        np.testing.assert_allclose(steps[t - 1], -lr * (mt / (1.0 - b1 ** t)) / (np.abs(g) + 1e-8), rtol=1e-11)
    np.testing.assert_allclose(v, g * g * (1.0 - b2 ** T), rtol=1e-13)
    np.testing.assert_allclose(m, (1.0 - b1) * g * (-1.0) ** (T + 1) * (1.0 - (-b1) ** T) / (1.0 + b1), rtol=1e-13)


def test_adam_second_moment_tracks_squares():
    """Gradients of growing size: v_t = (1 - beta2) sum_k beta2^(t-k) g_k^2 written out, against the update."""
    g1, g2, g3 = np.array([0.5, -2.0]), np.array([1.5, 1.0]), np.array([-3.0, 0.25])
    b1, b2, lr = 0.6, 0.85, 1e-2
    steps, m, v = _adam_run([g1, g2, g3], lr, b1, b2)
    m3 = (1 - b1) * (b1 * b1 * g1 + b1 * g2 + g3)
    v3 = (1 - b2) * (b2 * b2 * g1 ** 2 + b2 * g2 ** 2 + g3 ** 2)
    np.testing.assert_allclose(m, m3, rtol=1e-14)
    np.testing.assert_allclose(v, v3, rtol=1e-14)
    np.testing.assert_allclose(steps[2], -lr * (m3 / (1 - b1 ** 3)) / (np.sqrt(v3 / (1 - b2 ** 3)) + 1e-8),
                               rtol=1e-12)


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


def test_gelu_and_its_derivatives():
    """GELU(x) = x Phi(x) against scipy's normal cdf, and its first and second derivatives against
    Richardson-extrapolated central differences of the function itself (a mistake in a derivative
    formula, such as a dropped x phi(x) term, fails here before it reaches the Sobolev gradient)."""
    from scipy.stats import norm

    x = np.linspace(-7.0, 7.0, 281)
    np.testing.assert_allclose(mlp.gelu(x), x * norm.cdf(x), rtol=1e-14, atol=1e-15)  # 1 + erf cancels far left

    def rich(f, h):
        d = lambda s: (f(x + s) - f(x - s)) / (2 * s)  # noqa: E731
        return (4 * d(h / 2) - d(h)) / 3

    np.testing.assert_allclose(mlp.gelu_d1(x), rich(mlp.gelu, 1e-3), rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(mlp.gelu_d2(x), rich(mlp.gelu_d1, 1e-3), rtol=1e-8, atol=1e-10)
