"""FP64 reference of the surrogate network -- TEST INFRASTRUCTURE ONLY.

The surrogate of the log-likelihood is a fully connected network
6 -> 256 -> 256 -> 256 -> 1 with GELU activations (GELU(x) = x Phi(x)),
trained with a value + gradient ("Sobolev") loss

    L = (1/B) sum_b [ (f(z_b) - y_b)^2 + lambda_g |grad_z f(z_b) - g_b|^2 ].

Parameters live in one flat vector in the order W1 (256x6, row-major:
out x in), b1, W2 (256x256), b2, W3 (256x256), b3, w4 (256), b4 (1):
133,633 values.  The GPU keeps FP32 master weights and computes with BF16
copies; the functions here take whatever weights they are given (the tests
pass the BF16-rounded ones) and compute in FP64.

The parameter gradient is the chain rule of the loss written out: reverse
mode through the primal pass and through the reverse pass that forms
grad_z f (reverse over reverse).
"""

from __future__ import annotations

import math

import numpy as np

DIMS = (6, 256, 256, 256, 1)
N_PARAMS = 256 * 6 + 256 + 256 * 256 + 256 + 256 * 256 + 256 + 256 + 1


def layout():
    """(name, shape, offset) of each parameter block in the flat vector."""
    shapes = [("W1", (256, 6)), ("b1", (256,)), ("W2", (256, 256)), ("b2", (256,)),
              ("W3", (256, 256)), ("b3", (256,)), ("w4", (256,)), ("b4", (1,))]
    out, off = [], 0
    for name, shp in shapes:
        out.append((name, shp, off))
        off += int(np.prod(shp))
    assert off == N_PARAMS
    return out


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    return {name: theta[off:off + int(np.prod(shp))].reshape(shp) for name, shp, off in layout()}


def to_bf16(a) -> np.ndarray:
    """Round FP32 values to bfloat16 (round to nearest, ties to even); returned as FP64."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


_SQ2 = math.sqrt(2.0)
_ISQ2PI = 1.0 / math.sqrt(2.0 * math.pi)


def _erf(x):
    from scipy.special import erf
    return erf(x)


def gelu(x):
    return 0.5 * x * (1.0 + _erf(x / _SQ2))


def gelu_d1(x):
    """d/dx x Phi(x) = Phi(x) + x phi(x)."""
    return 0.5 * (1.0 + _erf(x / _SQ2)) + x * _ISQ2PI * np.exp(-0.5 * x * x)


def gelu_d2(x):
    """d2/dx2 x Phi(x) = phi(x) (2 - x^2)."""
    return _ISQ2PI * np.exp(-0.5 * x * x) * (2.0 - x * x)


def forward(theta, z):
    """f (B,) and grad_z f (B, 6) for inputs z (B, 6)."""
    p = unpack(theta)
    z = np.atleast_2d(np.asarray(z, dtype=np.float64))
    h1 = z @ p["W1"].T + p["b1"]
    a1 = gelu(h1)
    h2 = a1 @ p["W2"].T + p["b2"]
    a2 = gelu(h2)
    h3 = a2 @ p["W3"].T + p["b3"]
    a3 = gelu(h3)
    f = a3 @ p["w4"] + p["b4"][0]
    d3 = p["w4"] * gelu_d1(h3)
    d2 = (d3 @ p["W3"]) * gelu_d1(h2)
    d1 = (d2 @ p["W2"]) * gelu_d1(h1)
    gz = d1 @ p["W1"]
    return f, gz


def sobolev_loss_and_grad(theta, z, y, g, lam):
    """Loss (scalar) and its gradient with respect to the flat parameter vector.

    The loss reads the network twice: its value f and its input gradient
    grad_z f, which is itself a computation (the reverse pass below).  The
    parameter gradient is the chain rule applied to that whole graph: first
    the adjoints of the reverse pass (from the gradient-matching term), then
    the adjoints of the primal pass, which receive contributions both from f
    and from the activation slopes s_k = GELU'(h_k) that the reverse pass read
    (their derivative brings in GELU'')."""
    p = unpack(theta)
    z = np.atleast_2d(np.asarray(z, dtype=np.float64))
    y = np.asarray(y, dtype=np.float64)
    g = np.atleast_2d(np.asarray(g, dtype=np.float64))
    B = z.shape[0]
    W1, W2, W3, w4 = p["W1"], p["W2"], p["W3"], p["w4"]
    # primal pass
    h1 = z @ W1.T + p["b1"]
    a1, s1 = gelu(h1), gelu_d1(h1)
    h2 = a1 @ W2.T + p["b2"]
    a2, s2 = gelu(h2), gelu_d1(h2)
    h3 = a2 @ W3.T + p["b3"]
    a3, s3 = gelu(h3), gelu_d1(h3)
    f = a3 @ w4 + p["b4"][0]
    # reverse pass for grad_z f, with its intermediate values named
    d3 = w4 * s3            # df/dh3
    c2 = d3 @ W3            # df/da2
    d2 = c2 * s2            # df/dh2
    c1 = d2 @ W2            # df/da1
    d1 = c1 * s1            # df/dh1
    gz = d1 @ W1            # df/dz
    e = f - y
    r = gz - g
    loss = float(np.mean(e * e + lam * np.sum(r * r, axis=1)))

    # adjoints (x_bar = dL/dx), starting from the two outputs the loss reads
    f_bar = (2.0 / B) * e
    gz_bar = (2.0 * lam / B) * r
    grad = {}
    # through the reverse pass, last operation first
    grad["W1"] = d1.T @ gz_bar                  # gz = d1 W1
    d1_bar = gz_bar @ W1.T
    c1_bar = d1_bar * s1                        # d1 = c1 * s1
    s1_bar = d1_bar * c1
    grad["W2"] = d2.T @ c1_bar                  # c1 = d2 W2
    d2_bar = c1_bar @ W2.T
    c2_bar = d2_bar * s2                        # d2 = c2 * s2
    s2_bar = d2_bar * c2
    grad["W3"] = d3.T @ c2_bar                  # c2 = d3 W3
    d3_bar = c2_bar @ W3.T
    grad["w4"] = np.sum(d3_bar * s3, axis=0)    # d3 = w4 * s3
    s3_bar = d3_bar * w4
    # through the primal pass; each h_k feeds a_k = GELU(h_k) and s_k = GELU'(h_k)
    grad["w4"] = grad["w4"] + f_bar @ a3        # f = a3 . w4 + b4
    grad["b4"] = np.array([f_bar.sum()])
    a3_bar = np.outer(f_bar, w4)
    h3_bar = a3_bar * s3 + s3_bar * gelu_d2(h3)
    grad["W3"] = grad["W3"] + h3_bar.T @ a2     # h3 = a2 W3^T + b3
    grad["b3"] = h3_bar.sum(axis=0)
    a2_bar = h3_bar @ W3
    h2_bar = a2_bar * s2 + s2_bar * gelu_d2(h2)
    grad["W2"] = grad["W2"] + h2_bar.T @ a1     # h2 = a1 W2^T + b2
    grad["b2"] = h2_bar.sum(axis=0)
    a1_bar = h2_bar @ W2
    h1_bar = a1_bar * s1 + s1_bar * gelu_d2(h1)
    grad["W1"] = grad["W1"] + h1_bar.T @ z      # h1 = z W1^T + b1
    grad["b1"] = h1_bar.sum(axis=0)
    flat = np.zeros(N_PARAMS)
    for name, shp, off in layout():
        flat[off:off + int(np.prod(shp))] = np.asarray(grad[name]).reshape(-1)
    return loss, flat


def adam_step(theta, m, v, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015) with bias correction; step counts from 1."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
