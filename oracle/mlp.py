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

The parameter gradient of the gradient-matching term uses the identity
d/dtheta [r . grad_z f] = d/dtheta [D_r f] for a fixed vector r: the
directional derivative D_r f is a forward-mode tangent pass, and one reverse
pass through the primal and tangent computations gives both terms.
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
    """Loss (scalar) and its gradient with respect to the flat parameter vector."""
    p = unpack(theta)
    z = np.atleast_2d(np.asarray(z, dtype=np.float64))
    y = np.asarray(y, dtype=np.float64)
    g = np.atleast_2d(np.asarray(g, dtype=np.float64))
    B = z.shape[0]
    # primal pass
    h1 = z @ p["W1"].T + p["b1"]
    a1, s1 = gelu(h1), gelu_d1(h1)
    h2 = a1 @ p["W2"].T + p["b2"]
    a2, s2 = gelu(h2), gelu_d1(h2)
    h3 = a2 @ p["W3"].T + p["b3"]
    a3, s3 = gelu(h3), gelu_d1(h3)
    f = a3 @ p["w4"] + p["b4"][0]
    # input gradient (reverse mode)
    d3 = p["w4"] * s3
    d2 = (d3 @ p["W3"]) * s2
    d1 = (d2 @ p["W2"]) * s1
    gz = d1 @ p["W1"]
    e = f - y
    r = gz - g
    loss = float(np.mean(e * e + lam * np.sum(r * r, axis=1)))
    # tangent pass along r: the directional derivative D_r f
    t1 = r @ p["W1"].T
    u1 = s1 * t1
    t2 = u1 @ p["W2"].T
    u2 = s2 * t2
    t3 = u2 @ p["W3"].T
    u3 = s3 * t3
    # reverse pass of J = cf * f + ct * D_r f, with cf, ct, r held constant
    cf = (2.0 / B) * e
    ct = (2.0 * lam / B)
    grad = {}
    grad["w4"] = cf @ a3 + ct * u3.sum(axis=0)
    grad["b4"] = np.array([cf.sum()])
    a3b = np.outer(cf, p["w4"])               # adjoint of a3
    u3b = np.full_like(u3, ct) * p["w4"]      # adjoint of u3
    t3b = u3b * s3
    h3b = a3b * s3 + u3b * gelu_d2(h3) * t3
    grad["W3"] = h3b.T @ a2 + t3b.T @ u2
    grad["b3"] = h3b.sum(axis=0)
    a2b = h3b @ p["W3"]
    u2b = t3b @ p["W3"]
    t2b = u2b * s2
    h2b = a2b * s2 + u2b * gelu_d2(h2) * t2
    grad["W2"] = h2b.T @ a1 + t2b.T @ u1
    grad["b2"] = h2b.sum(axis=0)
    a1b = h2b @ p["W2"]
    u1b = t2b @ p["W2"]
    t1b = u1b * s1
    h1b = a1b * s1 + u1b * gelu_d2(h1) * t1
    grad["W1"] = h1b.T @ z + t1b.T @ r
    grad["b1"] = h1b.sum(axis=0)
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
