"""Seeded initial weights of the surrogate network 6 -> 256 -> 256 -> 256 -> 1.

Flat layout: W1 (256x6, out x in), b1, W2 (256x256), b2, W3 (256x256), b3,
w4 (256), b4: 133,633 values.  Each block is uniform on +-1/sqrt(fan_in) of
its layer and representable in FP32.  Input generation only.
"""

import math

import numpy as np

N_PARAMS = 256 * 6 + 256 + 256 * 256 + 256 + 256 * 256 + 256 + 256 + 1
_BLOCKS = [(256 * 6, 6), (256, 6), (256 * 256, 256), (256, 256), (256 * 256, 256), (256, 256), (256, 256), (1, 256)]


def init_params(seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    parts = []
    for n, fan_in in _BLOCKS:
        lim = 1.0 / math.sqrt(fan_in)
        parts.append(rng.uniform(-lim, lim, n))
    out = np.concatenate(parts).astype(np.float32)
    assert out.shape[0] == N_PARAMS
    return out
