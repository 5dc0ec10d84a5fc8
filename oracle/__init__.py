"""FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Plain, slow reference implementations used to check the GPU library:

* ``loglik``            -- the Hawkes log-likelihood and gradient (C, OpenMP),
* ``rate_parts``        -- background / triggering parts of each lambda_n,
* ``philox4x64_10`` and ``resample`` -- the counter-based location draw,
* ``oracle.mlp``        -- the surrogate network in NumPy FP64.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with
``paper_2407_11349_amd``.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "hawkes_oracle.c"
_LIB = _HERE / "libhawkes_oracle.so"

_lib = None


def build(force: bool = False) -> Path:
    """Compile the C oracle with gcc (no fast-math, no FP contraction)."""
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB.with_suffix(".so.tmp%d" % os.getpid())
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-Wextra", "-o", str(tmp), str(_SRC), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(str(_LIB))
        dp = ctypes.POINTER(ctypes.c_double)
        lib.hawkes_oracle_loglik.argtypes = [ctypes.c_int64, dp, dp, dp, dp, dp, ctypes.c_double, ctypes.c_int64,
                                             ctypes.c_int64, dp, dp, dp, dp, dp]
        lib.hawkes_oracle_loglik.restype = ctypes.c_int
        lib.hawkes_oracle_rate_parts.argtypes = [ctypes.c_int64, dp, dp, dp, dp, dp, ctypes.c_double,
                                                 ctypes.c_int64, ctypes.c_int64, dp, dp]
        lib.hawkes_oracle_rate_parts.restype = ctypes.c_int
        u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.hawkes_oracle_philox4x64_10.argtypes = [u64p, u64p, u64p]
        lib.hawkes_oracle_philox4x64_10.restype = None
        lib.hawkes_oracle_resample.argtypes = [ctypes.c_int64, ctypes.POINTER(ctypes.c_int32), dp,
                                               ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint64, dp, dp]
        lib.hawkes_oracle_resample.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def loglik(t, x, y, s, theta, rows=None, per_row=False, area=0.0):
    """Log-likelihood of rows [r0, r1) (default all), its 6-gradient, optional per-row terms.

    area = 0: Gaussian spatial background N2(.; tau_x^2); area > 0: the paper's spatially
    uniform background 1/area.  Returns (loglik, grad) or, with per_row=True,
    (loglik, grad, lam, Lam, ell).
    """
    lib = _load()
    t, x, y, s, th = _f64(t), _f64(x), _f64(y), _f64(s), _f64(theta)
    n = t.shape[0]
    r0, r1 = (0, n) if rows is None else rows
    ll = np.zeros(1)
    g = np.zeros(6)
    nr = max(r1 - r0, 0)
    lam = np.zeros(nr) if per_row else None
    comp = np.zeros(nr) if per_row else None
    ell = np.zeros(nr) if per_row else None
    rc = lib.hawkes_oracle_loglik(n, _dp(t), _dp(x), _dp(y), _dp(s), _dp(th), float(area), r0, r1, _dp(ll),
                                  _dp(g), _dp(lam), _dp(comp), _dp(ell))
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    if per_row:
        return float(ll[0]), g, lam, comp, ell
    return float(ll[0]), g


def rate_parts(t, x, y, s, theta, rows=None, area=0.0):
    """(bg, tr): background and triggering sums of lambda_n without mu and xi."""
    lib = _load()
    t, x, y, s, th = _f64(t), _f64(x), _f64(y), _f64(s), _f64(theta)
    n = t.shape[0]
    r0, r1 = (0, n) if rows is None else rows
    bg = np.zeros(r1 - r0)
    tr = np.zeros(r1 - r0)
    if lib.hawkes_oracle_rate_parts(n, _dp(t), _dp(x), _dp(y), _dp(s), _dp(th), float(area), r0, r1, _dp(bg),
                                    _dp(tr)):
        raise ValueError("oracle rejected its arguments")
    return bg, tr


def philox4x64_10(counter, key):
    lib = _load()
    c = (ctypes.c_uint64 * 4)(*[int(v) & (2**64 - 1) for v in counter])
    k = (ctypes.c_uint64 * 2)(*[int(v) & (2**64 - 1) for v in key])
    o = (ctypes.c_uint64 * 4)()
    lib.hawkes_oracle_philox4x64_10(c, k, o)
    return [int(v) for v in o]


def resample(county, rect, seed, iteration):
    """Uniform within-county location draw; returns new (x, y)."""
    lib = _load()
    county = np.ascontiguousarray(county, dtype=np.int32)
    rect = _f64(rect)
    n = county.shape[0]
    x = np.zeros(n)
    y = np.zeros(n)
    rc = lib.hawkes_oracle_resample(n, county.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(rect),
                                    rect.shape[0], int(seed), int(iteration), _dp(x), _dp(y))
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return x, y
