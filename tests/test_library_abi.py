"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, sizes workspaces, and rejects bad arguments on the host
before touching the GPU."""

import ctypes
import glob
import os
import re

import numpy as np
import pytest

from paper_2407_11349_amd import _lib

INCLUDE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")


def _declared():
    names = set()
    for h in sorted(glob.glob(os.path.join(INCLUDE, "*.h"))):
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names.update(re.findall(r"\b(hawkes_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 17
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_lib.EXPORTS)


def test_workspace_bytes(lib):
    assert lib.hawkes_workspace_bytes(0, 1) == 0
    assert lib.hawkes_workspace_bytes(10, 7) == 0
    assert lib.hawkes_workspace_bytes(-5, 0) == 0
    for prec in (0, 1):
        a = lib.hawkes_workspace_bytes(1, prec)
        b = lib.hawkes_workspace_bytes(100_000, prec)
        c = lib.hawkes_workspace_bytes(1_000_000, prec)
        assert 0 < a < b <= c
        assert a % 256 == 0 and c % 256 == 0
    # FP32 keeps extra staged source records
    assert lib.hawkes_workspace_bytes(5000, 1) > lib.hawkes_workspace_bytes(5000, 0)
    # O(n): a part linear in n plus a slot region of at most 704 MiB (under 10^9 bytes at 10^6 events)
    assert lib.hawkes_workspace_bytes(1_000_000, 1) < 10**9
    big = lib.hawkes_workspace_bytes(4_000_000, 1) - lib.hawkes_workspace_bytes(2_000_000, 1)
    assert big < 2_000_000 * 260
    for prec in (0, 1, 2):
        for n in (1, 700, 20_000, 1_000_000):
            lo, hi = lib.hawkes_workspace_min_bytes(n, prec), lib.hawkes_workspace_bytes(n, prec)
            assert 0 < lo <= hi and lo % 256 == 0
    assert lib.hawkes_workspace_min_bytes(0, 1) == 0


def test_strerror_and_codes(lib):
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert lib.hawkes_strerror(code)
    assert lib.hawkes_strerror(-99) == b"unknown status"


def _ev(n, p=0x100000, area=0.0):
    return _lib.Events(n, p, p, p, p, area)


def test_host_validation_paths(lib):
    th = _lib.Theta(0.5, 10.0, 7.0, 0.3, 2.0, 0.2)
    ev = _ev(1000)
    ws_need = lib.hawkes_workspace_bytes(1000, 1)
    fake = 0x200000  # never dereferenced: every call below fails host validation
    assert lib.hawkes_loglik(None, ctypes.byref(th), 1, 0, 10, fake, ws_need, fake, None, None) == -1
    assert lib.hawkes_loglik(ctypes.byref(_ev(0)), ctypes.byref(th), 1, 0, 0, fake, ws_need, fake, None,
                             None) == -1
    assert lib.hawkes_loglik(ctypes.byref(_ev(1000, 0)), ctypes.byref(th), 1, 0, 1, fake, ws_need, fake, None,
                             None) == -1
    assert lib.hawkes_loglik(ctypes.byref(ev), ctypes.byref(th), 3, 0, 10, fake, ws_need, fake, None, None) == -1
    for bad_area in (-1.0, float("nan"), float("inf")):
        eva = _ev(1000, area=bad_area)
        assert lib.hawkes_loglik(ctypes.byref(eva), ctypes.byref(th), 1, 0, 10, fake, ws_need, fake, None, None) == -1
        assert b"area" in lib.hawkes_last_error()
    for k in range(6):
        for bad in (0.0, -1.0, float("nan"), float("inf")):
            vals = [0.5, 10.0, 7.0, 0.3, 2.0, 0.2]
            vals[k] = bad
            tb = _lib.Theta(*vals)
            assert lib.hawkes_loglik(ctypes.byref(ev), ctypes.byref(tb), 1, 0, 10, fake, ws_need, fake, None, None) == -1
    assert b"theta" in lib.hawkes_last_error()
    for r0, r1 in ((-1, 5), (0, 1001), (7, 6)):
        assert lib.hawkes_loglik_grad(ctypes.byref(ev), ctypes.byref(th), 1, r0, r1, fake, ws_need, fake, fake,
                                      None, None) == -2
    ws_min = lib.hawkes_workspace_min_bytes(1000, 1)
    assert lib.hawkes_loglik(ctypes.byref(ev), ctypes.byref(th), 1, 0, 10, fake, ws_min - 256, fake, None, None) == -3
    assert lib.hawkes_loglik(ctypes.byref(ev), ctypes.byref(th), 1, 0, 10, fake + 8, ws_need, fake, None, None) == -3
    assert lib.hawkes_loglik(ctypes.byref(ev), ctypes.byref(th), 1, 0, 10, None, ws_need, fake, None, None) == -3
    assert lib.hawkes_loglik(ctypes.byref(ev), ctypes.byref(th), 1, 0, 10, fake, ws_need, None, None, None) == -1
    assert lib.hawkes_loglik_grad(ctypes.byref(ev), ctypes.byref(th), 1, 0, 10, fake, ws_need, fake, None,
                                  None, None) == -1
    assert lib.hawkes_resample_locations(10, None, fake, 3, 1, 2, fake, fake, None) == -1
    assert lib.hawkes_resample_locations(10, fake, fake, 0, 1, 2, fake, fake, None) == -1
    assert lib.hawkes_resample_locations(0, None, None, 3, 1, 2, None, None, None) == 0
    # per-call options out of range are refused before any work is enqueued
    for kw in ({"row_workgroups": -1}, {"row_workgroups": _lib.ROW_WGS_MAX + 1},
               {"symmetric_groups": -2}, {"symmetric_groups": _lib.SYM_GROUPS_MAX + 1}, {"reserved": 1},
               {"timing_start": fake}):
        o = _lib.Options(**kw)
        assert lib.hawkes_loglik(ctypes.byref(ev), ctypes.byref(th), 1, 0, 10, fake, ws_need, fake,
                                 ctypes.byref(o), None) == -1
    # the largest accepted values pass the option checks (and then fail on the workspace)
    o = _lib.Options(row_workgroups=_lib.ROW_WGS_MAX, symmetric_groups=_lib.SYM_GROUPS_MAX)
    assert lib.hawkes_loglik(ctypes.byref(ev), ctypes.byref(th), 1, 0, 10, fake, 256, fake, ctypes.byref(o),
                             None) == -3


def test_batch_host_validation(lib):
    ev = _ev(1000)
    ws_need = lib.hawkes_workspace_bytes(1000, 1)
    fake = 0x200000  # never dereferenced: every call below fails host validation
    good = (0.5, 10.0, 7.0, 0.3, 2.0, 0.2)
    arr = (_lib.Theta * 3)(_lib.Theta(*good), _lib.Theta(*good), _lib.Theta(*good))
    call = lib.hawkes_loglik_batch
    assert call(ctypes.byref(ev), arr, 0, 1, 0, 10, fake, ws_need, fake, None, None) == -1
    assert call(ctypes.byref(ev), None, 2, 1, 0, 10, fake, ws_need, fake, None, None) == -1
    assert call(ctypes.byref(ev), arr, 2, 1, 0, 10, fake, ws_need, None, None, None) == -1
    assert call(ctypes.byref(ev), arr, 2, 7, 0, 10, fake, ws_need, fake, None, None) == -1
    assert call(ctypes.byref(ev), arr, 2, 1, 0, 1001, fake, ws_need, fake, None, None) == -2
    ws_min = lib.hawkes_workspace_min_bytes(1000, 1)
    assert call(ctypes.byref(ev), arr, 2, 1, 0, 10, fake, ws_min - 256, fake, None, None) == -3
    # a bad component in any vector is caught before work is enqueued
    for k in range(3):
        vals = list(good)
        vals[5] = float("nan")
        bad = (_lib.Theta * 3)(*[_lib.Theta(*(vals if j == k else good)) for j in range(3)])
        assert call(ctypes.byref(ev), bad, 3, 1, 0, 10, fake, ws_need, fake, None, None) == -1
        assert b"theta" in lib.hawkes_last_error()
    # theta_array marshals (K, 6) inputs and rejects bad shapes
    a = _lib.theta_array([good, good])
    assert len(a) == 2 and a[1].omega == 0.2
    with pytest.raises(ValueError):
        _lib.theta_array([])
    with pytest.raises(ValueError):
        _lib.theta_array([good[:5]])


def test_mlp_leapfrog_host_validation(lib):
    fake = 0x200000  # never dereferenced: every call below fails host validation
    assert lib.hawkes_mlp_leapfrog(None, fake, 20, None) == -1
    assert lib.hawkes_mlp_leapfrog(fake, None, 20, None) == -1
    assert lib.hawkes_mlp_leapfrog(fake + 8, fake, 20, None) == -1
    assert lib.hawkes_mlp_leapfrog(fake, fake, 0, None) == -1
    assert lib.hawkes_mlp_leapfrog(fake, fake, 4097, None) == -1
    assert _lib.LEAPFROG_IO_DOUBLES * 8 == 336


def _declared_arity():
    """Parameter count of every function the headers declare (a `(void)` list counts as none)."""
    arity = {}
    for h in sorted(glob.glob(os.path.join(INCLUDE, "*.h"))):
        src = re.sub(r"/\*.*?\*/|//[^\n]*", "", open(h).read(), flags=re.S)
        for name, params in re.findall(r"\b(hawkes_[a-z0-9_]+)\s*\(([^;{)]*)\)\s*;", src):
            params = " ".join(params.split())
            arity[name] = 0 if params in ("", "void") else params.count(",") + 1
    return arity


def test_binding_argument_counts_match_the_headers(lib):
    arity = _declared_arity()
    assert set(arity) == set(_declared())
    for name, n in arity.items():
        assert len(getattr(lib, name).argtypes) == n, name


def test_a_workspace_sized_for_n_events_serves_every_smaller_set(lib):
    """The minimum is non-decreasing in n and never above the default, and the default's slot region is
    at most 704 MiB over the minimum's linear part, over sizes from 1 to 2 * 10^7 events."""
    ns = sorted(set(int(v) for v in np.logspace(0, 7.3, 1500)) | {511, 512, 513, 65535, 65536, 65537})
    for prec in (0, 1, 2):
        prev = 0
        for n in ns:
            lo, hi = lib.hawkes_workspace_min_bytes(n, prec), lib.hawkes_workspace_bytes(n, prec)
            assert prev <= lo <= hi, (prec, n)
            assert hi <= lo + (704 << 20) + 256, (prec, n)
            prev = lo
