"""AddressSanitizer/UndefinedBehaviorSanitizer builds (CPU only): the FP64 oracle with both
sanitizers (gcc), and the HIP library with both on its host code, each run by a driver in
tests/csrc.  A sanitizer report fails the driver; the sanitized oracle must also reproduce the
regular build's values."""

import os
import subprocess
import sys

import numpy as np

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ENV = {**os.environ, "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0", "UBSAN_OPTIONS": "print_stacktrace=1"}


def _driver(name):
    path = os.path.join(CSRC, name)
    if not os.path.exists(path):
        sys.path.insert(0, CSRC)
        from build_sanitized import build_sanitized

        build_sanitized()
    return path


def _lcg_events(n):
    st = 12345 + n
    mask = (1 << 64) - 1

    def nxt():
        nonlocal st
        st = (st * 6364136223846793005 + 1442695040888963407) & mask
        return (st >> 11) * 2.0 ** -53

    t, x, y, s = [], [], [], []
    acc = 0.0
    for _ in range(n):
        acc += 3.0 * nxt()
        t.append(np.floor(acc))
        x.append(50.0 * nxt())
        y.append(50.0 * nxt())
        s.append(0.5 + nxt())
    return np.array(t), np.array(x), np.array(y), np.array(s)


def test_sanitized_oracle_runs_clean_and_matches():
    res = subprocess.run([_driver("sanitize_oracle")], capture_output=True, text=True, env=ENV, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "ERROR: AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr
    lines = res.stdout.splitlines()
    assert lines[-1] == "OK"
    th = np.array([0.5, 10.0, 7.0, 0.3, 2.0, 0.2])
    checked = 0
    for ln in lines:
        if not ln.startswith("n "):
            continue
        f = ln.split()
        n, area = int(f[1]), float(f[3])
        ll, g = float(f[5]), np.array([float(v) for v in f[7:13]])
        t, x, y, s = _lcg_events(n)
        ll_ref, g_ref = oracle.loglik(t, x, y, s, th, area=area)
        assert ll == ll_ref and np.array_equal(g, g_ref)
        checked += 1
    assert checked == 10


def test_sanitized_library_host_validation_runs_clean():
    res = subprocess.run([_driver("sanitize_abi")], capture_output=True, text=True, env=ENV, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "ERROR: AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr
    assert res.stdout.strip().splitlines()[-1] == "OK"
