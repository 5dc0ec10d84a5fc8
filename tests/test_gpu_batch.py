"""GPU parity of the batched log-likelihood (hawkes_loglik_batch): several parameter vectors on the
same events, two per FP32 pair sweep sharing the pair geometry.

Each value is checked against the FP64 oracle at the parameter vector it belongs to (the same
tolerance as hawkes_loglik: 1e-9 relative), and against the single-vector call.  The first vector
of a fused pair is computed exactly as the single sweep computes it (bitwise equal outside the skip
mode).  For the second vector the FP64 squared distance and background exponent are formed from the
first vector's scaled positions and times and then rescaled, so its FP32 values are the single
sweep's up to the FP64 rounding of that rescaling, which changes an FP32 rounding in a few pairs per
billion: results agree to SECOND_TOL (measured 1.5e-13 at 2e4 events, 1e-15 at 1e6).  (Rounding the second vector's squared distance at the first
vector's scale instead moved its triggering sums by 4e-9 relative at 1e6 events: the hardware
exp2's error does not average out identically over two different sets of rounded arguments.)"""

import json
import os

import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2407_11349_amd as hk

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_values.json")
TOL_L = 1e-9
SECOND_TOL = 1e-12  # batch against single call, vectors after the first of a fused pair
AREA = 1.0e6


def _say(msg):
    print(msg, flush=True)


def _thetas():
    """Parameter vectors that differ in every component (as two points of an HMC trajectory do)."""
    a = synth.theta_default()
    b = a * np.array([1.15, 0.8, 1.3, 0.7, 1.25, 0.6])
    c = a * np.array([0.9, 1.2, 0.75, 1.1, 0.85, 1.4])
    return [a, b, c]


def _single(dev, th, prec, rows=None):
    v = hk.loglik(dev, th, precision=prec, rows=rows)
    torch.cuda.synchronize()
    return float(v.item())


def _batch(dev, ths, prec, rows=None):
    v = hk.loglik_batch(dev, np.array(ths), precision=prec, rows=rows)
    torch.cuda.synchronize()
    return v.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp32", "fp32_skip"])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_batch_matches_single_and_oracle(prec, k):
    ev = synth.generate(synth.N100K, n=20000, seed=61)
    dev = hk.DeviceEvents.from_arrays(ev.t, ev.x, ev.y, ev.s)
    ths = _thetas()[:k]
    got = _batch(dev, ths, prec)
    assert got.shape == (k,)
    for j, th in enumerate(ths):
        single = _single(dev, th, prec)
        ref, _ = oracle.loglik(ev.t, ev.x, ev.y, ev.s, th)
        rel_s = abs(got[j] - single) / abs(single)
        rel_o = abs(got[j] - ref) / abs(ref)
        _say(f"batch {prec} k={k} vector {j}: rel diff vs single {rel_s:.2e}, rel err vs oracle {rel_o:.2e}")
        assert rel_o <= TOL_L
        assert rel_s <= (0.0 if j % 2 == 0 and prec == "fp32" else SECOND_TOL)


def test_batch_first_vector_equals_single_sweep():
    """The first vector of a fused pair is computed exactly as the single forward sweep does it."""
    ev = synth.generate(synth.N100K, n=30000, seed=62)
    dev = hk.DeviceEvents.from_arrays(ev.t, ev.x, ev.y, ev.s)
    ths = _thetas()[:2]
    got = _batch(dev, ths, "fp32")
    single = _single(dev, ths[0], "fp32")
    _say(f"first vector: batch {got[0]!r} single {single!r}")
    assert got[0] == single


def test_batch_n100k_against_stored_oracle():
    gold = json.load(open(GOLDEN))["n100k"]
    ev = synth.generate(synth.N100K)
    th = np.array(gold["theta"])
    other = th * np.array([1.05, 0.95, 1.1, 0.9, 1.05, 0.9])
    dev = hk.DeviceEvents.from_arrays(ev.t, ev.x, ev.y, ev.s)
    for prec in ("fp32", "fp32_skip"):
        got = _batch(dev, [other, th], prec)
        rel = abs(got[1] - gold["loglik"]) / abs(gold["loglik"])
        single = _single(dev, other, prec)
        _say(f"n100k {prec}: second vector rel err vs stored oracle {rel:.2e}; "
             f"first vs single {abs(got[0] - single) / abs(single):.2e}")
        assert rel <= TOL_L
        assert abs(got[0] - single) <= (0.0 if prec == "fp32" else 1e-14 * abs(single))


def test_batch_n1m_against_stored_oracle():
    """The full workload (1e6 events, 1200 days): the stored FP64 oracle value as the second vector
    of a fused pair (exponents formed from the other vector's scaling) and as the first."""
    gold = json.load(open(GOLDEN))["n1m"]
    ev = synth.generate(synth.N1M)
    th = np.array(gold["theta"])
    other = th * np.array([0.97, 1.04, 0.95, 1.06, 0.96, 1.05])
    dev = hk.DeviceEvents.from_arrays(ev.t, ev.x, ev.y, ev.s)
    for prec in ("fp32", "fp32_skip"):
        got = _batch(dev, [other, th, th, other], prec)
        for j in (1, 2):
            rel = abs(got[j] - gold["loglik"]) / abs(gold["loglik"])
            _say(f"n1m {prec}: vector {j} rel err vs stored oracle {rel:.2e}")
            assert rel <= TOL_L
        # the same vector first and second of a pair
        assert abs(got[0] - got[3]) <= SECOND_TOL * abs(got[0])


@pytest.mark.parametrize("n", [1, 2, 3, 511, 513, 1537, 5003])
def test_batch_ragged_sizes(n):
    ev = synth.generate(synth.N2K, n=n, seed=700 + n)
    dev = hk.DeviceEvents.from_arrays(ev.t, ev.x, ev.y, ev.s)
    ths = _thetas()[:2]
    for prec in ("fp32", "fp32_skip", "fp64"):
        got = _batch(dev, ths, prec)
        for j, th in enumerate(ths):
            ref, _ = oracle.loglik(ev.t, ev.x, ev.y, ev.s, th)
            tol = 1e-12 if prec == "fp64" else TOL_L
            assert abs(got[j] - ref) <= tol * max(abs(ref), 1.0), (prec, j, got[j], ref)


def test_batch_fp64_equals_single_calls():
    ev = synth.generate(synth.N2K)
    dev = hk.DeviceEvents.from_arrays(ev.t, ev.x, ev.y, ev.s)
    ths = _thetas()
    got = _batch(dev, ths, "fp64")
    for j, th in enumerate(ths):
        assert got[j] == _single(dev, th, "fp64")


def test_batch_row_ranges_and_ties():
    """Row ranges take the row sweep; integer-day times give tie groups and MIXED tiles."""
    ev = synth.generate(synth.N100K, n=12000, seed=63)
    t = np.floor(ev.t)
    dev = hk.DeviceEvents.from_arrays(t, ev.x, ev.y, ev.s)
    ths = _thetas()[:2]
    for rows in ((0, 12000), (0, 1), (4097, 9000), (11999, 12000), (5, 5)):
        got = _batch(dev, ths, "fp32", rows=rows)
        for j, th in enumerate(ths):
            if rows[0] == rows[1]:
                assert got[j] == 0.0
                continue
            ref, _ = oracle.loglik(t, ev.x, ev.y, ev.s, th, rows=rows)
            single = _single(dev, th, "fp32", rows=rows)
            assert abs(got[j] - ref) <= TOL_L * abs(ref) + 5e-7 * np.sqrt(rows[1] - rows[0]), (rows, j)
            assert abs(got[j] - single) <= (0.0 if j == 0 else SECOND_TOL * abs(single) + 1e-9), (rows, j)


def test_batch_uniform_background():
    ev = synth.generate(synth.N100K, n=15000, seed=64)
    dev = hk.DeviceEvents.from_arrays(ev.t, ev.x, ev.y, ev.s, area=AREA)
    ths = _thetas()
    for prec in ("fp32", "fp32_skip"):
        got = _batch(dev, ths, prec)
        for j, th in enumerate(ths):
            ref, _ = oracle.loglik(ev.t, ev.x, ev.y, ev.s, th, area=AREA)
            rel = abs(got[j] - ref) / abs(ref)
            _say(f"uniform {prec} vector {j}: rel err vs oracle {rel:.2e}")
            assert rel <= TOL_L


def test_batch_skip_window_covers_both_vectors():
    """Vectors with very different tau_t and omega: the fused skip sweep must keep every tile
    either vector needs (the larger background window, the smaller omega's triggering window)."""
    ev = synth.generate(synth.N100K, n=20000, seed=65)
    dev = hk.DeviceEvents.from_arrays(ev.t, ev.x, ev.y, ev.s)
    a = synth.theta_default()
    a[2], a[5] = 0.5, 2.0   # short background window, short triggering window
    b = synth.theta_default()
    b[2], b[5] = 20.0, 0.05  # long ones
    for ths in ([a, b], [b, a]):
        got = _batch(dev, ths, "fp32_skip")
        for j, th in enumerate(ths):
            full = _single(dev, th, "fp32")
            ref, _ = oracle.loglik(ev.t, ev.x, ev.y, ev.s, th)
            # the skip mode against the full sweep: the far tiles' triggering terms summed in
            # another order (as in the single skip sweep, up to 1e-11 with tau_t = 0.5 d)
            assert abs(got[j] - full) <= 1e-11 * abs(full), (j, got[j], full)
            assert abs(got[j] - ref) <= TOL_L * abs(ref)


def test_batch_output_tensor_and_stream_order():
    """Results land in a caller-provided tensor; two batches on one workspace in a row."""
    ev = synth.generate(synth.N2K, n=3000, seed=66)
    dev = hk.DeviceEvents.from_arrays(ev.t, ev.x, ev.y, ev.s)
    ws = hk.Workspace(dev.n, "fp32")
    out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
    ths = _thetas()
    hk.loglik_batch(dev, np.array(ths[:2]), precision="fp32", ws=ws, out=out)
    first = out[:2].clone()
    hk.loglik_batch(dev, np.array(ths[1:]), precision="fp32", ws=ws, out=out[2:])
    torch.cuda.synchronize()
    v = out.cpu().numpy()
    assert np.all(np.isfinite(v))
    assert torch.equal(first, out[:2])
    # vector 1 as the second of one pair and the first of the next
    assert abs(v[1] - v[2]) <= SECOND_TOL * abs(v[1])


def test_cut_target_logp_batch_matches_logp():
    """The cut-posterior target's paired evaluation (used by the delayed-acceptance correction)
    against one-at-a-time evaluations under the same latent-location draw; invalid points give
    -inf without a library call."""
    from paper_2407_11349_amd.mcmc.cut import HawkesCutTarget

    ev = synth.generate(synth.N100K, n=8000, seed=67)
    dev = hk.DeviceEvents.from_arrays(ev.t, ev.x, ev.y, ev.s)
    county = torch.as_tensor(ev.county, dtype=torch.int32, device="cuda")
    rect = torch.as_tensor(ev.rect, dtype=torch.float64, device="cuda")
    for prec in ("fp32", "fp32_skip"):
        tgt = HawkesCutTarget(dev, county, rect, seed=5, precision=prec)
        tgt.resample(3)
        z0 = np.log(synth.theta_default())
        z1 = z0 + np.array([0.05, -0.1, 0.08, -0.2, 0.1, -0.3])
        pair = tgt.logp_batch([z0, z1])
        single = [tgt.logp(z0), tgt.logp(z1)]
        assert pair[0] == pytest.approx(single[0], rel=1e-14)
        assert pair[1] == pytest.approx(single[1], rel=SECOND_TOL)
        mixed = tgt.logp_batch([z0, np.full(6, np.nan), z1 + 100.0, z1])
        assert mixed[1] == -np.inf and mixed[2] == -np.inf
        assert mixed[0] == pytest.approx(single[0], rel=1e-14)
        assert mixed[3] == pytest.approx(single[1], rel=SECOND_TOL)


def test_batch_rescues_underflow_limited_rows_per_vector():
    """Narrow kernels put event 1's rate at ~1e-36, below what FP32 sums hold: each vector's
    finalize must put the row on its own rescue list and recompute it in FP64 (the list is
    restarted between the vectors of a pair)."""
    t = np.array([1.0, 1.5])
    x = np.array([0.0, 0.438])
    y = np.array([0.0, 0.0])
    s = np.array([1.0, 1.0])
    narrow = np.array([1.0, 0.05, 0.05, 1.0, 0.05, 1.0])
    wide = synth.theta_default()
    dev = hk.DeviceEvents.from_arrays(t, x, y, s)
    for ths in ([narrow, wide], [wide, narrow], [narrow, narrow * 1.01]):
        got = _batch(dev, ths, "fp32")
        for j, th in enumerate(ths):
            ref, _ = oracle.loglik(t, x, y, s, th)
            single = _single(dev, th, "fp32")
            assert abs(got[j] - ref) <= 5e-7, (j, got[j], ref)
            assert abs(got[j] - single) <= 1e-12 * abs(single), (j, got[j], single)
