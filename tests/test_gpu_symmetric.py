"""GPU checks of the symmetric FP32 sweep (whole event set): each background term of two
events in strictly ordered blocks is evaluated once and added to both events' sums.

Against the FP64 oracle it meets the FP32 tolerances (1e-9 loglik, 1e-6 gradient, 5e-6
per-event rate).  Against the row sweep of the same call (symmetric groups = 0) it differs
only in the order of FP32 background sums (a wave's 128 targets instead of 8-source groups),
and between group counts only in the FP64 order of partial sums."""

import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2407_11349_amd as hk
from paper_2407_11349_amd import _lib

pytestmark = pytest.mark.gpu

TOL_L, TOL_G, TOL_EV = 1e-9, 1e-6, 5e-6
DEFAULT_GROUPS = _lib.SYM_GROUPS_DEFAULT


def _say(msg):
    print(msg, flush=True)


def _run(dev, th, prec="fp32", groups=DEFAULT_GROUPS):
    """groups: the symmetric sweep's group count, or 0 for the row sweep over the whole set."""
    sg = groups if groups > 0 else -1
    ll, g = hk.loglik_grad(dev, th, precision=prec, symmetric_groups=sg)
    lam, comp = hk.event_terms(dev, th, precision=prec, symmetric_groups=sg)
    torch.cuda.synchronize()
    return float(ll.item()), g.cpu().numpy(), lam.cpu().numpy(), comp.cpu().numpy()


def _events(kind, n, seed):
    if kind == "dense":      # 100 days: a 512-event block spans ~2.5 days
        ev = synth.generate(synth.N2K, n=n, seed=seed)
        return ev.t, ev
    if kind == "sparse":     # 1000 days: a block spans ~25 days
        ev = synth.generate(synth.N100K, n=n, seed=seed)
        return ev.t, ev
    if kind == "days":       # integer days: blocks share days with their neighbours
        ev = synth.generate(synth.N2K, n=n, seed=seed)
        return np.floor(ev.t), ev
    if kind == "five_days":  # 5 distinct times: runs of ties many blocks long
        ev = synth.generate(synth.N2K, n=n, seed=seed)
        return np.floor(ev.t / 20.0) * 20.0, ev
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["dense", "sparse", "days", "five_days"])
def test_symmetric_against_oracle_and_row_sweep(kind):
    t, ev = _events(kind, 20000, 77)
    th = synth.theta_default()
    ll_ref, g_ref, lam_ref, comp_ref, _ = oracle.loglik(t, ev.x, ev.y, ev.s, th, per_row=True)
    dev = hk.DeviceEvents.from_arrays(t, ev.x, ev.y, ev.s)
    sym = _run(dev, th)
    row = _run(dev, th, groups=0)
    rel_l = abs(sym[0] - ll_ref) / abs(ll_ref)
    rel_g = np.max(np.abs(sym[1] - g_ref) / np.abs(g_ref))
    d_l = abs(sym[0] - row[0]) / abs(row[0])
    d_g = np.max(np.abs(sym[1] - row[1]) / np.abs(row[1]))
    _say(f"symmetric {kind}: loglik rel err {rel_l:.2e}, grad {rel_g:.2e}; vs row sweep {d_l:.2e}, {d_g:.2e}")
    assert rel_l <= TOL_L and rel_g <= TOL_G
    pos = lam_ref > 0
    np.testing.assert_allclose(sym[2][pos], lam_ref[pos], rtol=TOL_EV)
    np.testing.assert_allclose(sym[3], comp_ref, rtol=1e-13, atol=1e-13)
    # the two FP32 sweeps: only the order of FP32 background sums differs
    assert d_l <= 1e-10
    assert d_g <= 1e-7
    np.testing.assert_allclose(sym[2], row[2], rtol=1e-6)


@pytest.mark.parametrize("groups", [1, 2, 3, 5, 41, 160, 384])
def test_group_counts_change_only_fp64_order(groups):
    t, ev = _events("days", 9000, 3)
    th = synth.theta_default()
    dev = hk.DeviceEvents.from_arrays(t, ev.x, ev.y, ev.s)
    ref = _run(dev, th)
    got = _run(dev, th, groups=groups)
    assert got[0] == pytest.approx(ref[0], rel=1e-13)
    np.testing.assert_allclose(got[1], ref[1], rtol=1e-10)
    np.testing.assert_allclose(got[2], ref[2], rtol=1e-13)


@pytest.mark.parametrize("n", [1, 2, 511, 512, 513, 1024, 1537, 2049])
@pytest.mark.parametrize("prec", ["fp32", "fp32_skip"])
def test_block_edges_per_event(n, prec):
    """Sizes at and around block (512) and tile (256) boundaries, including a last block of
    one event: lanes past the end must add nothing to the column sums."""
    ev = synth.generate(synth.N2K, n=n, seed=1300 + n)
    th = synth.theta_default()
    th[2] = 1.5  # short background range in time: strict block pairs even at small n
    _, _, lam_ref, comp_ref, _ = oracle.loglik(ev.t, ev.x, ev.y, ev.s, th, per_row=True)
    for groups in (DEFAULT_GROUPS, 1):
        _, _, lam, comp = _run(hk.DeviceEvents.from_arrays(ev.t, ev.x, ev.y, ev.s), th, prec, groups)
        pos = lam_ref > 0
        np.testing.assert_allclose(lam[pos], lam_ref[pos], rtol=TOL_EV)
        np.testing.assert_allclose(comp, comp_ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("area", [0.0, 1e6])
def test_skip_equals_full_on_the_symmetric_sweep(area):
    """Over the whole set both modes use the same partition, and the terms the skip mode
    leaves out are exact zeros; only the order in which the far tiles' triggering terms are
    summed differs (the full sweep takes them in the column rotation), so the results agree
    to rounding of those terms, which are below e^(-omega * 104 d) = 1e-9 of the rates."""
    t, ev = _events("sparse", 30000, 12)
    th = synth.theta_default()
    dev = hk.DeviceEvents.from_arrays(t, ev.x, ev.y, ev.s, area=area)
    full = _run(dev, th, "fp32")
    skip = _run(dev, th, "fp32_skip")
    assert skip[0] == pytest.approx(full[0], rel=1e-14)
    np.testing.assert_allclose(skip[1], full[1], rtol=1e-11)
    np.testing.assert_allclose(skip[2], full[2], rtol=1e-12)
    assert np.array_equal(skip[3], full[3])


def test_uniform_background_ties_against_row_sweep():
    t, ev = _events("days", 20000, 5)
    th = synth.theta_default()
    dev = hk.DeviceEvents.from_arrays(t, ev.x, ev.y, ev.s, area=1e6)
    ll_ref, g_ref = oracle.loglik(t, ev.x, ev.y, ev.s, th, area=1e6)
    sym = _run(dev, th)
    row = _run(dev, th, groups=0)
    rel_l = abs(sym[0] - ll_ref) / abs(ll_ref)
    _say(f"symmetric uniform days: loglik rel err {rel_l:.2e}, vs row sweep {abs(sym[0] - row[0]) / abs(row[0]):.2e}")
    assert rel_l <= TOL_L
    np.testing.assert_allclose(sym[1], g_ref, rtol=TOL_G)
    # with the uniform background every pair with the same day gap has the same term, so the
    # FP32 rounding of the sums (and of exp2 at those few arguments) does not average out as
    # fast; the two sweeps agree to a few 1e-10 (measured 2.3e-10), both within 1e-9 of the oracle
    assert sym[0] == pytest.approx(row[0], rel=5e-10)
    np.testing.assert_allclose(sym[2], row[2], rtol=1e-6)


@pytest.mark.parametrize("kind", ["dense", "days"])
def test_fp64_symmetric_against_row_sweep_and_oracle(kind):
    """The FP64 sweep takes the same symmetric decomposition (column sums in FP64)."""
    t, ev = _events(kind, 6000, 21)
    th = synth.theta_default()
    ll_ref, g_ref, lam_ref, _, _ = oracle.loglik(t, ev.x, ev.y, ev.s, th, per_row=True)
    dev = hk.DeviceEvents.from_arrays(t, ev.x, ev.y, ev.s)
    sym = _run(dev, th, "fp64")
    row = _run(dev, th, "fp64", groups=0)
    assert abs(sym[0] - ll_ref) <= 1e-12 * abs(ll_ref)
    np.testing.assert_allclose(sym[1], g_ref, rtol=1e-10)
    np.testing.assert_allclose(sym[2], lam_ref, rtol=1e-12)
    assert sym[0] == pytest.approx(row[0], rel=1e-13)
    np.testing.assert_allclose(sym[1], row[1], rtol=1e-11)
