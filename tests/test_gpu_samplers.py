"""GPU parity of the sampler layer (cut-posterior HMC and delayed-acceptance HMC) over the HIP
likelihood: the same samplers, seeds and latent-location draws run once over the FP64 CPU
oracle (OracleCutTarget: oracle likelihood and the oracle's Philox draw) and once over
HawkesCutTarget (the HIP library's likelihood and draw).  With the FP64 sweep the two runs
must take the same accept/reject decisions and reach the same points within 1e-9; with the
FP32 sweep (1e-9 relative loglik, 1e-6 gradient) the same decisions and points within 1e-5.
The delayed-acceptance runs use a fixed quadratic surrogate, identical on both sides, so that
only the exact likelihood (stage 2 and the fallback) differs between them."""

import numpy as np
import pytest
import torch

import synth
import paper_2407_11349_amd as hk
from paper_2407_11349_amd.mcmc import HMC
from paper_2407_11349_amd.mcmc import experiment as ex
from paper_2407_11349_amd.mcmc.cut import HawkesCutTarget
from samplers_oracle_target import OracleCutTarget, QuadraticSurrogate

pytestmark = pytest.mark.gpu

N, SEED = 400, 77
STEP, INV_MASS, N_LEAPFROG, ITERS = 0.3, 0.05, 10, 20


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def setup():
    ev = synth.generate(synth.N2K, n=N, seed=5)
    ora = OracleCutTarget(ev.t, ev.s, ev.county, ev.rect, seed=SEED)
    ora.resample(0)
    zm = ex.find_mode(ora, np.log(synth.theta_default()), max_iter=100)
    return ev, zm


def _targets(ev, prec):
    ora = OracleCutTarget(ev.t, ev.s, ev.county, ev.rect, seed=SEED)
    dev = hk.DeviceEvents.from_arrays(ev.t, ev.x, ev.y, ev.s)
    gpu = HawkesCutTarget(dev, torch.from_numpy(ev.county).cuda(), torch.from_numpy(ev.rect).cuda(), seed=SEED,
                          precision=prec)
    return ora, gpu


def _hmc(target):
    return HMC(target, n_leapfrog=N_LEAPFROG, step_size=STEP, inv_mass=np.full(6, INV_MASS),
               rng=np.random.default_rng(3))


def _accepts(draws, z0):
    prev = np.vstack([z0[None, :], draws[:-1]])
    return [not np.array_equal(a, b) for a, b in zip(draws, prev)]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("fp32", 1e-5)])
def test_plain_hmc_matches_oracle_backed_run(setup, prec, tol):
    ev, zm = setup
    ora, gpu = _targets(ev, prec)
    _say(f"plain HMC parity {prec}: oracle run")
    r_o = ex.run_plain_hmc(ora, _hmc(ora), zm, ITERS, 1)
    _say(f"plain HMC parity {prec}: GPU run")
    r_g = ex.run_plain_hmc(gpu, _hmc(gpu), zm, ITERS, 1)
    acc_o, acc_g = _accepts(r_o.draws, zm), _accepts(r_g.draws, zm)
    assert acc_o == acc_g
    assert 0 < sum(acc_o) < ITERS  # both kinds of decision are exercised
    np.testing.assert_allclose(r_g.draws, r_o.draws, rtol=0, atol=tol)
    assert r_o.n_grad == r_g.n_grad


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("fp32", 1e-5)])
def test_delayed_acceptance_hmc_matches_oracle_backed_run(setup, prec, tol):
    ev, zm = setup
    sur = QuadraticSurrogate(zm, np.full(6, 1.0 / INV_MASS))
    ora, gpu = _targets(ev, prec)
    _say(f"DA-HMC parity {prec}: oracle run")
    r_o = ex.run_da_hmc(ora, sur, _hmc(ora), zm, ITERS, 30, ora.prior_var, seed=9)
    _say(f"DA-HMC parity {prec}: GPU run")
    r_g = ex.run_da_hmc(gpu, sur, _hmc(gpu), zm, ITERS, 30, gpu.prior_var, seed=9)
    assert r_o.stats == r_g.stats
    s = r_o.stats
    assert 0 < s["stage2_accept"] < s["stage1_accept"]  # stage 2 both accepts and rejects
    assert _accepts(r_o.draws, zm) == _accepts(r_g.draws, zm)
    np.testing.assert_allclose(r_g.draws, r_o.draws, rtol=0, atol=tol)
    assert r_o.n_loglik == r_g.n_loglik


def test_da_fallback_matches_oracle_backed_run(setup):
    """A surrogate far from the posterior: stage 2 rejects, the windowed acceptance drops below
    0.5 and iterations fall back to exact HMC; both runs take the same path."""
    ev, zm = setup
    sur = QuadraticSurrogate(zm + 1.5, np.full(6, 1.0 / INV_MASS))
    ora, gpu = _targets(ev, "fp64")
    runs = []
    for tgt in (ora, gpu):
        hmc = _hmc(tgt)
        da = ex.DelayedAcceptanceHMC(tgt, lambda z: (float(sur.value_and_grad(z)[0][0]) - 0.5 * float(z @ z) / 100.0,
                                                     sur.value_and_grad(z)[1][0] - z / 100.0),
                                     n_leapfrog=N_LEAPFROG, step_size=STEP, inv_mass=hmc.inv_mass,
                                     rng=np.random.default_rng(21), window=4)
        tgt.resample(50)
        st = da.init_state(zm)
        zs = []
        for it in range(ITERS):
            st, _, _ = da.step(st)
            zs.append(st.z.copy())
            tgt.resample(51 + it)
            st = da.refresh_exact(st)
        runs.append((np.array(zs), dict(da.stats)))
    (z_o, s_o), (z_g, s_g) = runs
    assert s_o == s_g and s_o["fallback"] > 0
    np.testing.assert_allclose(z_g, z_o, rtol=0, atol=1e-9)
