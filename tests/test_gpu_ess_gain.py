"""What the trained network gains over the method without it, end to end on the GPU (a reduced
version of the comparison the campaign runs at 10^6 events): on a clustered event set of 2 * 10^4
events, exact HMC (warm-up, then a plain chain whose gradient evaluations are the training tuples),
the BF16 surrogate trained on those tuples by the HIP kernels, then delayed-acceptance HMC driven
by it.  The surrogate chain must reach more effective samples per second than the plain chain
while its posterior means agree with the plain chain's within 3 combined Monte Carlo standard
errors (every draw is seeded: the outcome is reproducible; only the seconds vary)."""

import pytest
import torch

import synth
import paper_2407_11349_amd as hk
from paper_2407_11349_amd.mcmc.campaign import Campaign, CampaignConfig, GPUHooks
from paper_2407_11349_amd.mcmc.cut import HawkesCutTarget

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("fallback_prob", [0.0, 0.05])
def test_trained_surrogate_beats_plain_hmc_at_equal_accuracy(tmp_path, fallback_prob):
    """fallback_prob 0: the windowed exact-HMC fallback; 0.05: the fixed-mixture fallback."""
    ev = synth.generate_clustered(n=20_000, seed=1201)
    dev = hk.DeviceEvents.from_arrays(ev.t, ev.x, ev.y, ev.s)
    target = HawkesCutTarget(dev, torch.from_numpy(ev.county).cuda(), torch.from_numpy(ev.rect).cuda(), seed=2201,
                             precision="fp32_skip")
    cfg = CampaignConfig(n_warmup=120, n_plain=400, n_da=400, n_leapfrog=20, seed=7, chunk=100,
                         fallback_prob=fallback_prob)
    c = Campaign(str(tmp_path / "run"), target, GPUHooks(epochs=30, log=None), cfg,
                 log=lambda m: print(m, flush=True))
    assert c.run() == "done"
    s = c.summary()
    print({k: s[k] for k in ("ess_per_s_ratio", "max_mean_diff_in_combined_mcse", "max_rhat")},
          s["da_hmc"]["stats"], s["surrogate"], flush=True)
    assert s["da_hmc"]["ess_per_s"] > s["plain_hmc"]["ess_per_s"]
    assert s["means_agree_within_3_mcse"]
    assert s["max_rhat"] < 1.1
