"""Checkpoint/resume of the sampler comparison (CPU, oracle-backed target): a run split into
many calls, each restarting from the files of the last checkpoint in a fresh Campaign object,
takes exactly the steps of an uninterrupted run (same draws, statistics, tuples and surrogate),
and every iteration is logged as one JSON line."""

import json
import os

import numpy as np
import pytest

import synth
from paper_2407_11349_amd.mcmc import experiment as ex
from paper_2407_11349_amd.mcmc.campaign import Campaign, CampaignConfig, load_state
from samplers_oracle_target import OracleCutTarget, QuadraticSurrogate


class CPUHooks:
    """Mode search by L-BFGS; the 'surrogate' a quadratic fitted to the tuples (their mean and the
    spread of their positions), a deterministic function of the training data."""

    def find_mode(self, target, z0):
        return ex.find_mode(target, z0, max_iter=60)

    def train(self, Z, L, G, groups):
        m = Z.mean(axis=0)
        var = np.maximum(Z.var(axis=0), 1e-6)
        return {"m": m, "prec": 1.0 / var}, {"tuples": int(Z.shape[0]), "draws": int(np.unique(groups).shape[0])}

    def surrogate(self, a):
        return QuadraticSurrogate(a["m"], a["prec"])


CFG = CampaignConfig(n_warmup=44, n_plain=9, n_da=11, n_leapfrog=4, chunk=4, seed=3, init_eps=0.05,
                     init_inv_mass=0.05)


def _target():
    ev = synth.generate(synth.N2K, n=150, seed=8)
    return OracleCutTarget(ev.t, ev.s, ev.county, ev.rect, seed=91)


def test_resumed_run_equals_uninterrupted_run(tmp_path):
    a_dir, b_dir = str(tmp_path / "a"), str(tmp_path / "b")
    ca = Campaign(a_dir, _target(), CPUHooks(), CFG)
    assert ca.run() == "done"
    calls = 0
    while True:
        cb = Campaign(b_dir, _target(), CPUHooks(), CFG if calls == 0 else None)
        if cb.run(max_chunks=1) == "done":
            break
        calls += 1
        assert calls < 200
    assert calls > 10
    sa, sb = load_state(a_dir), load_state(b_dir)
    for k in ("warm_draws", "plain_draws", "da_draws", "tuples_z", "tuples_ll", "tuples_g", "tuples_group",
              "inv_mass", "sur_m", "sur_prec"):
        assert np.array_equal(sa["arrays"][k], sb["arrays"][k]), k
    for k in ("eps", "rng", "da", "counts", "k"):
        assert sa["meta"][k] == sb["meta"][k], k
    assert sa["arrays"]["warm_draws"].shape[0] == CFG.n_warmup
    assert sa["arrays"]["plain_draws"].shape[0] == CFG.n_plain
    assert sa["arrays"]["da_draws"].shape[0] == CFG.n_da
    # tuples: one per gradient evaluation of the plain chain (n_leapfrog + 1 per iteration)
    assert sa["arrays"]["tuples_z"].shape[0] == CFG.n_plain * (CFG.n_leapfrog + 1)
    st = sa["meta"]["da"]["stats"]
    assert st["iterations"] == CFG.n_da and st["accept"] > 0
    summ = Campaign(a_dir, _target(), CPUHooks()).summary()
    for key in ("ess_per_s_ratio", "means_agree_within_3_mcse", "max_rhat"):
        assert key in summ
    json.dumps(summ)


def test_iterations_are_logged_as_json_lines(tmp_path):
    d = str(tmp_path / "c")
    c = Campaign(d, _target(), CPUHooks(), CFG)
    c.run()
    lines = [json.loads(s) for s in open(os.path.join(d, "iterations.jsonl"))]
    phases = [r["phase"] for r in lines]
    assert phases.count("warmup") == CFG.n_warmup and phases.count("plain") == CFG.n_plain
    assert phases.count("da") == CFG.n_da
    for r in lines:
        assert len(r["z"]) == 6 and isinstance(r["accepted"], bool) and r["t"] >= 0.0
    # draw indices are consecutive across phases (one latent-location draw per iteration)
    ks = [r["k"] for r in lines]
    assert ks == list(range(1, len(ks) + 1))


def test_checkpoint_guards(tmp_path):
    d = str(tmp_path / "g")
    c = Campaign(d, _target(), CPUHooks(), CFG)
    c.run(max_chunks=2)
    other = CampaignConfig(**{**CFG.__dict__, "n_da": 5})
    with pytest.raises(ValueError):
        Campaign(d, _target(), CPUHooks(), other)
    # a checkpoint whose two files come from different saves is refused
    meta = json.load(open(os.path.join(d, "state.json")))
    meta["version"] += 1
    json.dump(meta, open(os.path.join(d, "state.json"), "w"))
    with pytest.raises(RuntimeError):
        load_state(d)


def test_lines_logged_after_the_last_save_are_dropped_on_resume(tmp_path):
    """A call that ends between two saves (killed mid-chunk) leaves log lines of iterations the next
    call runs again: resuming truncates the log to what the checkpoint covers, so every iteration
    appears once."""
    d = str(tmp_path / "k")
    c = Campaign(d, _target(), CPUHooks(), CFG)
    c.run(max_chunks=3)
    log_path = os.path.join(d, "iterations.jsonl")
    n_saved = len(open(log_path).read().splitlines())
    with open(log_path, "a") as f:  # what an interrupted chunk would have appended
        f.write(json.dumps({"phase": "warmup", "it": 999}) + "\n")
    c2 = Campaign(d, _target(), CPUHooks(), CFG)
    assert len(open(log_path).read().splitlines()) == n_saved
    assert c2.run() == "done"
    rows = [json.loads(line) for line in open(log_path)]
    assert [r["phase"] for r in rows].count("da") == CFG.n_da
    assert not any(r.get("it") == 999 for r in rows)


def test_checkpoint_from_before_a_new_config_field_resumes(tmp_path):
    """A checkpoint written before CampaignConfig gained a field (here fallback_prob) resumes with the
    field's default, under the explicit configuration too, and finishes like a fresh run."""
    d = str(tmp_path / "old")
    Campaign(d, _target(), CPUHooks(), CFG).run(max_chunks=2)
    meta = json.load(open(os.path.join(d, "state.json")))
    del meta["config"]["fallback_prob"]
    json.dump(meta, open(os.path.join(d, "state.json"), "w"))
    c = Campaign(d, _target(), CPUHooks(), CFG)
    assert c.cfg == CFG
    assert c.run() == "done"
    ref = str(tmp_path / "ref")
    Campaign(ref, _target(), CPUHooks(), CFG).run()
    assert np.array_equal(load_state(d)["arrays"]["da_draws"], load_state(ref)["arrays"]["da_draws"])
