"""Host-side logic of bench.py (no GPU): the pair counts behind the FLOP figures, the one-GPU guard, and the
rule that counter-derived fields are reported only for the kernel source they were taken on."""

import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _brute_pair_counts(t):
    n = len(t)
    bg = sum(1 for i in range(n) for j in range(n) if t[i] != t[j])
    causal = sum(1 for i in range(n) for j in range(n) if t[j] < t[i])
    return bg, causal


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_pair_counts_match_brute_force_with_ties(seed):
    rng = np.random.default_rng(seed)
    t = np.sort(rng.integers(0, 12, size=60).astype(np.float64))  # integer days: many ties
    assert bench.pair_counts(t) == _brute_pair_counts(t)


def test_pair_counts_without_ties_give_twenty_flop_per_ordered_pair():
    # background for all N(N-1) ordered pairs, triggering for the N(N-1)/2 causal ones
    n = 1000
    t = np.sort(np.random.default_rng(3).uniform(0, 100, n))
    bg, causal = bench.pair_counts(t)
    assert bg == n * (n - 1) and causal == n * (n - 1) // 2
    flop = bench.FLOP_BG * bg + bench.FLOP_TRIG * causal
    assert flop == 20 * n * (n - 1)


def test_surrogate_flop_counts():
    # 6 -> 256 -> 256 -> 256 -> 1: one pass through the weights is 132,864 multiply-adds; inference is a
    # forward and a reverse pass
    assert bench.MLP_MACS == 6 * 256 + 2 * 256 * 256 + 256 == 132_864
    assert bench.MLP_INFER_FLOP == 531_456


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), ([], {"WORLD_SIZE": "2"})])
def test_more_than_one_gpu_is_refused_with_a_message(argv, env):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv], capture_output=True, text=True,
                       env={**os.environ, **env}, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def _fake_root(tmp_path, profile_hash):
    csrc = tmp_path / "paper_2407_11349_amd" / "csrc"
    csrc.mkdir(parents=True)
    shutil.copy(os.path.join(ROOT, "paper_2407_11349_amd", "csrc", "hawkes_loglik.hip"), csrc / "hawkes_loglik.hip")
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "pair_f32_n1m_traffic.md").write_text(
        "| quantity | value |\n|---|---|\n| HBM bytes per evaluation | 1.5e+11 |\n"
        f"| kernel source hash | {profile_hash} |\n")
    (prof / "pair_f32_n1m_valu_mix.md").write_text(
        "| quantity | value |\n|---|---|\n| issue bound at 2.4 GHz (ms) | 300.0 |\n"
        f"| kernel source hash | {profile_hash} |\n")
    return tmp_path


def test_counter_fields_follow_the_kernel_source(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    _fake_root(tmp_path, "0" * 16)
    assert bench.measured_traffic() is None and bench.issue_bound_ms() is None  # taken on another source
    (tmp_path / "profiles" / "pair_f32_n1m_traffic.md").write_text(
        "| quantity | value |\n|---|---|\n| HBM bytes per evaluation | 1.5e+11 |\n"
        f"| kernel source hash | {bench.kernel_source_hash()} |\n")
    assert bench.measured_traffic() == 1.5e11
    assert bench.issue_bound_ms() is None
    with open(tmp_path / "paper_2407_11349_amd" / "csrc" / "hawkes_loglik.hip", "a") as f:
        f.write("\n")  # any edit of the kernel source retires the counters
    assert bench.measured_traffic() is None


def test_missing_profiles_give_no_fields(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.profile_fields("pair_f32_n1m_traffic.md") == {}
    assert bench.measured_traffic() is None
