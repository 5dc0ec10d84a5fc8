"""Benchmark: log-likelihood + gradient pairs/s at N = 1e6 on one MI355X.

One step = one pass of the hot path over the 1e6-event workload (1200 days,
3000 rectangular counties, LogNormal(5, 1.5) densities): redraw every latent
location uniformly inside its county (the cut-posterior X-update), then one
fused FP32 log-likelihood + 6-gradient evaluation with FP64 finalize.
Inputs are synthetic and resident in HBM before timing starts.

Prints one JSON line.  Extra fields: the same evaluation in the FP64 sweep,
the FP32 skip mode (same result without the exactly-zero background terms;
reported apart, never as the O(N^2) metric), the forward-only sweep for one
and for two parameter vectors, the roofline of the dominant kernel (pair
sweep), the path's smaller steps (latent-location draw, surrogate inference
and training step), a reduced live run of the surrogate-HMC vs plain-HMC
comparison (ESS/s), and the FP64 CPU oracle timed on a bounded sample of
target rows on the host cores.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "loglik+grad pairs/s at N=1M, FP32 vs FP64; ESS/s surrogate-HMC vs plain HMC"
PEAK_FP32_TFLOPS = 157.3  # MI355X FP32 vector: 256 CU x 2.4 GHz x 256 FLOP/clk
PEAK_BF16_TFLOPS = 2500.0  # MI355X dense BF16 matrix cores (no sparsity)
PEAK_FP64_TFLOPS = 78.6  # MI355X FP64 vector
# v_exp_f32 issue rate measured on the box (31.9 lane-ops/clk/CU, profiles/valu_rates_gfx950.md)
EXP_PEAK_PER_S = 1.958e13
# algorithmic FLOP per pair of the fused sweep (FMA = 2, add/sub/mul = 1; exp counted apart):
# background 15 for every pair, triggering 10 more for causal pairs
FLOP_BG, FLOP_TRIG = 15, 10
# the symmetric sweep adds a pair's background term to the source's sums too: 1 add + 2 FMA
FLOP_COL = 5


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the pair-sweep source: traffic counters are valid only for the kernel they measured."""
    import hashlib

    src = os.path.join(ROOT, "paper_2407_11349_amd", "csrc", "hawkes_loglik.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def profile_fields(name: str) -> dict:
    """The two-column table rows of a committed rocprofv3 summary under profiles/, if its counters
    were taken on the current kernel source (its `kernel source hash` row); else {}."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return {}
    fields = {}
    for line in open(path):
        if line.startswith("|") and line.count("|") >= 3:
            cells = [c.strip() for c in line.strip().strip("|").split("|")]
            if len(cells) >= 2:
                fields.setdefault(cells[0], cells[1])
    return fields if fields.get("kernel source hash") == kernel_source_hash() else {}


def measured_traffic() -> float | None:
    """HBM bytes of one evaluation's pair sweep (its pair-kernel passes and folds) from the committed counter
    summary (None if stale)."""
    try:
        return float(profile_fields("pair_f32_n1m_traffic.md")["HBM bytes per evaluation"])
    except (KeyError, ValueError):
        return None


def issue_bound_ms() -> float | None:
    """The pair sweep's VALU issue bound at 2.4 GHz (its counted instruction mix weighted by the
    measured single-kind issue rates) from the committed SQ counter summary (None if stale)."""
    try:
        return float(profile_fields("pair_f32_n1m_valu_mix.md")["issue bound at 2.4 GHz (ms)"])
    except (KeyError, ValueError):
        return None


def pair_counts(t: np.ndarray) -> tuple[int, int]:
    """(background pairs, causal pairs) with ties excluded, from sorted times."""
    lo = np.searchsorted(t, t, side="left")
    hi = np.searchsorted(t, t, side="right")
    n = t.shape[0]
    causal = int(lo.sum())
    bg = int((n - (hi - lo)).sum())
    return bg, causal


def parity_vs_stored_oracle(hk, torch, ev, th, ws32) -> dict | None:
    """Untimed: FP32 and FP64 loglik+grad at the generator's locations against the FP64 oracle's
    stored value of this workload (tests/golden/oracle_values.json, written from oracle/ only);
    relative errors, the gradient's per component (max) and as a vector norm."""
    path = os.path.join(ROOT, "tests", "golden", "oracle_values.json")
    gold = json.load(open(path)).get("n1m") if os.path.exists(path) else None
    if gold is None or gold["n"] != ev.n or not np.allclose(gold["theta"], th):
        return None
    dev = hk.DeviceEvents.from_arrays(ev.t, ev.x, ev.y, ev.s, device="cuda")
    g_ref = np.array(gold["grad"])
    out = {"reference": "FP64 oracle, stored (n1m, generator locations)", "tolerance": {"loglik": 1e-9, "grad": 1e-6}}
    for prec in ("fp32", "fp64"):
        ws = ws32 if prec == "fp32" else hk.Workspace(ev.n, "fp64")
        ll, g = hk.loglik_grad(dev, th, precision=prec, ws=ws)
        torch.cuda.synchronize()
        ll, g = float(ll.item()), g.cpu().numpy()
        out[prec] = {"loglik_rel_err": abs(ll - gold["loglik"]) / abs(gold["loglik"]),
                     "grad_rel_err_max": float(np.max(np.abs(g - g_ref) / np.abs(g_ref))),
                     "grad_rel_err_norm": float(np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref))}
    return out


def cpu_baseline(ev, th, budget_s: float = 15.0) -> dict:
    """The FP64 oracle on a bounded sample of target rows x all sources."""
    import oracle

    n = ev.n
    probe = 200
    t0 = time.perf_counter()
    oracle.loglik(ev.t, ev.x, ev.y, ev.s, th, rows=(n // 2, n // 2 + probe))
    dt = time.perf_counter() - t0
    rows = int(max(probe, min(n, probe * budget_s / max(dt, 1e-3))))
    r0 = (n - rows) // 2
    t0 = time.perf_counter()
    oracle.loglik(ev.t, ev.x, ev.y, ev.s, th, rows=(r0, r0 + rows))
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": rows * (n - 1) / dt, "unit": "pairs/s", "cores": cores, "kind": "oracle",
            "sample": f"{rows} target rows (middle of the time range) x {n} sources, loglik+grad, FP64, "
                      f"{dt:.1f} s"}


# Surrogate network 6 -> 256 -> 256 -> 256 -> 1: multiply-adds of one pass through its weights (biases and GELUs
# not counted), and the passes per sample of inference (value + input gradient) and of one training step
# (primal, input-gradient reverse, tangent along the gradient residual, the reverse of primal and tangent
# through W3 and W2 (two cotangents each), and the per-sample weight-gradient outer products, two per matrix).
MLP_H, MLP_DZ = 256, 6
MLP_MACS = MLP_DZ * MLP_H + 2 * MLP_H * MLP_H + MLP_H
MLP_INFER_FLOP = 2 * 2 * MLP_MACS
MLP_TRAIN_FLOP = 2 * (MLP_MACS                      # primal
                      + MLP_MACS                    # reverse for grad_z f
                      + MLP_DZ * MLP_H + 2 * MLP_H * MLP_H  # tangent along r
                      + 4 * MLP_H * MLP_H           # two cotangents through W3^T and W2^T
                      + 2 * MLP_MACS)               # weight-gradient outer products (two per matrix)
HBM_PEAK_GBS = 8000.0


def event_ms(torch, fn, reps: int) -> float:
    """Average milliseconds per call of fn, by HIP events on torch's current stream (the library enqueues its
    kernels there), after one untimed call."""
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) / reps


def component_timings(hk, torch, county, rect, x, y) -> dict:
    """The path's smaller steps: the latent-location draw at the workload's size, and the surrogate network's
    inference (batch 1, as inside a leapfrog trajectory, and a large batch) and training step."""
    from paper_2407_11349_amd.surrogate import P as MLP_P, SurrogateNet
    from synth.mlp_init import init_params

    n = int(county.shape[0])
    it = [0]

    def draw():
        it[0] += 1
        hk.resample_locations(county, rect, 2002, it[0], x, y)

    ms = event_ms(torch, draw, 50)
    nbytes = n * (4 + 16) + rect.numel() * 8  # county id in, x and y out, the rectangle table once
    out = {"resample": {"us_per_call": ms * 1e3, "events": n, "algorithmic_bytes": nbytes,
                        "achieved_gbs": nbytes / (ms / 1e3) / 1e9,
                        "frac_of_hbm_peak": nbytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS}}
    net = SurrogateNet(init_params(0))
    g = torch.Generator(device="cuda").manual_seed(0)
    z1 = torch.randn(1, 6, device="cuda", generator=g)
    zb = torch.randn(21000, 6, device="cuda", generator=g)
    ms1 = event_ms(torch, lambda: net.forward(z1), 200)
    msb = event_ms(torch, lambda: net.forward(zb), 10)
    t0 = time.perf_counter()
    for _ in range(50):
        f, gz = net.forward(z1)
        f.cpu(), gz.cpu()
    host_us = (time.perf_counter() - t0) / 50 * 1e6
    out["mlp_forward"] = {
        "batch1_us": ms1 * 1e3, "batch1_host_round_trip_us": host_us,
        "batch21000_ms": msb, "samples_per_s": 21000 / (msb / 1e3),
        "flop_per_sample": MLP_INFER_FLOP, "achieved_tflops": MLP_INFER_FLOP * 21000 / (msb / 1e3) / 1e12,
        "frac_of_bf16_dense_peak": MLP_INFER_FLOP * 21000 / (msb / 1e3) / 1e12 / PEAK_BF16_TFLOPS,
        "note": "value and input gradient; batch 21000 on the matrix cores (BF16 weights, activations as hi + lo "
                "BF16 pairs, so the cores execute twice the counted FLOP; FP32 accumulation), batch 1 by the "
                "one-sample kernel"}
    B = 256
    zt = torch.randn(B, 6, device="cuda", generator=g)
    yt = torch.randn(B, device="cuda", generator=g)
    gt = torch.randn(B, 6, device="cuda", generator=g)
    grad = torch.empty(MLP_P, dtype=torch.float32, device="cuda")
    step = [0]

    def train_step():
        step[0] += 1
        net.loss_grad(zt, yt, gt, 1.0, grad=grad)
        net.adam_step(grad, step[0], 1e-4)

    mst = event_ms(torch, train_step, 50)
    out["mlp_train_step"] = {
        "batch": B, "ms_per_step": mst, "flop_per_sample": MLP_TRAIN_FLOP,
        "achieved_tflops": MLP_TRAIN_FLOP * B / (mst / 1e3) / 1e12,
        "frac_of_bf16_dense_peak": MLP_TRAIN_FLOP * B / (mst / 1e3) / 1e12 / PEAK_BF16_TFLOPS,
        "note": "Sobolev loss, parameter gradient and Adam update for one batch (3 kernels: training pass and "
                "weight-gradient contraction on the matrix cores, Adam with the BF16 refresh)"}
    return out


def sampler_costs(args, hk, synth, torch):
    """Per-call costs of the samplers' exact steps on the clustered workload at another size (no chains): the
    latent-location draw, one loglik+gradient (plain HMC: 21 per iteration), one two-vector loglik (the
    delayed-acceptance correction) and a 20-step surrogate trajectory, at the posterior scales of the 1e5 runs."""
    from paper_2407_11349_amd.surrogate import SurrogateNet, Standardiser, Surrogate
    from synth.mlp_init import init_params

    ev = synth.generate_clustered(n=args.sampler_costs)
    dev = hk.DeviceEvents.from_arrays(ev.t, ev.x, ev.y, ev.s, device="cuda")
    county = torch.from_numpy(ev.county).cuda()
    rect = torch.from_numpy(ev.rect).cuda()
    th = np.exp(np.array([-0.198, 2.535, 2.421, -1.709, 2.550, -1.082]))  # posterior means at 1e5 events
    th2 = np.stack([th, th * np.array([1.01, 0.99, 1.01, 0.99, 1.01, 0.99])])
    ws = hk.Workspace(ev.n, "fp32_skip")
    it = [0]

    def draw():
        it[0] += 1
        hk.resample_locations(county, rect, 2002, it[0], dev.x, dev.y)

    grad = event_ms(torch, lambda: hk.loglik_grad(dev, th, precision="fp32_skip", ws=ws), 3)
    pair = event_ms(torch, lambda: hk.loglik_batch(dev, th2, precision="fp32_skip", ws=ws), 3)
    one = event_ms(torch, lambda: hk.loglik(dev, th, precision="fp32_skip", ws=ws), 3)
    rs = event_ms(torch, draw, 10)
    std = Standardiser(m_z=np.log(th), s_z=np.full(6, 0.03), m_y=0.0, s_y=4.0)
    sur = Surrogate(SurrogateNet(init_params(3)), std)
    z0 = np.log(th)
    t0 = time.perf_counter()
    for _ in range(20):
        sur.leapfrog(z0, np.zeros(6), np.zeros(6), 0.25, np.full(6, 1e-3), 20, 100.0)
    traj = (time.perf_counter() - t0) / 20 * 1e3
    res = {"workload": ev.config.name, "n_events": ev.n, "precision": "fp32_skip",
           "ms_loglik_grad": grad, "ms_loglik_pair": pair, "ms_loglik": one, "ms_resample": rs,
           "ms_surrogate_trajectory_20_steps_host_round_trip": traj,
           "ms_plain_hmc_iteration": 21 * grad + rs,
           "note": "kernel time of each call (HIP events on the library's stream); the trajectory includes its "
                   "host round trip"}
    print(json.dumps(res), flush=True)


def run_surrogate_fit(args, hk, synth, torch):
    """Surrogate training at 1e5 events: exact-HMC burn-in on the cut posterior recording about 20,000
    (log theta, l, dl/dlog theta) tuples, 60 epochs of the HIP Sobolev training, and the held-out errors over
    whole held-out latent-location draws."""
    from paper_2407_11349_amd.mcmc.experiment import surrogate_fit

    # n100k: the generator of the FP32 precision checks (uniform times); clustered: the branching-process
    # workload of the sampler comparison at the same size
    ev = synth.generate(synth.N100K) if args.fit_workload == "n100k" else synth.generate_clustered(n=100_000)
    cfg = ev.config
    dev = hk.DeviceEvents.from_arrays(ev.t, ev.x, ev.y, ev.s, device="cuda")
    county = torch.from_numpy(ev.county).cuda()
    rect = torch.from_numpy(ev.rect).cuda()
    out = surrogate_fit(dev, county, rect, n_burn=args.fit_burn, log=log)
    held = out["surrogate"]
    res = {"metric": "surrogate held-out loglik error", "value": held["loglik_rmse_within_draw"], "unit": "nats",
           "higher_is_better": False, "data": "synthetic",
           "config": {"workload": cfg.name, "n_events": ev.n, "tuples": held["tuples"], "epochs": held["epochs"],
                      "network": "6-256-256-256-1 GELU, BF16 weights, FP32 accumulation",
                      "loss": "Sobolev (value + gradient), lambda 1"},
           "detail": out}
    print(json.dumps(res), flush=True)


def run_ess(args, hk, synth, torch):
    """ESS/s of delayed-acceptance HMC with the BF16 surrogate against plain exact-gradient HMC, both on the
    cut posterior (X redrawn every iteration) with the FP32 GPU likelihood, 20 leapfrog steps."""
    from paper_2407_11349_amd.mcmc.experiment import compare

    # a clustered (branching-process) workload: its posterior is concentrated, unlike that of the
    # uniform-time workloads whose temporal scale is not identified
    ev = synth.generate_clustered(n=args.ess_n)
    cfg = ev.config
    dev = hk.DeviceEvents.from_arrays(ev.t, ev.x, ev.y, ev.s, device="cuda")
    county = torch.from_numpy(ev.county).cuda()
    rect = torch.from_numpy(ev.rect).cuda()
    out = compare(dev, county, rect, n_burn=args.ess_burn, n_iter=args.ess_iter, n_warmup=args.ess_warmup, log=log,
                  replicate=args.ess_replicate, fallback_prob=args.fallback_prob)
    res = {"metric": "ESS/s surrogate-HMC vs plain HMC", "value": out["ess_per_s_ratio"], "unit": "ratio",
           "higher_is_better": True, "data": "synthetic",
           "config": {"workload": cfg.name, "n_events": ev.n, "burn_in": args.ess_burn, "iterations": args.ess_iter,
                      "warmup": args.ess_warmup, "leapfrog": 20, "step": "resample X + sampler iteration",
                      "replicate": args.ess_replicate},
           "detail": out}
    print(json.dumps(res), flush=True)


def ess_reduced(hk, synth, torch) -> dict:
    """The sampler comparison, reduced so that it runs live in the default bench (about 10 s): a clustered
    event set of 2 * 10^4 events, FP32 skip-mode likelihood with X redrawn every iteration, 120 exact-HMC
    warm-up iterations, 400 plain exact-gradient HMC iterations whose gradient evaluations train the BF16
    surrogate (30 epochs), then 400 delayed-acceptance HMC iterations driven by it (20 leapfrog steps, exact
    fallback below windowed acceptance 0.5).  ESS/s = min over the six parameters of bulk-ESS / chain seconds.
    The same code runs the comparison at 10^6 events as a checkpointed campaign (--ess-campaign)."""
    import tempfile

    from paper_2407_11349_amd.mcmc.campaign import Campaign, CampaignConfig, GPUHooks
    from paper_2407_11349_amd.mcmc.cut import HawkesCutTarget

    ev = synth.generate_clustered(n=20_000, seed=1201)
    dev = hk.DeviceEvents.from_arrays(ev.t, ev.x, ev.y, ev.s, device="cuda")
    target = HawkesCutTarget(dev, torch.from_numpy(ev.county).cuda(), torch.from_numpy(ev.rect).cuda(), seed=2201,
                             precision="fp32_skip")
    cfg = CampaignConfig(n_warmup=120, n_plain=400, n_da=400, n_leapfrog=20, seed=7, chunk=100)
    with tempfile.TemporaryDirectory() as d:
        c = Campaign(os.path.join(d, "run"), target, GPUHooks(epochs=30, log=None), cfg, log=lambda m: None)
        phase = c.run()
        s = c.summary()
    if phase != "done":
        raise RuntimeError(f"reduced sampler comparison ended in phase {phase}")
    return {"workload": ev.config.name, "n_events": ev.n,
            "iterations": {"warmup": cfg.n_warmup, "plain_hmc": cfg.n_plain, "da_hmc": cfg.n_da},
            "leapfrog": cfg.n_leapfrog,
            "plain_hmc_ess_per_s": s["plain_hmc"]["ess_per_s"], "da_hmc_ess_per_s": s["da_hmc"]["ess_per_s"],
            "ess_per_s_ratio": s["ess_per_s_ratio"],
            "ess_per_s_ratio_incl_training": s["ess_per_s_ratio_incl_training"],
            "max_mean_diff_in_combined_mcse": s["max_mean_diff_in_combined_mcse"],
            "means_agree_within_3_mcse": s["means_agree_within_3_mcse"], "max_rhat": s["max_rhat"],
            "seconds": s["seconds"],
            "note": "live, reduced: 2e4 events and 400 + 400 iterations; the comparison at 1e6 events "
                    "(2,000 DA-HMC iterations) is a multi-hour campaign checkpointed over several runs "
                    "(bench.py --ess-campaign)"}


def run_campaign(args, hk, synth, torch):
    """The comparison of plain HMC and surrogate DA-HMC at 1e6 events as a resumable campaign: continues the
    run checkpointed in args.ess_campaign until the deadline, saves, and prints the summary so far.  Workload:
    the clustered (branching-process) event set at the shape of the 1e6 benchmark (1200 days, 50 x 60
    counties, LogNormal(5, 1.5) densities), FP32 skip-mode likelihood, 20 leapfrog steps."""
    from paper_2407_11349_amd.mcmc.campaign import Campaign, CampaignConfig, GPUHooks
    from paper_2407_11349_amd.mcmc.cut import HawkesCutTarget

    t_start = time.time()
    ev = synth.generate_clustered(n=args.ess_n, t_max=1200.0, rho_sdlog=1.5, seed=1104)
    log(f"campaign workload {ev.config.name}: {ev.n} events generated in {time.time() - t_start:.1f} s")
    dev = hk.DeviceEvents.from_arrays(ev.t, ev.x, ev.y, ev.s, device="cuda")
    county = torch.from_numpy(ev.county).cuda()
    rect = torch.from_numpy(ev.rect).cuda()
    # replicate r > 0: other random numbers throughout (latent-location draws, chains, surrogate training)
    r = int(args.ess_replicate)
    target = HawkesCutTarget(dev, county, rect, seed=2004 + 100 * r, precision="fp32_skip",
                             workspace_bytes=(args.workspace_mib << 20) if args.workspace_mib else None)
    cfg = CampaignConfig(n_warmup=args.campaign_warmup, n_plain=args.campaign_plain, n_da=args.ess_iter,
                         n_leapfrog=20, seed=1 + r, fallback_prob=args.fallback_prob)
    c = Campaign(args.ess_campaign, target, GPUHooks(seed=5 + r, log=log), cfg, log=log)
    phase = c.run(deadline_s=args.deadline_s)
    out = {"metric": "ESS/s surrogate-HMC vs plain HMC", "unit": "ratio", "higher_is_better": True,
           "data": "synthetic", "phase": phase,
           "config": {"workload": ev.config.name, "n_events": ev.n, "step": "resample X + sampler iteration",
                      "replicate": r, **cfg.__dict__},
           "summary": c.summary()}
    with open(os.path.join(args.ess_campaign, "summary.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: out[k] for k in ("metric", "phase", "config")}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=None, help="override the event count (testing only)")
    ap.add_argument("--workspace-mib", type=int, default=4096,
                    help="FP32 workspace of the timed sweep in MiB (0: hawkes_workspace_bytes); more room means "
                         "fewer passes of the pair sweep, the same results")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-skip", action="store_true", help="do not time the FP32 skip mode")
    ap.add_argument("--no-ess", action="store_true", help="do not run the reduced sampler comparison")
    ap.add_argument("--ess", action="store_true",
                    help="run the surrogate-HMC vs plain-HMC ESS/s comparison instead (minutes of GPU time)")
    ap.add_argument("--ess-n", type=int, default=100_000, help="events of the ESS comparison workload")
    ap.add_argument("--ess-warmup", type=int, default=300)
    ap.add_argument("--ess-burn", type=int, default=1000)
    ap.add_argument("--ess-iter", type=int, default=2000)
    ap.add_argument("--ess-campaign", metavar="DIR", default=None,
                    help="continue the resumable 1e6-event comparison checkpointed in DIR until --deadline-s")
    ap.add_argument("--deadline-s", type=float, default=800.0)
    ap.add_argument("--campaign-warmup", type=int, default=150)
    ap.add_argument("--campaign-plain", type=int, default=600)
    ap.add_argument("--fallback-prob", type=float, default=0.0,
                    help="DA-HMC exact-HMC fallback: 0 = when the windowed acceptance drops below 0.5 (not "
                         "invariant in general), q > 0 = an exact-HMC step with fixed probability q (invariant)")
    ap.add_argument("--ess-replicate", type=int, default=0,
                    help="repeat the comparison with other random numbers (latent draws, chains, training)")
    ap.add_argument("--components", action="store_true",
                    help="only time the smaller steps (latent-location draw, surrogate inference and training)")
    ap.add_argument("--surrogate-fit", action="store_true",
                    help="train the surrogate on ~20,000 burn-in tuples of the 1e5-event workload and report its "
                         "held-out error (a few GPU minutes)")
    ap.add_argument("--fit-burn", type=int, default=952, help="burn-in iterations recorded for --surrogate-fit")
    ap.add_argument("--fit-workload", choices=("n100k", "clustered"), default="n100k",
                    help="event set of --surrogate-fit")
    ap.add_argument("--sampler-costs", type=int, default=0, metavar="N",
                    help="only time the samplers' exact steps on the clustered workload with N events")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES device-to-device (scales the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the pair sweep of one GPU is the measured unit; "
              "splitting target rows across GPUs is a design that this program does not run.", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_probe:
        src = torch.ones(args.copy_probe // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": src.numel() * 4}))
        return

    import synth
    import paper_2407_11349_amd as hk

    if args.ess_campaign:
        run_campaign(args, hk, synth, torch)
        return
    if args.ess:
        run_ess(args, hk, synth, torch)
        return
    if args.surrogate_fit:
        run_surrogate_fit(args, hk, synth, torch)
        return
    if args.sampler_costs:
        sampler_costs(args, hk, synth, torch)
        return

    cfg = synth.N1M
    ev = synth.generate(cfg, n=args.n)
    th = synth.theta_default()
    n = ev.n
    dev = hk.DeviceEvents.from_arrays(ev.t, ev.x, ev.y, ev.s, device="cuda")
    county = torch.from_numpy(ev.county).cuda()
    rect = torch.from_numpy(ev.rect).cuda()
    if args.components:
        print(json.dumps({"workload": cfg.name, "n_events": n,
                          "components": component_timings(hk, torch, county, rect, dev.x, dev.y)}), flush=True)
        return
    ws = hk.Workspace(n, "fp32", nbytes=(args.workspace_mib << 20) if args.workspace_mib else None)
    out_ll = torch.empty(1, dtype=torch.float64, device="cuda")
    out_g = torch.empty(6, dtype=torch.float64, device="cuda")
    seed = 2002
    bg_pairs, causal_pairs = pair_counts(ev.t)
    flop_per_launch = FLOP_BG * bg_pairs + FLOP_TRIG * causal_pairs
    exp_per_launch = bg_pairs + causal_pairs
    # what the symmetric sweep executes: each background term once for the pair (about half of
    # bg_pairs, exactly so without ties) plus its column sums (3 accumulations, FLOP_COL)
    flop_executed = (FLOP_BG + FLOP_COL) * bg_pairs // 2 + FLOP_TRIG * causal_pairs
    exp_executed = bg_pairs // 2 + causal_pairs

    def step(it, timer=None):
        hk.resample_locations(county, rect, seed, it, dev.x, dev.y)
        hk.loglik_grad(dev, th, precision="fp32", ws=ws, out=out_ll, grad=out_g, timer=timer)

    log(f"bench: n={n} warmup={args.warmup} steps={args.steps}")
    for it in range(args.warmup):
        step(it)
        torch.cuda.synchronize()
        log(f"warmup step {it} done: loglik {out_ll.item():.6f}")

    # one pair of caller-owned HIP events per step, recorded by the library around the pair sweep on
    # the step's stream and read after the timed region (no host synchronisation inside it)
    timers = [hk.SweepTimer() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(args.warmup + k, timers[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kernel_ms = [tm.elapsed_ms() for tm in timers]
    log(f"timed {args.steps} steps in {elapsed:.3f} s; pair sweep ms {['%.2f' % v for v in kernel_ms]}")
    ll_last = float(out_ll.item())
    assert np.isfinite(ll_last) and ws.status() == 0

    ms_step = elapsed / args.steps * 1e3
    pairs = n * (n - 1)
    value = pairs / (ms_step / 1e3)
    kms = float(np.mean(kernel_ms))
    achieved = flop_per_launch / (kms / 1e3) / 1e12

    result = {
        "metric": METRIC, "value": value, "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
        "config": {"workload": cfg.name, "n_events": n, "days": cfg.t_max, "counties": cfg.nx * cfg.ny,
                   "rho_sdlog": cfg.rho_sdlog, "step": "resample X + FP32 loglik+grad (FP64 finalize)",
                   "parallelism": "single GPU"},
        "loglik_grad_evals_per_s": 1e3 / ms_step,
        "workspace_bytes": ws.nbytes,
        "roofline": {"bound": "alu", "kernel": "pair sweep of one evaluation (k_pair_f32<grad> passes + k_fold)",
                     "achieved": achieved,
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": measured_traffic(), "kernel_ms": kms, "kernel_source_hash": kernel_source_hash(), "flop_per_launch": flop_per_launch,
                     "exp_per_launch": exp_per_launch, "exp_per_s": exp_per_launch / (kms / 1e3),
                     "executed": {"flop_per_launch": flop_executed, "exp_per_launch": exp_executed,
                                  "achieved": flop_executed / (kms / 1e3) / 1e12,
                                  "frac": flop_executed / (kms / 1e3) / 1e12 / PEAK_FP32_TFLOPS,
                                  "exp_per_s": exp_executed / (kms / 1e3),
                                  "exp_frac_of_measured_exp_peak": exp_executed / (kms / 1e3) / EXP_PEAK_PER_S,
                                  "issue_bound_ms": issue_bound_ms(),
                                  "frac_of_issue_bound": (issue_bound_ms() / kms) if issue_bound_ms() else None,
                                  "note": "FLOP the symmetric sweep performs (each background term "
                                          "once per pair, plus column sums); frac above uses the "
                                          "fixed per-ordered-pair count; issue bound from the SQ "
                                          "instruction counters of this kernel source"}},
    }

    # the same evaluation in the library's default workspace (hawkes_workspace_bytes: under 1 GiB at 1e6
    # events, so more passes of the pair sweep)
    wsd = hk.Workspace(n, "fp32")
    hk.loglik_grad(dev, th, precision="fp32", ws=wsd, out=out_ll, grad=out_g)
    tm = hk.SweepTimer()
    hk.loglik_grad(dev, th, precision="fp32", ws=wsd, out=out_ll, grad=out_g, timer=tm)
    result["default_workspace"] = {"workspace_bytes": wsd.nbytes, "pair_sweep_ms": tm.elapsed_ms(),
                                   "note": "pair sweep time with the default workspace (the timed steps use "
                                           "workspace_bytes above); results are bitwise the same"}
    log(f"default workspace ({wsd.nbytes / 2**20:.0f} MiB): pair sweep {tm.elapsed_ms():.1f} ms")
    del wsd

    if not args.no_fp64:
        ws64 = hk.Workspace(n, "fp64", nbytes=(args.workspace_mib << 20) if args.workspace_mib else None)
        hk.loglik_grad(dev, th, precision="fp64", ws=ws64, out=out_ll, grad=out_g)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        hk.loglik_grad(dev, th, precision="fp64", ws=ws64, out=out_ll, grad=out_g)
        torch.cuda.synchronize()
        d64 = time.perf_counter() - t1
        result["fp64"] = {"value": pairs / d64, "unit": "pairs/s", "ms_per_eval": d64 * 1e3,
                          "fp32_speedup": (pairs / (ms_step / 1e3)) / (pairs / d64),
                          "achieved_tflops": flop_per_launch / d64 / 1e12,
                          "frac_of_fp64_peak": flop_per_launch / d64 / 1e12 / PEAK_FP64_TFLOPS,
                          "note": "same fixed algorithmic FLOP count as the FP32 roofline (exponentials "
                                  "counted apart; each is ~17 FP64 operations here)"}
        log(f"fp64 evaluation: {d64 * 1e3:.1f} ms")
        del ws64

    # the forward-only sweep (log-likelihood without gradient: the exact evaluations of the delayed-acceptance
    # correction); reported apart from the loglik+grad metric
    hk.loglik(dev, th, precision="fp32", ws=ws, out=out_ll)
    tm = hk.SweepTimer()
    hk.loglik(dev, th, precision="fp32", ws=ws, out=out_ll, timer=tm)
    kms_fwd = tm.elapsed_ms()
    torch.cuda.synchronize()
    result["fp32_loglik_only"] = {"kernel_ms": kms_fwd, "pairs_per_s": pairs / (kms_fwd / 1e3),
                                  "note": "forward-only sweep (S0, G0 per target), pair kernel time"}
    log(f"fp32 loglik-only pair kernel: {kms_fwd:.1f} ms")

    # two parameter vectors in one forward-only sweep (the pair geometry formed once for both): the
    # delayed-acceptance correction compares the current and the proposed vector under one draw
    th2 = np.stack([th, th * np.array([1.02, 0.98, 1.03, 0.97, 1.02, 0.98])])
    out2 = torch.empty(2, dtype=torch.float64, device="cuda")
    hk.loglik_batch(dev, th2, precision="fp32", ws=ws, out=out2)
    tm = hk.SweepTimer()
    hk.loglik_batch(dev, th2, precision="fp32", ws=ws, out=out2, timer=tm)
    kms_b2 = tm.elapsed_ms()
    torch.cuda.synchronize()
    result["fp32_loglik_batch2"] = {
        "kernel_ms": kms_b2, "cost_vs_one_vector": kms_b2 / kms_fwd,
        "pairs_per_s": 2 * pairs / (kms_b2 / 1e3),
        "note": "forward-only sweep for two parameter vectors at once; pairs counted once per vector"}
    log(f"fp32 loglik batch of 2 pair kernel: {kms_b2:.1f} ms ({kms_b2 / kms_fwd:.2f} x one vector)")

    if not args.no_skip:
        # the FP32 sweep without the background terms that are exactly zero in FP32 (time gap
        # past ~14.9 tau_t): same result, less work; reported apart from the O(N^2) metric
        wss = hk.Workspace(n, "fp32_skip", nbytes=ws.nbytes)
        ll_s = torch.empty(1, dtype=torch.float64, device="cuda")
        g_s = torch.empty(6, dtype=torch.float64, device="cuda")
        hk.loglik_grad(dev, th, precision="fp32_skip", ws=wss, out=ll_s, grad=g_s)
        hk.loglik_grad(dev, th, precision="fp32", ws=ws, out=out_ll, grad=out_g)
        tm = hk.SweepTimer()
        hk.loglik_grad(dev, th, precision="fp32_skip", ws=wss, out=ll_s, grad=g_s, timer=tm)
        kms_skip = tm.elapsed_ms()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        hk.loglik_grad(dev, th, precision="fp32_skip", ws=wss, out=ll_s, grad=g_s)
        torch.cuda.synchronize()
        dskip = time.perf_counter() - t1
        full_ll, skip_ll = float(out_ll.item()), float(ll_s.item())
        result["fp32_skip"] = {
            "ms_per_eval": dskip * 1e3, "kernel_ms": kms_skip, "speedup_vs_fp32": ms_step / (dskip * 1e3),
            "effective_pairs_per_s": pairs / dskip,
            "loglik_rel_diff_vs_fp32": abs(skip_ll - full_ll) / abs(full_ll),
            "grad_rel_diff_vs_fp32": float(((g_s - out_g).abs() / out_g.abs()).max().item()),
            "note": "pairs whose background term is exactly 0 in FP32 are not swept; not the O(N^2) metric"}
        log(f"fp32_skip evaluation: {dskip * 1e3:.1f} ms (kernel {kms_skip:.1f} ms)")
        del wss

    if n == synth.N1M.n:
        par = parity_vs_stored_oracle(hk, torch, ev, th, ws)
        if par is not None:
            result["parity"] = par
            log(f"parity vs stored oracle: fp32 loglik {par['fp32']['loglik_rel_err']:.2e} grad "
                f"{par['fp32']['grad_rel_err_max']:.2e}; fp64 loglik {par['fp64']['loglik_rel_err']:.2e} grad "
                f"{par['fp64']['grad_rel_err_max']:.2e}")

    comp = component_timings(hk, torch, county, rect, dev.x, dev.y)
    result["components"] = comp
    log(f"resample {comp['resample']['us_per_call']:.1f} us ({comp['resample']['achieved_gbs']:.0f} GB/s); "
        f"mlp forward batch 1 {comp['mlp_forward']['batch1_us']:.1f} us, batch 21000 "
        f"{comp['mlp_forward']['batch21000_ms']:.2f} ms; train step {comp['mlp_train_step']['ms_per_step']:.3f} ms")

    if not args.no_ess:
        log("reduced sampler comparison (2e4 events) ...")
        try:
            result["ess_reduced"] = ess_reduced(hk, synth, torch)
            e = result["ess_reduced"]
            log(f"ESS/s DA-HMC {e['da_hmc_ess_per_s']:.1f} vs plain HMC {e['plain_hmc_ess_per_s']:.1f}: ratio "
                f"{e['ess_per_s_ratio']:.2f}, means within {e['max_mean_diff_in_combined_mcse']:.2f} MCSE")
        except Exception as exc:  # reported in the line; the headline figures above stand on their own
            log(f"reduced sampler comparison failed: {exc!r}")
            result["ess_reduced"] = {"error": repr(exc)}

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(ev, th)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
