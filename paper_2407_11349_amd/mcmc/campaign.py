"""Resumable sampler comparison on the cut posterior: checkpoint/resume of every chain's state.

The paper's chains ran for most of a day each (Section 3.2); the comparison of plain HMC with
surrogate delayed-acceptance HMC at 10^6 events likewise outlasts one process, so it runs as a
sequence of calls that each continue from the last checkpoint until a deadline and write a new
one.  A run split over any number of calls takes exactly the steps of an uninterrupted run:
every random-number generator, adaptation state, chain draw, surrogate weight and training
tuple is saved, and the latent-location draw of an iteration is a pure function of its global
index (Philox counter).

Phases (each resumable at any iteration boundary):
  mode     the highest posterior mode under draw 0 (hooks.find_mode),
  warmup   exact HMC, step size by dual averaging and a diagonal mass from the warm-up draws,
  plain    exact HMC with fixed step size (jittered per iteration) and mass: the plain chain
           of the comparison; every gradient evaluation's (log theta, l, dl/dlog theta, draw)
           tuple is kept as training data for the surrogate,
  train    the surrogate trained on the tuples (hooks.train; whole draws held out),
  da       delayed-acceptance HMC from the plain chain's end point with the trained surrogate,
  done     both chains finished; summary() gives ESS/s and the equal-accuracy checks.

Every iteration appends one JSON line (phase, index, draw index, position, log density when
known, acceptance, step size, elapsed seconds) to the run's log.
"""

from __future__ import annotations

import json
import os
import time
from collections import deque
from dataclasses import asdict, dataclass

import numpy as np

from .da_hmc import DAState, DelayedAcceptanceHMC
from .ess import bulk_ess, mcse_mean, split_rhat
from .hmc import HMC, DualAveraging

PHASES = ("mode", "warmup", "plain", "train", "da", "done")


@dataclass
class CampaignConfig:
    n_warmup: int = 150
    n_plain: int = 600
    n_da: int = 2000
    n_leapfrog: int = 20
    jitter: float = 0.2       # step-size jitter of both compared chains after warm-up
    seed: int = 1
    chunk: int = 10           # iterations between checkpoints
    init_eps: float = 0.01
    init_inv_mass: float = 1e-4
    fallback_prob: float = 0.0  # 0: the windowed-acceptance fallback; q > 0: exact HMC with probability q


def _sync():
    try:
        import torch

        if torch.cuda.is_initialized():
            torch.cuda.synchronize()
    except ImportError:
        pass


# ----------------------------------------------------------------------------- checkpoint files

def save_state(path: str, state: dict) -> None:
    """state: JSON-able scalars and lists under 'meta', NumPy arrays under 'arrays'.  Written to
    temporary files and renamed, so an interrupted save leaves the previous checkpoint intact."""
    os.makedirs(path, exist_ok=True)
    arrays = {k: np.asarray(v) for k, v in state["arrays"].items()}
    tmp_npz = os.path.join(path, "state.tmp.npz")
    np.savez(tmp_npz, **arrays)
    tmp_json = os.path.join(path, "state.tmp.json")
    with open(tmp_json, "w") as f:
        json.dump(state["meta"], f)
    os.replace(tmp_npz, os.path.join(path, "state.npz"))
    os.replace(tmp_json, os.path.join(path, "state.json"))


def load_state(path: str) -> dict | None:
    j, z = os.path.join(path, "state.json"), os.path.join(path, "state.npz")
    if not (os.path.exists(j) and os.path.exists(z)):
        return None
    with open(j) as f:
        meta = json.load(f)
    with np.load(z, allow_pickle=False) as d:
        arrays = {k: d[k].copy() for k in d.files}
    if "_version" not in arrays or int(arrays.pop("_version")) != meta.get("version"):
        raise RuntimeError(f"checkpoint {path}: state.json and state.npz are from different saves")
    return {"meta": meta, "arrays": arrays}


def _rng_state(rng: np.random.Generator) -> dict:
    st = rng.bit_generator.state
    return json.loads(json.dumps(st, default=int))


def _rng_from(state: dict) -> np.random.Generator:
    bg = getattr(np.random, state["bit_generator"])()
    bg.state = state
    return np.random.Generator(bg)


# ----------------------------------------------------------------------------- the driver

class Campaign:
    """One comparison run bound to a checkpoint directory.  `target` is a cut-posterior target
    (HawkesCutTarget or an equivalent with resample / logp / logp_batch / logp_and_grad /
    _prior / prior_var); `hooks` supplies find_mode(target, z0), train(Z, L, G, groups) ->
    (arrays, info) and surrogate(arrays) -> an object with value_and_grad (and optionally
    leapfrog)."""

    def __init__(self, ckpt_dir: str, target, hooks, config: CampaignConfig | None = None, z0=None, log=None):
        self.dir = ckpt_dir
        self.target = target
        self.hooks = hooks
        self.log = log
        st = load_state(ckpt_dir)
        if st is None:
            cfg = config or CampaignConfig()
            z0 = np.log(np.array([0.5, 10.0, 7.0, 0.3, 2.0, 0.2])) if z0 is None else np.asarray(z0, np.float64)
            self.meta = {"version": 0, "phase": "mode", "config": asdict(cfg), "k": 0, "it": 0,
                         "seconds": {p: 0.0 for p in PHASES}, "counts": {}, "info": {}}
            self.arrays = {"z": z0.copy()}
        else:
            self.meta, self.arrays = st["meta"], st["arrays"]
            # a field added to CampaignConfig after the checkpoint was written takes its default
            self.meta["config"] = {**asdict(CampaignConfig()), **self.meta["config"]}
            if config is not None and asdict(config) != self.meta["config"]:
                raise ValueError("the checkpoint was written with another configuration")
            # iterations logged after the last save are run again: drop their lines
            log_path = os.path.join(ckpt_dir, "iterations.jsonl")
            saved = self.meta.get("log_bytes")
            if saved is not None and os.path.exists(log_path) and os.path.getsize(log_path) > saved:
                with open(log_path, "r+b") as f:
                    f.truncate(saved)
        self.cfg = CampaignConfig(**self.meta["config"])
        self._sur = None

    # -- bookkeeping
    @property
    def phase(self) -> str:
        return self.meta["phase"]

    def _save(self):
        log_path = os.path.join(self.dir, "iterations.jsonl")
        self.meta["log_bytes"] = os.path.getsize(log_path) if os.path.exists(log_path) else 0
        self.meta["version"] += 1
        save_state(self.dir, {"meta": self.meta, "arrays": {**self.arrays, "_version": self.meta["version"]}})

    def _jsonl(self, rec: dict):
        with open(os.path.join(self.dir, "iterations.jsonl"), "a") as f:
            f.write(json.dumps(rec) + "\n")

    def _next_phase(self):
        self.meta["phase"] = PHASES[PHASES.index(self.phase) + 1]
        self.meta["it"] = 0

    def _append(self, name, row):
        row = np.asarray(row, dtype=np.float64)[None, ...]
        self.arrays[name] = row if name not in self.arrays else np.concatenate([self.arrays[name], row])

    # -- phases
    def _hmc(self, jitter=0.0):
        m = self.meta
        hmc = HMC(self.target, n_leapfrog=self.cfg.n_leapfrog, step_size=m["eps"],
                  inv_mass=self.arrays["inv_mass"], rng=_rng_from(m["rng"]), jitter=jitter)
        return hmc

    def _run_mode(self):
        self.target.resample(0)
        t0 = time.time()
        z = self.hooks.find_mode(self.target, self.arrays["z"])
        self.meta["seconds"]["mode"] += time.time() - t0
        self.arrays["z"] = np.asarray(z, dtype=np.float64)
        self.meta["eps"] = self.cfg.init_eps
        self.arrays["inv_mass"] = np.full(6, self.cfg.init_inv_mass)
        self.meta["rng"] = _rng_state(np.random.default_rng(self.cfg.seed))
        self.meta["da_state"] = {"mu": None, "hbar": 0.0, "log_eps_bar": 0.0, "t": 0,
                                 "log_eps0": float(np.log(self.cfg.init_eps))}
        self.meta["k"] = 1
        self._next_phase()

    def _dual_averaging(self) -> DualAveraging:
        d = self.meta["da_state"]
        da = DualAveraging(d["log_eps0"], target=0.8)
        if d["mu"] is not None:
            da.mu, da.hbar, da.log_eps_bar, da.t = d["mu"], d["hbar"], d["log_eps_bar"], d["t"]
        return da

    def _store_dual_averaging(self, da: DualAveraging):
        self.meta["da_state"] = {"mu": da.mu, "hbar": da.hbar, "log_eps_bar": da.log_eps_bar, "t": da.t,
                                 "log_eps0": self.meta["da_state"]["log_eps0"]}

    def _run_warmup(self, n_iter):
        """As the warm-up of experiment.burn_in: dual averaging towards acceptance 0.8, the mass from
        the second quarter of the draws at mid warm-up, dual averaging restarted there."""
        hmc = self._hmc()
        da = self._dual_averaging()
        half = self.cfg.n_warmup // 2
        _sync()
        t0 = time.time()
        for _ in range(n_iter):
            it, k = self.meta["it"], self.meta["k"]
            self.target.resample(k)
            s = hmc.init_state(self.arrays["z"])
            s, acc, a = hmc.step(s)
            hmc.eps = da.update(a)
            self._append("warm_draws", s.z)
            if it + 1 == half and half >= 20:
                w = self.arrays["warm_draws"][half // 2:]
                var = w.var(axis=0)
                if np.all(var > 0):
                    hmc.inv_mass = var
                da = DualAveraging(np.log(hmc.eps), target=0.8)
                self.meta["da_state"]["log_eps0"] = float(np.log(hmc.eps))
            self.arrays["z"] = s.z
            self._jsonl({"phase": "warmup", "it": it, "k": k, "z": s.z.tolist(), "logp": s.logp, "accepted": acc,
                         "accept_prob": a, "eps": hmc.eps, "t": time.time() - t0})
            self.meta["it"] += 1
            self.meta["k"] += 1
            if self.meta["it"] == self.cfg.n_warmup:
                hmc.eps = da.final()
                break
        _sync()
        self.meta["seconds"]["warmup"] += time.time() - t0
        self.meta["eps"] = float(hmc.eps)
        self.arrays["inv_mass"] = np.asarray(hmc.inv_mass, dtype=np.float64)
        self.meta["rng"] = _rng_state(hmc.rng)
        self._store_dual_averaging(da)
        if self.meta["it"] == self.cfg.n_warmup:
            self.meta["rng"] = _rng_state(np.random.default_rng(self.cfg.seed + 1000))
            self._next_phase()

    def _run_plain(self, n_iter):
        hmc = self._hmc(jitter=self.cfg.jitter)
        rec = _Recorder(self.target, self)
        hmc.target = rec
        c = self.meta["counts"].setdefault("plain", {"accept": 0, "n_grad": 0})
        _sync()
        t0 = time.time()
        for _ in range(n_iter):
            it, k = self.meta["it"], self.meta["k"]
            self.target.resample(k)
            rec.group = k
            s = hmc.init_state(self.arrays["z"])
            s, acc, a = hmc.step(s)
            c["accept"] += int(acc)
            self.arrays["z"] = s.z
            self._append("plain_draws", s.z)
            self._jsonl({"phase": "plain", "it": it, "k": k, "z": s.z.tolist(), "logp": s.logp, "accepted": acc,
                         "accept_prob": a, "eps": hmc.eps, "t": time.time() - t0})
            self.meta["it"] += 1
            self.meta["k"] += 1
            if self.meta["it"] == self.cfg.n_plain:
                break
        _sync()
        self.meta["seconds"]["plain"] += time.time() - t0
        c["n_grad"] += rec.count
        rec.flush()
        self.meta["rng"] = _rng_state(hmc.rng)
        if self.meta["it"] == self.cfg.n_plain:
            self._next_phase()

    def _run_train(self):
        a = self.arrays
        _sync()
        t0 = time.time()
        sur_arrays, info = self.hooks.train(a["tuples_z"], a["tuples_ll"], a["tuples_g"],
                                            a["tuples_group"].astype(np.int64))
        _sync()
        self.meta["seconds"]["train"] += time.time() - t0
        for name, v in sur_arrays.items():
            self.arrays["sur_" + name] = np.asarray(v)
        self.meta["info"]["surrogate"] = info
        self.meta["rng"] = _rng_state(np.random.default_rng(self.cfg.seed + 2000))
        self.meta["da"] = {"window": [], "stats": None}
        self._next_phase()

    def surrogate(self):
        if self._sur is None:
            sa = {k[4:]: v for k, v in self.arrays.items() if k.startswith("sur_")}
            self._sur = self.hooks.surrogate(sa)
        return self._sur

    def _da_sampler(self):
        sur = self.surrogate()
        pv = self.target.prior_var

        def sur_post(z):
            ll, g = sur.value_and_grad(z)
            return float(ll[0]) - 0.5 * float(np.dot(z, z)) / pv, g[0] - np.asarray(z) / pv

        traj = None
        if hasattr(sur, "leapfrog"):
            def traj(z, p, grad, eps, inv_mass, n):
                return sur.leapfrog(z, p, grad, eps, inv_mass, n, pv)
        da = DelayedAcceptanceHMC(self.target, sur_post, n_leapfrog=self.cfg.n_leapfrog, step_size=self.meta["eps"],
                                  inv_mass=self.arrays["inv_mass"], rng=_rng_from(self.meta["rng"]),
                                  trajectory=traj, jitter=self.cfg.jitter, fallback_prob=self.cfg.fallback_prob)
        d = self.meta["da"]
        da.window = deque(d["window"], maxlen=da.window.maxlen)
        if d["stats"] is not None:
            da.stats = dict(d["stats"])
        return da, sur_post

    def _run_da(self, n_iter):
        da, sur_post = self._da_sampler()
        n0 = self.target.n_loglik
        g0 = self.target.n_grad
        _sync()
        t0 = time.time()
        z = self.arrays["z"]
        if self.meta["it"] == 0:
            self.target.resample(self.meta["k"])
            st = da.init_state(z)
        else:
            # an iteration boundary: the current point's exact value under the new draw is computed when
            # a proposal next reaches stage 2; its surrogate value and gradient are the saved ones
            self.target.resample(self.meta["k"])
            st = DAState(z, None, float(self.arrays["da_s"]), self.arrays["da_sg"].copy())
        for _ in range(n_iter):
            it = self.meta["it"]
            st, acc, stage = da.step(st)
            self.arrays["z"] = st.z
            self._append("da_draws", st.z)
            self._jsonl({"phase": "da", "it": it, "k": self.meta["k"], "z": st.z.tolist(), "logp": st.logp,
                         "accepted": acc, "stage": stage, "eps": da.eps, "t": time.time() - t0})
            self.meta["it"] += 1
            self.meta["k"] += 1
            if self.meta["it"] == self.cfg.n_da:
                break
            self.target.resample(self.meta["k"])
            st = da.refresh_exact(st)
        _sync()
        self.meta["seconds"]["da"] += time.time() - t0
        c = self.meta["counts"].setdefault("da", {"n_loglik": 0, "n_grad": 0})
        c["n_loglik"] += self.target.n_loglik - n0
        c["n_grad"] += self.target.n_grad - g0
        self.meta["rng"] = _rng_state(da.rng)
        self.meta["da"] = {"window": list(da.window), "stats": dict(da.stats)}
        self.arrays["da_s"] = np.array(st.s, dtype=np.float64)
        self.arrays["da_sg"] = np.asarray(st.s_grad, dtype=np.float64)
        if self.meta["it"] == self.cfg.n_da:
            self._next_phase()

    # -- entry points
    def run(self, deadline_s: float | None = None, max_chunks: int | None = None) -> str:
        """Continues from the checkpoint in chunks of `chunk` iterations, saving after each, until
        the deadline (seconds from now), max_chunks chunks, or the end.  Returns the phase reached."""
        t_end = None if deadline_s is None else time.time() + deadline_s
        chunks = 0
        while self.phase != "done":
            if (t_end is not None and time.time() >= t_end) or (max_chunks is not None and chunks >= max_chunks):
                break
            ph = self.phase
            if ph == "mode":
                self._run_mode()
            elif ph == "warmup":
                self._run_warmup(self.cfg.chunk)
            elif ph == "plain":
                self._run_plain(self.cfg.chunk)
            elif ph == "train":
                self._run_train()
            elif ph == "da":
                self._run_da(self.cfg.chunk)
            self._save()
            chunks += 1
            if self.log:
                self.log(f"campaign: phase {ph} -> {self.phase}, iteration {self.meta['it']}, draw {self.meta['k']}")
        return self.phase

    def summary(self) -> dict:
        """ESS/s of both chains (min over the six parameters of bulk-ESS / chain seconds; DA also with
        its training time), split R-hat, and whether the posterior means agree within 3 combined MCSE."""
        out = {"config": self.meta["config"], "phase": self.phase, "seconds": self.meta["seconds"],
               "counts": self.meta["counts"], "surrogate": self.meta["info"].get("surrogate")}
        res = {}
        for name, key in (("plain_hmc", "plain_draws"), ("da_hmc", "da_draws")):
            if key not in self.arrays:
                continue
            d = self.arrays[key]
            secs = self.meta["seconds"]["plain" if name == "plain_hmc" else "da"]
            ess = [bulk_ess(d[:, i][None, :]) for i in range(d.shape[1])]
            res[name] = {"iterations": int(d.shape[0]), "seconds": secs, "mean": d.mean(axis=0).tolist(),
                         "mcse": [mcse_mean(d[:, i][None, :]) for i in range(d.shape[1])], "bulk_ess": ess,
                         "rhat": [split_rhat(d[:, i][None, :]) for i in range(d.shape[1])],
                         "min_bulk_ess": float(min(ess)), "ess_per_s": float(min(ess)) / max(secs, 1e-9)}
        out.update(res)
        if "da_hmc" in res:
            res["da_hmc"]["ess_per_s_incl_training"] = res["da_hmc"]["min_bulk_ess"] / (
                res["da_hmc"]["seconds"] + self.meta["seconds"]["train"])
            res["da_hmc"]["stats"] = self.meta["da"]["stats"]
        if "plain_hmc" in res and "da_hmc" in res:
            mp, md = np.array(res["plain_hmc"]["mean"]), np.array(res["da_hmc"]["mean"])
            se = np.sqrt(np.array(res["plain_hmc"]["mcse"]) ** 2 + np.array(res["da_hmc"]["mcse"]) ** 2)
            out["max_mean_diff_in_combined_mcse"] = float(np.max(np.abs(mp - md) / se))
            out["means_agree_within_3_mcse"] = bool(np.all(np.abs(mp - md) <= 3 * se))
            out["max_rhat"] = float(max(max(res["plain_hmc"]["rhat"]), max(res["da_hmc"]["rhat"])))
            out["ess_per_s_ratio"] = res["da_hmc"]["ess_per_s"] / res["plain_hmc"]["ess_per_s"]
            out["ess_per_s_ratio_incl_training"] = (res["da_hmc"]["ess_per_s_incl_training"]
                                                    / res["plain_hmc"]["ess_per_s"])
        return out


class _Recorder:
    """Target wrapper of the plain chain: every finite gradient evaluation's tuple (z, l, dl/dz, draw)
    is kept and appended to the campaign's arrays at flush()."""

    def __init__(self, target, campaign: Campaign):
        self.t = target
        self.c = campaign
        self.group = 0
        self.rows = []
        self.count = 0

    @property
    def prior_var(self):
        return self.t.prior_var

    def logp(self, z):
        return self.t.logp(z)

    def logp_and_grad(self, z):
        lp, g = self.t.logp_and_grad(z)
        self.count += 1
        if np.isfinite(lp):
            z = np.asarray(z, dtype=np.float64)
            plp, pg = self.t._prior(z)
            self.rows.append((z.copy(), lp - plp, np.asarray(g) - pg, self.group))
        return lp, g

    def flush(self):
        if not self.rows:
            return
        a = self.c.arrays
        for name, col in (("tuples_z", 0), ("tuples_ll", 1), ("tuples_g", 2), ("tuples_group", 3)):
            v = np.array([r[col] for r in self.rows], dtype=np.float64)
            a[name] = v if name not in a else np.concatenate([a[name], v])
        self.rows = []


# ----------------------------------------------------------------------------- GPU hooks

class GPUHooks:
    """The mode search of the experiment module, the HIP-trained BF16 surrogate (whole draws held out,
    values fitted up to one offset per draw), and the surrogate rebuilt from its saved weights."""

    def __init__(self, lam=1.0, epochs=60, seed=5, log=None):
        self.lam, self.epochs, self.seed, self.log = lam, epochs, seed, log

    def find_mode(self, target, z0):
        from .experiment import best_mode

        return best_mode(target, z0, log=self.log)

    def train(self, Z, L, G, groups):
        from synth.mlp_init import init_params

        from ..surrogate import Standardiser, Surrogate, SurrogateNet, group_means, train

        rng = np.random.default_rng(7)
        ids = np.unique(groups)
        held = rng.permutation(ids)[: max(1, ids.shape[0] // 10)]
        is_te = np.isin(groups, held)
        tr, te = np.nonzero(~is_te)[0], np.nonzero(is_te)[0]
        remap = {g: i for i, g in enumerate(np.unique(groups[tr]))}
        gtr = np.array([remap[g] for g in groups[tr]], dtype=np.int64)
        std = Standardiser.fit(Z[tr], L[tr], gtr)
        net = SurrogateNet(init_params(3))
        hist = train(net, std, Z[tr], L[tr], G[tr], lam=self.lam, epochs=self.epochs, batch=256, lr=1e-3,
                     seed=self.seed, log=self.log, groups=gtr)
        sur = Surrogate(net, std)
        yh, gh = sur.value_and_grad(Z[te])
        gte = np.unique(groups[te], return_inverse=True)[1]
        err = yh - L[te]
        err_c = err - group_means(err, gte)[gte]
        spread_c = L[te] - group_means(L[te], gte)[gte]
        info = {"tuples": int(Z.shape[0]), "train_tuples": int(tr.shape[0]), "held_out_tuples": int(te.shape[0]),
                "held_out_draws": int(held.shape[0]), "final_loss": hist[-1],
                "loglik_rmse_within_draw": float(np.sqrt(np.mean(err_c ** 2))),
                "loglik_spread_within_draw": float(np.sqrt(np.mean(spread_c ** 2))),
                "grad_rel_rmse": float(np.sqrt(np.mean((gh - G[te]) ** 2)) / np.sqrt(np.mean(G[te] ** 2)))}
        arrays = {"params": net.params().cpu().numpy(), "m_z": std.m_z, "s_z": std.s_z,
                  "m_y": np.array(std.m_y), "s_y": np.array(std.s_y)}
        return arrays, info

    def surrogate(self, a):
        from ..surrogate import Standardiser, Surrogate, SurrogateNet

        std = Standardiser(np.asarray(a["m_z"]), np.asarray(a["s_z"]), float(a["m_y"]), float(a["s_y"]))
        return Surrogate(SurrogateNet(a["params"]), std)
