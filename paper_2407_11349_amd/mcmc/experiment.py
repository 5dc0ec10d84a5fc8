"""Surrogate training from HMC burn-in and the ESS/s comparison of plain HMC
with surrogate delayed-acceptance HMC, on the cut posterior with the GPU
likelihood (latent locations redrawn every iteration).

Pipeline:
  1. exact-HMC burn-in: a mode search, a warm-up that adapts the step size and
     a diagonal mass, then fixed-parameter iterations in which every leapfrog
     point's (log theta, l, d l / d log theta) tuple is recorded;
  2. the surrogate is trained on the tuples (90/10 split) with the Sobolev
     loss, by the HIP train kernels; held-out errors are reported;
  3. from the burn-in end state, plain HMC and DA-HMC run the same number of
     iterations; ESS/s = min over the six parameters of bulk-ESS / wall
     seconds, reported with and without the surrogate's training cost.
"""

from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np
import torch

from .cut import HawkesCutTarget
from .da_hmc import DelayedAcceptanceHMC
from .ess import bulk_ess, mcse_mean, split_rhat
from .hmc import HMC, DualAveraging
from ..surrogate import Standardiser, Surrogate, SurrogateNet, group_means, train


def _sync():
    """Waits for queued GPU work, so wall-clock intervals cover it (no-op before any GPU use)."""
    if torch.cuda.is_initialized():
        torch.cuda.synchronize()


class RecordingTarget:
    """Wraps a target and records (z, loglik, grad loglik wrt z) at every gradient evaluation."""

    def __init__(self, target: HawkesCutTarget):
        self.t = target
        self.z, self.ll, self.g, self.grp = [], [], [], []
        self.group = 0  # id of the current latent-location draw

    def logp(self, z):
        return self.t.logp(z)

    def logp_and_grad(self, z):
        lp, g = self.t.logp_and_grad(z)
        if np.isfinite(lp):
            z = np.asarray(z, dtype=np.float64)
            prior_lp, prior_g = self.t._prior(z)
            self.z.append(z.copy())
            self.ll.append(lp - prior_lp)
            self.g.append(g - prior_g)
            self.grp.append(self.group)
        return lp, g


@dataclass
class ChainResult:
    draws: np.ndarray
    seconds: float
    n_loglik: int
    n_grad: int
    stats: dict


def _summary(draws: np.ndarray) -> dict:
    return {
        "mean": draws.mean(axis=0).tolist(),
        "mcse": [mcse_mean(draws[:, i][None, :]) for i in range(draws.shape[1])],
        "bulk_ess": [bulk_ess(draws[:, i][None, :]) for i in range(draws.shape[1])],
        "rhat": [split_rhat(draws[:, i][None, :]) for i in range(draws.shape[1])],
    }


def find_mode(target, z0, max_iter: int = 200) -> np.ndarray:
    """Posterior mode under the current latent locations (L-BFGS on the exact log density and
    gradient): the chains start there instead of spending burn-in on the approach."""
    from scipy.optimize import minimize

    def f(z):
        lp, g = target.logp_and_grad(z)
        if not np.isfinite(lp):
            return 1e300, np.zeros_like(z)
        return -lp, -np.asarray(g)

    res = minimize(f, np.asarray(z0, dtype=np.float64), jac=True, method="L-BFGS-B",
                   options={"maxiter": max_iter})
    return np.asarray(res.x, dtype=np.float64)


# Extra starts of the mode search, as offsets of log theta from z0: the two kernels can trade
# roles (a long-memory, wide triggering kernel with a narrow background, or the reverse),
# and the mode nearest to the usual starting values need not be the highest.
# step-size jitter of the compared HMC samplers (plain and delayed acceptance) after warm-up
STEP_JITTER = 0.2

# further starts of the mode search, as offsets of log theta from the default: a long-memory triggering kernel
# (two of them), and a wider, stronger one
MODE_START_OFFSETS = ([0.0, 0.0, 0.0, -0.5, 0.0, -4.0], [0.0, 0.0, 0.0, -0.8, 1.0, -5.0],
                      [0.0, 0.0, 0.0, 0.7, 1.8, 0.0])


def best_mode(target, z0, offsets=MODE_START_OFFSETS, log=None) -> np.ndarray:
    """The highest of the modes found from z0 and from z0 + each offset."""
    best, best_lp = None, -np.inf
    for off in ([0.0] * len(z0),) + tuple(offsets):
        zm = find_mode(target, np.asarray(z0, dtype=np.float64) + np.asarray(off))
        lp = target.logp(zm)
        if log:
            log(f"mode from offset {off}: z {np.round(zm, 4)} logp {lp:.3f}")
        if lp > best_lp:
            best, best_lp = zm, lp
    return best


def burn_in(target: HawkesCutTarget, z0, n_iter: int, n_leapfrog=20, seed=0, n_warmup=300, log=None):
    """Exact HMC on the cut posterior in three phases: a mode search (the highest mode from
    several starts); n_warmup iterations that tune the step size (dual averaging) and a
    diagonal mass (variance of the second quarter of the warm-up draws); then n_iter
    iterations with both fixed, in which every gradient evaluation's tuple is recorded
    (n_iter (n_leapfrog + 1) tuples)."""
    t0 = time.time()
    target.resample(0)
    z = best_mode(target, z0, log=log)
    if log:
        log(f"mode search: z {np.round(z, 4)}")
    hmc = HMC(target, n_leapfrog=n_leapfrog, step_size=0.01, inv_mass=np.full(len(z), 1e-4),
              rng=np.random.default_rng(seed))
    s = hmc.init_state(z)
    da = DualAveraging(np.log(hmc.eps), target=0.8)
    draws = []
    half = n_warmup // 2
    for it in range(n_warmup):
        s, _, a = hmc.step(s)
        hmc.eps = da.update(a)
        draws.append(s.z.copy())
        if it + 1 == half and half >= 20:
            var = np.array(draws[half // 2:]).var(axis=0)
            if np.all(var > 0):
                hmc.inv_mass = var
            da = DualAveraging(np.log(hmc.eps), target=0.8)
        # cut posterior: a new X draw, then the exact density and gradient under it
        target.resample(it + 1)
        s = hmc.init_state(s.z)
        if log and (it + 1) % 100 == 0:
            log(f"warm-up {it + 1}/{n_warmup}: eps {hmc.eps:.3g} z {np.round(s.z, 4)}")
    hmc.eps = da.final()
    rec = RecordingTarget(target)
    hmc.target = rec
    s = hmc.init_state(s.z)
    acc = 0
    for it in range(n_iter):
        s, a, _ = hmc.step(s)
        acc += a
        target.resample(n_warmup + it + 1)
        rec.group += 1
        s = hmc.init_state(s.z)
        if log and (it + 1) % 100 == 0:
            log(f"burn-in {it + 1}/{n_iter}: accept {acc / (it + 1):.2f} z {np.round(s.z, 4)}")
    hmc.target = target
    return hmc, s, rec, time.time() - t0


def run_plain_hmc(target: HawkesCutTarget, hmc: HMC, z0, n_iter: int, it0: int, log=None) -> ChainResult:
    hmc.jitter = STEP_JITTER
    n0, g0 = target.n_loglik, target.n_grad
    _sync()
    t0 = time.time()
    target.resample(it0)
    s = hmc.init_state(z0)
    draws = []
    acc = 0
    for it in range(n_iter):
        s, a, _ = hmc.step(s)
        acc += a
        draws.append(s.z.copy())
        target.resample(it0 + it + 1)
        s = hmc.init_state(s.z)
        if log and (it + 1) % 200 == 0:
            log(f"hmc {it + 1}/{n_iter}: accept {acc / (it + 1):.2f} z {np.round(s.z, 4)}")
    _sync()
    return ChainResult(np.array(draws), time.time() - t0, target.n_loglik - n0, target.n_grad - g0,
                       {"accept": acc / n_iter})


def run_mh(target: HawkesCutTarget, z0, inv_mass, n_iter: int, it0: int, n_adapt=200, seed=13,
           log=None) -> ChainResult:
    """The paper's kernel: univariate random-walk MH sweeps (6 proposals, forward-only exact
    densities), each after a fresh latent-location draw.  Proposal scales start at 2.4 posterior
    sd (from the HMC warm-up) and adapt over n_adapt untimed sweeps with a diminishing rate."""
    from .mh import UnivariateMH

    mh = UnivariateMH(target, scales=2.4 * np.sqrt(np.asarray(inv_mass)), rng=np.random.default_rng(seed))
    z = np.asarray(z0, dtype=np.float64)
    for it in range(n_adapt):
        target.resample(it0 + it)
        z, _ = mh.sweep(z, None, adapt_rate=0.5 / np.sqrt(it + 1.0))
    mh.accepts[:] = 0
    mh.tries[:] = 0
    n0, g0 = target.n_loglik, target.n_grad
    _sync()
    t0 = time.time()
    draws = []
    for it in range(n_iter):
        target.resample(it0 + n_adapt + it)
        z, _ = mh.sweep(z)  # the current point's density under the new draw, paired with the first proposal
        draws.append(z.copy())
        if log and (it + 1) % 500 == 0:
            log(f"mh {it + 1}/{n_iter}: acceptance {np.round(mh.acceptance(), 2)}")
    _sync()
    return ChainResult(np.array(draws), time.time() - t0, target.n_loglik - n0, target.n_grad - g0,
                       {"acceptance": mh.acceptance().tolist(), "scales": mh.scales.tolist()})


def run_da_hmc(target: HawkesCutTarget, sur: Surrogate, hmc: HMC, z0, n_iter: int, it0: int, prior_var: float,
               log=None, seed=11, fallback_prob=0.0) -> ChainResult:
    def sur_post(z):
        ll, g = sur.value_and_grad(z)
        return float(ll[0]) - 0.5 * float(np.dot(z, z)) / prior_var, g[0] - np.asarray(z) / prior_var

    def trajectory(z, p, grad, eps, inv_mass, n):
        return sur.leapfrog(z, p, grad, eps, inv_mass, n, prior_var)

    da = DelayedAcceptanceHMC(target, sur_post, n_leapfrog=hmc.n_leapfrog, step_size=hmc.eps,
                              inv_mass=hmc.inv_mass, rng=np.random.default_rng(seed),
                              trajectory=trajectory if hasattr(sur, "leapfrog") else None, jitter=STEP_JITTER,
                              fallback_prob=fallback_prob)
    n0, g0 = target.n_loglik, target.n_grad
    _sync()
    t0 = time.time()
    target.resample(it0)
    st = da.init_state(z0)
    draws = []
    for it in range(n_iter):
        st, _, _ = da.step(st)
        draws.append(st.z.copy())
        target.resample(it0 + it + 1)
        st = da.refresh_exact(st)
        if log and (it + 1) % 200 == 0:
            log(f"da-hmc {it + 1}/{n_iter}: {da.stats}")
    _sync()
    return ChainResult(np.array(draws), time.time() - t0, target.n_loglik - n0, target.n_grad - g0, dict(da.stats))


def fit_surrogate(rec: "RecordingTarget", lam=1.0, epochs=60, seed=5, log=None):
    """Trains the surrogate on the recorded (log theta, l, dl/dlog theta, draw) tuples of a burn-in, with 10% of
    the latent-location draws held out whole; returns the surrogate and its held-out errors.  A draw shifts l by
    an offset the surrogate does not model, so the value error is measured within each held-out draw, after
    removing that draw's mean error (the value term of the loss is fitted up to one offset per draw too)."""
    from synth.mlp_init import init_params

    Zt, Lt, Gt, Ht = np.array(rec.z), np.array(rec.ll), np.array(rec.g), np.array(rec.grp, dtype=np.int64)
    n = Zt.shape[0]
    rng = np.random.default_rng(7)
    n_groups = int(Ht.max()) + 1
    held_groups = rng.permutation(n_groups)[: max(1, n_groups // 10)]
    is_te = np.isin(Ht, held_groups)
    tr, te = np.nonzero(~is_te)[0], np.nonzero(is_te)[0]
    remap = np.full(n_groups, -1, dtype=np.int64)
    remap[np.unique(Ht[tr])] = np.arange(np.unique(Ht[tr]).shape[0])
    std = Standardiser.fit(Zt[tr], Lt[tr], remap[Ht[tr]])
    t0 = time.time()
    net = SurrogateNet(init_params(3))
    hist = train(net, std, Zt[tr], Lt[tr], Gt[tr], lam=lam, epochs=epochs, batch=256, lr=1e-3, seed=seed, log=log,
                 groups=remap[Ht[tr]])
    _sync()
    t_train = time.time() - t0
    sur = Surrogate(net, std)
    yh, gh = sur.value_and_grad(Zt[te])
    err = yh - Lt[te]
    gte = Ht[te]
    err_c = err - group_means(err, gte)[gte]
    spread_c = Lt[te] - group_means(Lt[te], gte)[gte]
    held = {"tuples": int(n), "draws": n_groups, "held_out_draws": int(held_groups.shape[0]),
            "held_out_tuples": int(te.shape[0]), "train_seconds": t_train, "epochs": epochs, "final_loss": hist[-1],
            "loglik_rmse_within_draw": float(np.sqrt(np.mean(err_c ** 2))),
            "loglik_spread_within_draw": float(np.sqrt(np.mean(spread_c ** 2))),
            "loglik_spread_across_draws": float(Lt[te].std()),
            "loglik_rel_err_rms": float(np.sqrt(np.mean((err_c / Lt[te]) ** 2))),
            "grad_rel_rmse": float(np.sqrt(np.mean((gh - Gt[te]) ** 2)) / np.sqrt(np.mean(Gt[te] ** 2)))}
    if log:
        log(f"surrogate: {held}")
    return sur, held


def surrogate_fit(events, county, rect, *, n_burn=952, n_leapfrog=20, seed=2002, lam=1.0, epochs=60, n_warmup=300,
                  log=None) -> dict:
    """Surrogate training on one event set: exact-HMC burn-in on the cut posterior recording n_burn (n_leapfrog + 1)
    tuples (952 x 21 = 19,992), then fit_surrogate; returns the held-out errors and the burn-in and training
    times."""
    target = HawkesCutTarget(events, county, rect, seed=seed, precision="fp32_skip")
    z0 = np.log(np.array([0.5, 10.0, 7.0, 0.3, 2.0, 0.2]))
    hmc, st, rec, t_burn = burn_in(target, z0, n_burn, n_leapfrog, seed=1, n_warmup=n_warmup, log=log)
    _, held = fit_surrogate(rec, lam=lam, epochs=epochs, seed=5, log=log)
    return {"burn_in_seconds": t_burn, "step_size": hmc.eps, "n_burn": n_burn, "n_warmup": n_warmup,
            "surrogate": held}


def compare(events, county, rect, *, n_burn=1000, n_iter=2000, n_leapfrog=20, seed=2002, lam=1.0, epochs=60,
            n_warmup=300, log=None, replicate: int = 0, fallback_prob: float = 0.0) -> dict:
    """The sampler comparison on one event set.  `replicate` r > 0 repeats it with other random numbers
    throughout: latent-location draws (Philox seed + 100 r), warm-up and burn-in, surrogate training and the
    three samplers."""
    r = int(replicate)
    target = HawkesCutTarget(events, county, rect, seed=seed + 100 * r, precision="fp32_skip")
    z0 = np.log(np.array([0.5, 10.0, 7.0, 0.3, 2.0, 0.2]))
    hmc, st, rec, t_burn = burn_in(target, z0, n_burn, n_leapfrog, seed=1 + r, n_warmup=n_warmup, log=log)
    sur, held = fit_surrogate(rec, lam=lam, epochs=epochs, seed=5 + r, log=log)
    t_train = held["train_seconds"]
    it0 = n_warmup + n_burn + 1
    plain = run_plain_hmc(target, hmc, st.z, n_iter, it0, log=log)
    dah = run_da_hmc(target, sur, hmc, st.z, n_iter, it0 + n_iter + 1, target.prior_var, log=log, seed=11 + r,
                     fallback_prob=fallback_prob)
    mh = run_mh(target, st.z, hmc.inv_mass, n_iter, it0 + 2 * n_iter + 2, log=log, seed=13 + r)
    out = {"burn_in_seconds": t_burn, "surrogate": held, "step_size": hmc.eps, "n_iter": n_iter, "replicate": r}
    for name, r in (("plain_hmc", plain), ("da_hmc", dah), ("univariate_mh", mh)):
        s = _summary(r.draws)
        ess_min = float(np.min(s["bulk_ess"]))
        out[name] = {"seconds": r.seconds, "n_loglik": r.n_loglik, "n_grad": r.n_grad, "stats": r.stats,
                     "min_bulk_ess": ess_min, "ess_per_s": ess_min / r.seconds, **s}
    out["da_hmc"]["ess_per_s_incl_training"] = out["da_hmc"]["min_bulk_ess"] / (dah.seconds + t_train)
    mp, md = np.array(out["plain_hmc"]["mean"]), np.array(out["da_hmc"]["mean"])
    se = np.sqrt(np.array(out["plain_hmc"]["mcse"]) ** 2 + np.array(out["da_hmc"]["mcse"]) ** 2)
    out["means_agree_within_3_mcse"] = bool(np.all(np.abs(mp - md) <= 3 * se))
    out["ess_per_s_ratio"] = out["da_hmc"]["ess_per_s"] / out["plain_hmc"]["ess_per_s"]
    out["mh_ess_per_s_ratio_to_plain_hmc"] = out["univariate_mh"]["ess_per_s"] / out["plain_hmc"]["ess_per_s"]
    return out
