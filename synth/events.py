"""Synthetic stand-in for the paper's one-million-case COVID-19 data set.

The paper analyses about 10^6 hospital cases spread over roughly 1,200 days and
about 3,000 U.S. counties, each county carrying a population density (its
Section 3.2 and Table 2, where densities run from about 35 to 74,000 per square
mile).  That data set is not available here, so every workload is drawn from a
seeded recipe with the same shape:

* times: sorted i.i.d. uniform draws on [0, T] days;
* locations: an equal-weight mixture of 10 isotropic Gaussians (sd 20 km) whose
  centres are uniform in a 1000 x 1000 km box;
* counties: a regular nx x ny grid of rectangles over the box; an event belongs
  to the cell that contains its mixture draw (index clamped to the box);
* densities: one LogNormal(5, sdlog) draw per county, shared by its events;
* bandwidth scale: s_n = (rho_n / median_n rho_n)^(-1/2), so that the
  triggering sd of source n is h0 * s_n (the paper's model 2 with the density
  normalised by its median).

A second recipe, ``generate_clustered``, adds the temporal and space-time
clustering that the model describes (epidemic waves with their own hot spots,
and cases that follow earlier nearby cases), so that a posterior over the six
parameters is concentrated; the sampler comparison runs on it.

Nothing here evaluates the likelihood.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class WorkloadConfig:
    name: str
    n: int
    t_max: float          # days
    nx: int               # county grid columns
    ny: int               # county grid rows
    rho_sdlog: float
    seed: int
    box_km: float = 1000.0
    n_centres: int = 10
    centre_sd_km: float = 20.0
    rho_meanlog: float = 5.0


# The workloads: a small FP64 parity case, 1e5 events, and 1e6 events (the
# likelihood benchmark, with per-iteration location resampling).
N2K = WorkloadConfig("n2000_100d_200c", 2_000, 100.0, 10, 20, 1.0, 1000)
N100K = WorkloadConfig("n100k_1000d_3000c", 100_000, 1000.0, 50, 60, 1.0, 1001)
N1M = WorkloadConfig("n1m_1200d_3000c", 1_000_000, 1200.0, 50, 60, 1.5, 1002)
WORKLOADS = {w.name: w for w in (N2K, N100K, N1M)}

# Parameter vector (mu, tau_x [km], tau_t [d], xi, h0 [km], omega [1/d]).
THETA_NAMES = ("mu", "tau_x", "tau_t", "xi", "h0", "omega")


def theta_default() -> np.ndarray:
    """The parameter values every workload is evaluated at."""
    return np.array([0.5, 10.0, 7.0, 0.3, 2.0, 0.2], dtype=np.float64)


@dataclass
class EventSet:
    t: np.ndarray          # (n,) float64, nondecreasing, days
    x: np.ndarray          # (n,) float64, km
    y: np.ndarray          # (n,) float64, km
    s: np.ndarray          # (n,) float64, bandwidth scale (> 0)
    county: np.ndarray     # (n,) int32 county id
    rect: np.ndarray       # (C, 4) float64 rows (x0, y0, x1, y1)
    rho_county: np.ndarray  # (C,) float64
    config: WorkloadConfig = field(repr=False, default=None)

    @property
    def n(self) -> int:
        return int(self.t.shape[0])


def _county_rects(cfg: WorkloadConfig) -> np.ndarray:
    wx = cfg.box_km / cfg.nx
    wy = cfg.box_km / cfg.ny
    iy, ix = np.divmod(np.arange(cfg.nx * cfg.ny), cfg.nx)
    return np.stack([ix * wx, iy * wy, (ix + 1) * wx, (iy + 1) * wy], axis=1).astype(np.float64)


def generate(k: str | WorkloadConfig, n: int | None = None, seed: int | None = None) -> EventSet:
    """Draw workload ``k`` (a name in WORKLOADS or a WorkloadConfig).

    ``n`` and ``seed`` override the event count and seed while keeping the rest
    of the recipe (used for smaller parity cases of the same shape).
    """
    cfg = WORKLOADS[k] if isinstance(k, str) else k
    n = cfg.n if n is None else int(n)
    seed = cfg.seed if seed is None else int(seed)
    rng = np.random.default_rng(seed)

    t = np.sort(rng.uniform(0.0, cfg.t_max, n))
    centres = rng.uniform(0.0, cfg.box_km, (cfg.n_centres, 2))
    comp = rng.integers(0, cfg.n_centres, n)
    xy = centres[comp] + rng.normal(0.0, cfg.centre_sd_km, (n, 2))

    wx = cfg.box_km / cfg.nx
    wy = cfg.box_km / cfg.ny
    ix = np.clip(np.floor(xy[:, 0] / wx), 0, cfg.nx - 1).astype(np.int64)
    iy = np.clip(np.floor(xy[:, 1] / wy), 0, cfg.ny - 1).astype(np.int64)
    county = (iy * cfg.nx + ix).astype(np.int32)

    rho_county = rng.lognormal(cfg.rho_meanlog, cfg.rho_sdlog, cfg.nx * cfg.ny)
    rho = rho_county[county]
    s = (rho / np.median(rho)) ** -0.5

    return EventSet(
        t=np.ascontiguousarray(t),
        x=np.ascontiguousarray(xy[:, 0]),
        y=np.ascontiguousarray(xy[:, 1]),
        s=np.ascontiguousarray(s),
        county=county,
        rect=_county_rects(cfg),
        rho_county=rho_county,
        config=cfg,
    )


def generate_clustered(n: int = 100_000, seed: int = 1101, t_max: float = 1000.0, nx: int = 50, ny: int = 60,
                       rho_sdlog: float = 1.0, branching: float = 0.6, delay_days: float = 5.0, h_km: float = 12.0,
                       n_waves: int = 6, wave_sd_days: float = 25.0, uniform_share: float = 0.3) -> EventSet:
    """A seeded branching (cluster) process over the workloads' box and county grid.

    Immigrant cases: times from ``n_waves`` Gaussian epidemic waves (centres uniform on
    [0.1, 0.9] t_max, sd ``wave_sd_days``), each wave with its own 10-centre mixture of
    locations (centres uniform in the box, sd 20 km), plus a ``uniform_share`` of cases
    uniform in time and in the box.  Spatial clustering is thus local in time: with one
    mixture for all times, the long-run persistence of the centres is explained best by a
    triggering kernel that never decays (omega -> 0), and the posterior runs off along
    that ridge.  Every case has Poisson(``branching``) offspring, each
    ``Exp(mean delay_days)`` later and displaced by N(0, (h_km s)^2) per axis, s the
    bandwidth scale of the parent's county.  Cases after t_max are dropped and the set is
    thinned uniformly at random to exactly n events.

    The displacement scale is chosen above the county cells' size (20 x 16.7 km on the
    default grid): the cut posterior redraws every location uniformly within its county, so
    offspring structure finer than a county is lost, and with h_km = 2 the triggering kernel
    instead settled at county or hot-spot scale in two competing posterior modes of nearly
    equal height.  At 12 km the mode near the generating scales is higher than any other by
    about 100 nats or more under every latent draw tried.
    """
    cfg = WorkloadConfig(f"n{n // 1000}k_clustered_{int(t_max)}d_{nx * ny}c", n, t_max, nx, ny, rho_sdlog, seed)
    rng = np.random.default_rng(seed)
    rho_county = rng.lognormal(cfg.rho_meanlog, cfg.rho_sdlog, nx * ny)
    wx, wy = cfg.box_km / nx, cfg.box_km / ny

    def county_of(xy):
        ix = np.clip(np.floor(xy[:, 0] / wx), 0, nx - 1).astype(np.int64)
        iy = np.clip(np.floor(xy[:, 1] / wy), 0, ny - 1).astype(np.int64)
        return (iy * nx + ix).astype(np.int32)

    n0 = int(1.1 * n * (1.0 - branching))
    n_unif = int(uniform_share * n0)
    n_wave = n0 - n_unif
    wave_c = rng.uniform(0.1 * t_max, 0.9 * t_max, n_waves)
    wave_centres = rng.uniform(0.0, cfg.box_km, (n_waves, cfg.n_centres, 2))
    w = rng.integers(0, n_waves, n_wave)
    t0 = np.concatenate([rng.uniform(0.0, t_max, n_unif), wave_c[w] + rng.normal(0.0, wave_sd_days, n_wave)])
    xy0 = np.concatenate([rng.uniform(0.0, cfg.box_km, (n_unif, 2)),
                          wave_centres[w, rng.integers(0, cfg.n_centres, n_wave)]
                          + rng.normal(0.0, cfg.centre_sd_km, (n_wave, 2))])
    keep = (t0 > 0.0) & (t0 < t_max)
    t0, xy0 = t0[keep], xy0[keep]
    med = np.median(rho_county[county_of(xy0)])
    ts, xys = [t0], [xy0]
    gt, gxy = t0, xy0
    while gt.shape[0]:
        k = rng.poisson(branching, gt.shape[0])
        pt, pxy = np.repeat(gt, k), np.repeat(gxy, k, axis=0)
        sd = h_km * (rho_county[county_of(pxy)] / med) ** -0.5
        ct = pt + rng.exponential(delay_days, pt.shape[0])
        cxy = pxy + rng.normal(0.0, 1.0, (pt.shape[0], 2)) * sd[:, None]
        inside = ct < t_max
        gt, gxy = ct[inside], cxy[inside]
        ts.append(gt)
        xys.append(gxy)
    t = np.concatenate(ts)
    xy = np.concatenate(xys)
    if t.shape[0] < n:
        raise ValueError(f"the cluster process gave {t.shape[0]} < {n} events; raise the immigrant count")
    pick = np.sort(rng.choice(t.shape[0], n, replace=False))
    t, xy = t[pick], xy[pick]
    order = np.argsort(t, kind="stable")
    t, xy = t[order], xy[order]
    county = county_of(xy)
    rho = rho_county[county]
    s_ = (rho / np.median(rho)) ** -0.5
    return EventSet(t=np.ascontiguousarray(t), x=np.ascontiguousarray(xy[:, 0]), y=np.ascontiguousarray(xy[:, 1]),
                    s=np.ascontiguousarray(s_), county=county, rect=_county_rects(cfg), rho_county=rho_county,
                    config=cfg)
