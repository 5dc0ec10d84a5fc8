"""Bulk effective sample size and split R-hat (Vehtari, Gelman, Simpson,
Carpenter and Buerkner, 2021), the diagnostics the paper reports for its
chains (Section 3.2).  Draws are rank-normalised over all split chains; the
autocorrelation sum uses Geyer's initial positive and monotone sequences."""

from __future__ import annotations

import numpy as np
from scipy import stats


def _split(draws: np.ndarray) -> np.ndarray:
    """(chains, n) -> (2*chains, n//2): first and second half of every chain."""
    draws = np.atleast_2d(np.asarray(draws, dtype=np.float64))
    h = draws.shape[1] // 2
    return np.concatenate([draws[:, :h], draws[:, draws.shape[1] - h:]], axis=0)


def _rank_normalise(x: np.ndarray) -> np.ndarray:
    r = stats.rankdata(x.ravel(), method="average").reshape(x.shape)
    return stats.norm.ppf((r - 0.375) / (x.size + 0.25))


def _autocov(x: np.ndarray) -> np.ndarray:
    """Autocovariance of one chain at all lags (biased estimator, via FFT)."""
    n = x.shape[0]
    xc = x - x.mean()
    m = 1 << (2 * n - 1).bit_length()
    f = np.fft.rfft(xc, m)
    ac = np.fft.irfft(f * np.conj(f), m)[:n]
    return ac / n


def ess(draws: np.ndarray) -> float:
    """ESS of (chains, n) draws (no splitting or ranking): Geyer-truncated autocorrelations."""
    x = np.atleast_2d(np.asarray(draws, dtype=np.float64))
    m, n = x.shape
    if n < 4:
        return float("nan")
    acov = np.array([_autocov(c) for c in x])
    chain_var = acov[:, 0] * n / (n - 1.0)
    W = chain_var.mean()
    var_plus = W * (n - 1.0) / n
    if m > 1:
        var_plus += x.mean(axis=1).var(ddof=1)
    if var_plus <= 0:
        return float(m * n)
    rho = 1.0 - (W - acov.mean(axis=0)) / var_plus
    rho[0] = 1.0
    # Geyer: sums of adjacent pairs, truncated at the first non-positive pair, made monotone
    pairs = []
    t = 0
    while t + 1 < n:
        p = rho[t] + rho[t + 1]
        if p <= 0:
            break
        pairs.append(p)
        t += 2
    pairs = np.minimum.accumulate(np.array(pairs)) if pairs else np.array([1.0])
    tau = -1.0 + 2.0 * pairs.sum()
    tau = max(tau, 1.0 / np.log10(m * n))
    return float(m * n / tau)


def bulk_ess(draws: np.ndarray) -> float:
    """Bulk-ESS: ESS of rank-normalised split chains."""
    return ess(_rank_normalise(_split(draws)))


def split_rhat(draws: np.ndarray) -> float:
    """Rank-normalised split R-hat."""
    x = _rank_normalise(_split(draws))
    m, n = x.shape
    W = x.var(axis=1, ddof=1).mean()
    B = n * x.mean(axis=1).var(ddof=1)
    var_plus = (n - 1.0) / n * W + B / n
    return float(np.sqrt(var_plus / W))


def mcse_mean(draws: np.ndarray) -> float:
    """Monte Carlo standard error of the mean from the (non-ranked) split-chain ESS."""
    x = np.atleast_2d(np.asarray(draws, dtype=np.float64))
    return float(x.std(ddof=1) / np.sqrt(ess(_split(x))))
