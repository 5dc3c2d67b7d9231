"""Host-side statistics of Monte Carlo series (measurement, not the sampled path).

The autocorrelation function of the total magnetisation over sweeps or
cumulative updates, C(t) = (<M(0)M(t)> - <M>^2) / (<M^2> - <M>^2) (Fig. 1
caption of the paper), estimated jointly from many independent chains: the
mean is taken over all chains and times, the lagged products are averaged
over chains and time origins.  The integrated autocorrelation time
tau_int = 1/2 + sum_{t=1}^{W} C(t) uses the automatic window (smallest W with
W >= c * tau_int(W), c = 5).  The window presumes positive correlations: when
its sum is below 1/2 (anticorrelated successive values, e.g. local sweeps that
flip most spins) it stops at W = 1, and tau_int is then the initial positive
sequence estimate -1/2 + sum_{k<=K} (C(2k) + C(2k+1)), K the last k before a
pair sum is not positive (Geyer).  Effective independent samples = n / (2 tau_int).
"""
from __future__ import annotations

import numpy as np


def autocorrelation_chains(m: np.ndarray) -> np.ndarray:
    """C(t) for t = 0 .. T/2 - 1 from an array [chains, T]."""
    m = np.asarray(m, dtype=np.float64)
    if m.ndim == 1:
        m = m[None, :]
    chains, T = m.shape
    d = m - m.mean()
    var = float((d * d).mean())
    if var == 0.0:
        return np.concatenate(([1.0], np.zeros(max(0, T // 2 - 1))))
    return np.array([float((d[:, :T - t] * d[:, t:]).mean()) / var for t in range(max(1, T // 2))])


def _initial_positive_sequence(rho: np.ndarray) -> tuple[float, int]:
    total, k = 0.0, 0
    while 2 * k + 1 < len(rho):
        pair = rho[2 * k] + rho[2 * k + 1]
        if pair <= 0.0:
            break
        total += pair
        k += 1
    return total - 0.5, 2 * k - 1


def tau_int_chains(m: np.ndarray, c: float = 5.0) -> float:
    """tau_int, not clamped: a series whose successive values are
    anticorrelated has tau_int < 1/2, i.e. more than one effective sample per
    step (then from the initial positive sequence)."""
    return tau_int_window(m, c)["tau_int"]


def tau_int_window(m: np.ndarray, c: float = 5.0) -> dict:
    """tau_int with its window W and whether the window condition W >= c tau
    was met before the lags ran out (T/2); when it was not, tau is a lower
    bound of the series' integrated autocorrelation time.  Anticorrelated
    series (windowed sum below 1/2) take the initial positive sequence; its
    last lag is reported as the window."""
    rho = autocorrelation_chains(m)
    tau = 0.5
    for w in range(1, len(rho)):
        tau += rho[w]
        if w >= c * max(tau, 0.0):
            if tau < 0.5:
                ips, last = _initial_positive_sequence(rho)
                return {"tau_int": float(ips), "window": last, "converged": True,
                        "estimator": "initial positive sequence"}
            return {"tau_int": float(tau), "window": w, "converged": True}
    return {"tau_int": float(tau), "window": len(rho) - 1, "converged": False}


def effective_samples(m: np.ndarray, c: float = 5.0) -> float | None:
    """n / (2 tau_int), None when tau_int is not positive (too short a series)."""
    m = np.asarray(m)
    tau = tau_int_chains(m, c)
    return m.size / (2.0 * tau) if tau > 0 else None


def mean_and_error(x: np.ndarray, c: float = 5.0) -> tuple[float, float]:
    """Mean of a series [chains, T] and its standard error, the variance of
    the mean inflated by 2 tau_int (at least the naive error: tau_int is
    floored at 1/2 here, so an anticorrelated series is not credited with an
    error below the independent-sample one)."""
    x = np.asarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[None, :]
    var = float(x.var())
    tau = max(tau_int_chains(x, c), 0.5) if var > 0 else 0.5
    return float(x.mean()), float(np.sqrt(var * 2.0 * tau / x.size))


def agree(a: tuple[float, float], b: tuple[float, float], sigmas: float = 2.0) -> bool:
    """Two (mean, error) estimates agree within `sigmas` combined standard errors."""
    return abs(a[0] - b[0]) <= sigmas * float(np.hypot(a[1], b[1])) + 1e-12 * max(abs(a[0]), abs(b[0]), 1.0)
