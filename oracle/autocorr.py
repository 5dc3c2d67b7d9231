"""Autocorrelation of a Monte Carlo series (Fig. 1 caption, "Basics of DQMC").

C(t) = (<M(0) M(t)> - <M>^2) / (<M^2> - <M>^2) over the series of total
magnetisations, one entry per sweep (or per cumulative step).  The integrated
time tau_int = 1/2 + sum_{t=1}^{W} C(t) uses Sokal's automatic window: the
smallest W with W >= c tau_int(W), c = 5.  That window presumes positive
correlations; when the windowed sum is below 1/2 (successive entries
anticorrelated, e.g. local sweeps that flip most spins) it stops at W = 1 on a
meaningless, possibly negative value, and tau_int is then Geyer's initial
positive sequence estimate -1/2 + sum_{k=0}^{K} (C(2k) + C(2k+1)), K the last
k before a pair sum is not positive.  (The paper defines C(t) only; both
estimators are readings.)  Effective independent samples of a series of n
entries: n / (2 tau_int).

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np


def autocorrelation(m) -> np.ndarray:
    m = np.asarray(m, dtype=np.float64)
    n = len(m)
    d = m - m.mean()
    var = float(d @ d) / n
    return np.array([float(d[: n - t] @ d[t:]) / (n - t) / var for t in range(n // 2)])


def tau_int_ips(m) -> float:
    """Geyer's initial positive sequence estimate of tau_int."""
    rho = autocorrelation(m)
    total = 0.0
    for k in range(len(rho) // 2):
        pair = rho[2 * k] + rho[2 * k + 1]
        if pair <= 0.0:
            break
        total += pair
    return float(total - 0.5)


def tau_int(m, c: float = 5.0) -> float:
    rho = autocorrelation(m)
    tau = 0.5
    for w in range(1, len(rho)):
        tau += rho[w]
        if w >= c * tau:
            break
    return float(tau) if tau >= 0.5 else tau_int_ips(m)


def effective_samples(m, c: float = 5.0) -> float:
    return len(m) / (2.0 * tau_int(m, c))
