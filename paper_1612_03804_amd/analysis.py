"""Host-side statistics of Monte Carlo series (measurement, not the sampled path).

The autocorrelation function of the total magnetisation over sweeps or
cumulative updates, C(t) = (<M(0)M(t)> - <M>^2) / (<M^2> - <M>^2) (Fig. 1
caption of the paper), estimated jointly from many independent chains: the
mean is taken over all chains and times, the lagged products are averaged
over chains and time origins.  The integrated autocorrelation time
tau_int = 1/2 + sum_{t=1}^{W} C(t) uses the automatic window (smallest W with
W >= c * tau_int(W), c = 5); effective independent samples = n / (2 tau_int).
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


def tau_int_chains(m: np.ndarray, c: float = 5.0) -> float:
    rho = autocorrelation_chains(m)
    tau = 0.5
    for w in range(1, len(rho)):
        tau += rho[w]
        if w >= c * tau:
            break
    return float(max(tau, 0.5))


def effective_samples(m: np.ndarray, c: float = 5.0) -> float:
    m = np.asarray(m)
    n = m.size
    return n / (2.0 * tau_int_chains(m, c))
