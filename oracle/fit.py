"""Self-learning fit of the effective action (Eq. 3 and the R^2 score of "Results").

Eq. (3) sets -beta H_eff[C] = ln omega[C]; the couplings come from a
multi-linear regression over the training configurations.  Reading taken:
unweighted ordinary least squares with an intercept on y_n = ln|W_f(s_n)|,
design rows [1, F_1(s_n), ..., F_K(s_n)], solved by SciPy's least squares.
R^2 = 1 - sum (y - yhat)^2 / sum (y - ybar)^2, which equals the paper's
1 - <(H_eff - H)^2> / (<H^2> - <H>^2) because an OLS fit with an intercept has
zero mean residual and beta cancels.

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .effective import features


def design(model, terms, fields) -> np.ndarray:
    return np.stack([np.concatenate(([1.0], features(model, terms, s))) for s in fields])


def fit(model, terms, fields, logabs):
    """(c0, lambda[K], R^2)."""
    x = design(model, terms, fields)
    y = np.asarray(logabs, dtype=np.float64)
    theta, *_ = sla.lstsq(x, y)
    res = y - x @ theta
    r2 = 1.0 - float(res @ res) / float(((y - y.mean()) ** 2).sum())
    return float(theta[0]), theta[1:], r2
