"""Local-update DQMC sweep ("Basics of DQMC").

Flipping s_{i,l} multiplies B_l on the right by 1 + delta e_i e_i^T with
delta = exp(2 dtau xi s_{i,l}) - 1.  With G = G_{l-1} the Green's function of
the cyclic chain whose rightmost factor is B_l, the determinant ratio is

    R = det(1 + A(1 + Delta)) / det(1 + A) = 1 + delta (1 - G_ii)        (O(1))

and on acceptance (Sherman-Morrison)

    G <- G - (delta / R) (e_i - G[:, i]) G[i, :]                        (O(N^2)).

After all sites of slice l: G_l = B_l G_{l-1} B_l^{-1} (wrap).  Every n_stab
slices G is recomputed from scratch and the wrap drift max|G - G_fresh| kept.

Readings where the paper is silent: Metropolis on |R| with strict
u < |R|; slices ascending 1..L, sites ascending 0..N-1; recompute at
l % n_stab == 0; uniform u from Philox with key (seed, TAG_LOCAL) and counter
(site, slice-1, sweep, chain).

Test infrastructure only.
"""
from __future__ import annotations

import math
import numpy as np

from .lattice import kinetic_propagators, field_diagonal
from .philox import uniform, TAG_LOCAL
from . import stable


def sweep(model, s, g, logabs, sign, *, seed: int, sweep_index: int, chain: int = 0,
          e=None, einv=None, want_trace=False):
    """One sweep over the N*L space-time sites.  s (int8 [L][N]) and g (G_0 = G)
    are updated in place.  Returns (logabs, sign, accepts, max_drift[, trace])
    where trace lists (l, i, R, u, accepted) for every proposal."""
    if e is None:
        e, einv = kinetic_propagators(model.lx, model.ly, model.t, model.mu, model.dtau)
    n, L = model.n_sites, model.n_slices
    a = model.dtau * model.xi
    accepts = 0
    drift = 0.0
    trace = [] if want_trace else None
    key = (seed, TAG_LOCAL)
    for l in range(1, L + 1):
        for i in range(n):
            delta = math.exp(2.0 * a * float(s[l - 1, i])) - 1.0
            r = 1.0 + delta * (1.0 - g[i, i])
            u = uniform((i, l - 1, sweep_index, chain), key)
            acc = u < abs(r)
            if want_trace:
                trace.append((l, i, r, u, acc))
            if acc:
                col = -g[:, i].copy()
                col[i] += 1.0
                g -= (delta / r) * np.outer(col, g[i, :])
                s[l - 1, i] = -s[l - 1, i]
                logabs += math.log(abs(r))
                sign *= 1 if r > 0 else -1
                accepts += 1
        d = field_diagonal(s[l - 1], model.dtau, model.xi)
        g[:, :] = e @ ((d[:, None] * g) / d[None, :]) @ einv
        if l % model.n_stab == 0:
            fresh = stable.green_at_slice(model, s, l, e=e)
            drift = max(drift, float(np.max(np.abs(g - fresh))))
            g[:, :] = fresh
    if want_trace:
        return logabs, sign, accepts, drift, trace
    return logabs, sign, accepts, drift
