"""QR/UDV-stabilised evaluation of log|det(1 + B_L...B_1)|, its sign and G.

The paper only cites the O(beta N^3) stabilised DQMC algorithm (Introduction;
"Basics of DQMC") without describing it.  This is the textbook procedure:
keep the partial product as U diag(D) V with U orthogonal, D the graded scales
and V well conditioned; every n_stab slices multiply the new slices into U,
scale by D and refactor with a column-pivoted QR (LAPACK dgeqp3 via SciPy).
At the end, with D_b = max(D, 1) and D_s = min(D, 1),

    1 + U D V = U D_b M,   M = D_b^{-1} U^T + D_s V,
    log|W_f| = sum log D_b + log|det M|,   sign = sign det U * sign det M,
    G = M^{-1} D_b^{-1} U^T.

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .lattice import kinetic_propagators, field_diagonal


def udv_chain(model, s, order=None, e=None):
    """U, D, V with U diag(D) V = B_{order[-1]} ... B_{order[0]}.

    Slices are taken n_stab at a time in the given order (default 1..L); the
    last block may be shorter."""
    if e is None:
        e, _ = kinetic_propagators(model.lx, model.ly, model.t, model.mu, model.dtau)
    n = model.n_sites
    order = list(range(1, model.n_slices + 1)) if order is None else list(order)
    u, d, v = np.eye(n), np.ones(n), np.eye(n)
    for b0 in range(0, len(order), model.n_stab):
        x = u.copy()
        for l in order[b0:b0 + model.n_stab]:
            x = e @ (field_diagonal(s[l - 1], model.dtau, model.xi)[:, None] * x)
        x = x * d[None, :]
        q, r, p = sla.qr(x, pivoting=True)            # x[:, p] = q r
        dn = np.abs(np.diag(r))
        t = np.empty_like(r)
        t[:, p] = r / dn[:, None]                      # (D^{-1} R) Pi^T
        u, d, v = q, dn, t @ v
    return u, d, v


def udv_finish(u, d, v, want_green=True):
    """log|det(1 + U D V)|, its sign and (optionally) (1 + U D V)^{-1}."""
    db = np.maximum(d, 1.0)
    ds = np.minimum(d, 1.0)
    m = u.T / db[:, None] + ds[:, None] * v
    lu, piv = sla.lu_factor(m)
    diag = np.diag(lu)
    logabs = float(np.sum(np.log(db)) + np.sum(np.log(np.abs(diag))))
    sdu = int(np.sign(np.linalg.slogdet(u)[0]))
    nswap = int(np.count_nonzero(piv != np.arange(len(piv))))
    sign = sdu * (-1) ** nswap * int(np.prod(np.sign(diag)))
    g = sla.lu_solve((lu, piv), u.T / db[:, None]) if want_green else None
    return logabs, sign, g


def weight(model, s):
    """(log|W_f|, sign) of one field, stabilised."""
    logabs, sign, _ = udv_finish(*udv_chain(model, s), want_green=False)
    return logabs, sign


def green(model, s):
    """(log|W_f|, sign, G) of one field, stabilised."""
    return udv_finish(*udv_chain(model, s))


def green_at_slice(model, s, m: int, e=None):
    """G_m = (1 + B_m...B_1 B_L...B_{m+1})^{-1}, stabilised, from the cyclic
    chain that starts at slice m+1 (kinetic factor e, default exp(-dtau K))."""
    L = model.n_slices
    order = list(range(m + 1, L + 1)) + list(range(1, m + 1))
    return udv_finish(*udv_chain(model, s, order, e=e))[2]
