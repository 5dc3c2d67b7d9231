"""Effective bosonic action and cumulative update ("Formalism of SLDQMC").

Eq. (2) writes H_eff = E_0 + sum J s s + ..., with symmetry-reduced couplings
of range gamma.  Here each independent coupling is a term k = (r, dl): spatial
shell r (sites at the r-th smallest squared distance on the torus) and time
separation dl >= 0.  The partner multiset of x = (i, l) is

    P_k(x) = {(i + delta, l + sigma dl mod L) : delta in shell r, sigma = +-1}  (dl > 0)
    P_k(x) = {(i + delta, l)                 : delta in shell r}              (dl = 0)

h_k(x) = sum_{y in P_k(x)} s_y and F_k(s) = 1/2 sum_x s_x h_k(x).  The term
(0, 0) is the one-body term of the expansion (a uniform field on the
auxiliary spins, the first of the terms Eq. (2) leaves as "..."): h(x) = 1 and
F = sum_x s_x.  A single-determinant weight has no s -> -s symmetry, so this
term carries most of the variance of ln omega.  The effective log-weight is
S_eff = c0 + sum_k lambda_k F_k with lambda_k = -beta J_k and c0 = -beta E_0
(Eq. 3 fits it to ln omega).  Flipping x changes it by
dS = -2 s_x sum_k lambda_k h_k(x) whenever x is not its own partner.

Effective moves (step iii): one move picks a colour class uniformly at random
and applies Metropolis (u < exp(dS)) to every site of the class; a class is
one time slice and one colour of a greedy spatial colouring of the dl = 0
coupling graph, so no two of its sites interact and the move is a product of
commuting single-site kernels.  A random class choice makes the chain
reversible with respect to exp(S_eff), which Eq. (4) assumes.

Cumulative update (steps iii-iv, Eq. 4):
    logA = [ln|W(s')| - ln|W(s)|] - [S_eff(s') - S_eff(s)],  accept iff ln u < min(0, logA).

Random numbers: Philox key (seed, TAG_EFFECTIVE); class choice of move t of
cumulative step c uses counter (0, t, c, chain) and "below(n_classes)"; the
Metropolis draw of site x = (i, l) uses counter (1 + (l-1) N + i, t, c, chain).
Acceptance uses key (seed, TAG_CUMULATIVE), counter (0, 0, c, chain).

Test infrastructure only.
"""
from __future__ import annotations

import math
from functools import lru_cache
import numpy as np

from .philox import uniform, below, TAG_EFFECTIVE, TAG_CUMULATIVE


@lru_cache(maxsize=None)
def shell_offsets(r: int, max_shell: int = 8):
    """Integer offsets (dx, dy) of the r-th shell: shell 0 is (0,0), shell 1 the
    four nearest neighbours, shell 2 the four diagonals, shell 3 (+-2,0),(0,+-2)...
    Shells are ordered by squared Euclidean length of the offset."""
    rng = range(-max_shell, max_shell + 1)
    lengths = sorted({dx * dx + dy * dy for dx in rng for dy in rng})
    d2 = lengths[r]
    return tuple((dx, dy) for dx in rng for dy in rng if dx * dx + dy * dy == d2)


def partners(model, term, i: int, l: int):
    """Partner multiset P_k((i, l)) as a list of (site, slice) with slice 1-based
    (empty for the one-body term)."""
    r, dl = term
    if r == 0 and dl == 0:
        return []
    lx, ly, L = model.lx, model.ly, model.n_slices
    x, y = i % lx, i // lx
    out = []
    for dx, dy in shell_offsets(r):
        j = (x + dx) % lx + lx * ((y + dy) % ly)
        if dl == 0:
            out.append((j, l))
        else:
            for sg in (1, -1):
                out.append((j, (l - 1 + sg * dl) % L + 1))
    return out


def check_terms(model, terms):
    """A term is usable when 0 <= dl <= L/2 and no site is its own partner
    (which small tori can cause, e.g. (+-2, 0) on Lx = 2)."""
    for r, dl in terms:
        if dl < 0 or dl > model.n_slices // 2:
            raise ValueError(f"unusable term {(r, dl)}")
        if (0, 1) in partners(model, (r, dl), 0, 1):
            raise ValueError(f"term {(r, dl)} makes a site its own partner")


def local_fields(model, terms, s):
    """h[k, l-1, i] = h_k((i, l)): the partner sums written as cyclic shifts of
    the field viewed as [L][Ly][Lx] (np.roll(a, -k)[j] = a[j + k])."""
    L, lx, ly = model.n_slices, model.lx, model.ly
    s3 = np.asarray(s, dtype=np.float64).reshape(L, ly, lx)
    h = np.zeros((len(terms), L, ly, lx))
    for k, (r, dl) in enumerate(terms):
        if r == 0 and dl == 0:
            h[k] = 1.0
            continue
        for dx, dy in shell_offsets(r):
            for sg in ((0,) if dl == 0 else (1, -1)):
                h[k] += np.roll(s3, shift=(-sg * dl, -dy, -dx), axis=(0, 1, 2))
    return h.reshape(len(terms), L, lx * ly)


def local_fields_slice(model, terms, s, l: int):
    """h[k, i] = h_k((i, l)) at one slice l (1-based): the same partner sums as
    local_fields, taken only from the slices l and l +- dl that slice l's
    partners lie on."""
    L, lx, ly = model.n_slices, model.lx, model.ly
    s3 = np.asarray(s, dtype=np.float64).reshape(L, ly, lx)
    h = np.zeros((len(terms), ly, lx))
    for k, (r, dl) in enumerate(terms):
        if r == 0 and dl == 0:
            h[k] = 1.0
            continue
        for dx, dy in shell_offsets(r):
            for sg in ((0,) if dl == 0 else (1, -1)):
                h[k] += np.roll(s3[(l - 1 + sg * dl) % L], shift=(-dy, -dx), axis=(0, 1))
    return h.reshape(len(terms), lx * ly)


def local_fields_bruteforce(model, terms, s):
    """Same as local_fields, by summing the explicit partner lists (small cases)."""
    n, L = model.n_sites, model.n_slices
    h = np.zeros((len(terms), L, n))
    for k, term in enumerate(terms):
        for l in range(1, L + 1):
            for i in range(n):
                if term == (0, 0):
                    h[k, l - 1, i] = 1
                else:
                    h[k, l - 1, i] = sum(int(s[ll - 1, j]) for j, ll in partners(model, term, i, l))
    return h


def features(model, terms, s) -> np.ndarray:
    """F_k(s) = 1/2 sum_x s_x h_k(x), and sum_x s_x for the one-body term
    (exact half-integers in FP64)."""
    h = local_fields(model, terms, s)
    half = np.array([1.0 if tuple(t) == (0, 0) else 0.5 for t in terms])
    return half * np.einsum("li,kli->k", s.astype(np.float64), h)


def action(model, terms, c0, lam, s) -> float:
    """S_eff(s) = c0 + sum_k lambda_k F_k(s)."""
    return float(c0 + np.dot(lam, features(model, terms, s)))


def flip_delta(model, terms, lam, s, i: int, l: int) -> float:
    """dS for flipping (i, l): -2 s_x sum_k lambda_k h_k(x)."""
    tot = 0.0
    for k, term in enumerate(terms):
        if tuple(term) == (0, 0):
            tot += lam[k]
        else:
            tot += lam[k] * sum(int(s[ll - 1, j]) for j, ll in partners(model, term, i, l))
    return -2.0 * float(s[l - 1, i]) * tot


def spatial_colouring(model, terms, net_range: int = 0):
    """Greedy colouring of the sites, ascending index, smallest free colour,
    on the graph linking i to every spatial partner of the dl = 0 terms and,
    when net_range > 0, to every site within that periodic Chebyshev distance
    (the reach of a flip through the learned action's two 3^3 convolutions is
    2, so sites closer than 5 interact through it)."""
    n = model.n_sites
    nbr = [set() for _ in range(n)]
    for term in terms:
        if term[1] != 0:
            continue
        for i in range(n):
            for j, _ in partners(model, term, i, 1):
                if j != i:
                    nbr[i].add(j)
                    nbr[j].add(i)
    for i in range(n):
        x, y = i % model.lx, i // model.lx
        for dy in range(-net_range, net_range + 1):
            for dx in range(-net_range, net_range + 1):
                j = (x + dx) % model.lx + model.lx * ((y + dy) % model.ly)
                if j != i:
                    nbr[i].add(j)
                    nbr[j].add(i)
    col = [-1] * n
    for i in range(n):
        used = {col[j] for j in nbr[i] if col[j] >= 0}
        c = 0
        while c in used:
            c += 1
        col[i] = c
    return col


def colour_classes(model, terms, net_range: int = 0):
    """Class index c_s + n_colours * (l - 1) lists the sites i with colour c_s
    at slice l; returns the list of (l, [sites])."""
    col = spatial_colouring(model, terms, net_range)
    nc = max(col) + 1
    return [(l, [i for i in range(model.n_sites) if col[i] == c])
            for l in range(1, model.n_slices + 1) for c in range(nc)]


def effective_move(model, terms, lam, s, classes, *, seed, step, move, chain=0, net_params=None):
    """One colour-class move in place; returns (#accepted, sum of accepted dS).
    With net_params the action is S_lin + S_net and each flip's change of
    S_net comes from two full forward passes (oracle.net.flip_delta)."""
    key = (seed, TAG_EFFECTIVE)
    cls = below(len(classes), (0, move, step, chain), key)
    l, sites = classes[cls]
    hsum = np.tensordot(np.asarray(lam, dtype=np.float64), local_fields_slice(model, terms, s, l), axes=1)
    ds = [-2.0 * float(s[l - 1, i]) * float(hsum[i]) for i in sites]   # pre-move field
    if net_params is not None:
        from . import net
        ds = [d + net.flip_delta(net_params, model, s, i, l) for d, i in zip(ds, sites)]
    acc, tot = 0, 0.0
    for i, d in zip(sites, ds):
        u = uniform((1 + (l - 1) * model.n_sites + i, move, step, chain), key)
        if u < math.exp(d):
            s[l - 1, i] = -s[l - 1, i]
            acc += 1
            tot += d
    return acc, tot


def effective_sweep(model, terms, lam, s, n_moves, *, seed, step, chain=0, classes=None, net_params=None):
    """n_moves colour-class moves in place; returns (#accepted, sum dS)."""
    classes = classes or colour_classes(model, terms, 4 if net_params is not None else 0)
    acc, tot = 0, 0.0
    for m in range(n_moves):
        a, d = effective_move(model, terms, lam, s, classes, seed=seed, step=step, move=m, chain=chain,
                              net_params=net_params)
        acc += a
        tot += d
    return acc, tot


def cumulative_step(model, terms, c0, lam, s, logabs, sign, n_moves, weight_fn, *,
                    seed, step, chain=0, classes=None, net_params=None):
    """One cumulative update (Eq. 4).  Returns (s, logabs, sign, accepted, logA)
    with s replaced by the proposal when accepted.  weight_fn(s) -> (log|W|, sign).
    With net_params the effective action is S_lin + S_net."""
    prop = s.copy()
    effective_sweep(model, terms, lam, prop, n_moves, seed=seed, step=step, chain=chain, classes=classes,
                    net_params=net_params)
    ds = float(np.dot(lam, features(model, terms, prop) - features(model, terms, s)))
    if net_params is not None:
        from . import net
        ds += net.forward(net_params, model, prop)[0] - net.forward(net_params, model, s)[0]
    new_logabs, new_sign = weight_fn(prop)
    log_a = (new_logabs - logabs) - ds
    u = uniform((0, 0, step, chain), (seed, TAG_CUMULATIVE))
    lu = -math.inf if u == 0.0 else math.log(u)
    if new_sign != 0 and lu < min(0.0, log_a):
        return prop, new_logabs, new_sign, True, log_a
    return s, logabs, sign, False, log_a
