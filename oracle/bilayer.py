"""The paper's own workload ("Results", Eq. 6): spin-1/2 fermions on a
bilayer square lattice (layers lambda = 1, 2, intralayer hopping t, chemical
potential mu) coupled to transverse-field Ising spins (ferromagnetic J,
transverse field h) through H_sf = -xi sum_i s^z_i (sigma^z_{i1} - sigma^z_{i2}).

After the Trotter decomposition ("Basics of DQMC", Eq. 1) the Ising spins are
the auxiliary field s_{i,l} = +-1 (one per site of the layer pair and slice)
and the weight of a configuration is

    omega(s) = phi(s) prod_f det(1 + B^f_L ... B^f_1).

The four fermion flavours f = (lambda, sigma) do not mix (no interlayer
hopping).  Flavour f sees the potential -xi s eta_f with eta_f = sigma in
layer 1 and -sigma in layer 2, so B^f_l = E diag(exp(dtau xi eta_f s_{.,l})),
E = exp(-dtau K) of one layer.  In the single-flavour notation of the hot path
(d_l = exp(-dtau xi s)) eta = -1 is W_f(s) and eta = +1 is W_f(-s); two
flavours have each, so

    omega(s) = phi(s) [W_f(s) W_f(-s)]^2 >= 0        (no sign problem).

phi is the weight of the Ising spins alone (Eq. 1's fermion-free factor): the
standard quantum-to-classical mapping of H_s = -J sum_<ij> s^z s^z
- h sum_i s^x with slices of width dtau gives, up to a constant factor
(sqrt(sinh(2 dtau h) / 2) per site and slice),

    ln phi = dtau J sum_l sum_<ij> s_{i,l} s_{j,l} + K_tau sum_{i,l} s_{i,l} s_{i,l+1},
    K_tau = -1/2 ln tanh(dtau h),

time periodic, bonds <ij> counted with multiplicity as in the hopping matrix
(a length-2 dimension carries each bond twice).

Local update of one spin (the DQMC step of "Basics of DQMC" for this weight):
with G^a the Green's function of the field s and G^b that of -s (both of the
chain ending at B_l), the flip s_{i,l} -> -s_{i,l} has

    R_a = 1 + delta_a (1 - G^a_ii),  delta_a = exp(+2 dtau xi s_{i,l}) - 1,
    R_b = 1 + delta_b (1 - G^b_ii),  delta_b = exp(-2 dtau xi s_{i,l}) - 1,
    ratio = phi(s')/phi(s) (R_a R_b)^2,

accepted iff u < ratio; both Green's functions then take their rank-1
update, and after each slice both are wrapped.

Test infrastructure only.
"""
from __future__ import annotations

import math
import numpy as np

from . import stable
from .lattice import hopping_matrix, kinetic_propagators, field_diagonal
from .philox import uniform, TAG_LOCAL


def bare_coupling(dtau: float, h: float) -> float:
    """K_tau = -1/2 ln tanh(dtau h) of the Ising spins along imaginary time."""
    return -0.5 * math.log(math.tanh(dtau * h))


def bonds(lx: int, ly: int):
    """Nearest-neighbour bonds (i, j) of the periodic lattice, one per site and
    direction (so a length-2 dimension lists each pair twice)."""
    out = []
    for y in range(ly):
        for x in range(lx):
            i = x + lx * y
            out.append((i, (x + 1) % lx + lx * y))
            out.append((i, x + lx * ((y + 1) % ly)))
    return out


def bare_log_weight(model, J: float, h: float, s) -> float:
    """ln phi(s) of the Ising spins (up to its constant), written out over
    bonds and time neighbours."""
    L = model.n_slices
    kt = bare_coupling(model.dtau, h)
    tot = 0.0
    for l in range(L):
        for i, j in bonds(model.lx, model.ly):
            tot += model.dtau * J * float(s[l][i]) * float(s[l][j])
        for i in range(model.n_sites):
            tot += kt * float(s[l][i]) * float(s[(l + 1) % L][i])
    return tot


def log_weight(model, J: float, h: float, s) -> float:
    """ln omega(s) = ln phi + 2 (ln|W_f(s)| + ln|W_f(-s)|) from the stabilised
    single-flavour determinants."""
    s = np.asarray(s)
    la, sa = stable.weight(model, s)
    lb, sb = stable.weight(model, -s)
    if sa == 0 or sb == 0:
        return -math.inf
    return bare_log_weight(model, J, h, s) + 2.0 * (la + lb)


def fermion_log_weight_single_particle(model, s) -> float:
    """ln prod_f det(1 + B^f_L ... B^f_1) built directly from Eq. 6 on the
    4N-dimensional single-particle space (index (lambda, sigma, site)): the
    hopping acts within each layer and spin, the coupling is
    -xi s (sigma^z_1 - sigma^z_2).  Dense 4N x 4N matrices, no use of the
    flavour factorisation."""
    n, L = model.n_sites, model.n_slices
    k1 = hopping_matrix(model.lx, model.ly, model.t, model.mu)
    k = np.kron(np.eye(4), k1)                     # (lambda, sigma) blocks
    w, q = np.linalg.eigh(k)
    e = (q * np.exp(-model.dtau * w)) @ q.T
    sz = [(1, 1.0), (1, -1.0), (2, 1.0), (2, -1.0)]  # (layer, sigma) of the four blocks
    prod = np.eye(4 * n)
    for l in range(1, L + 1):
        v = np.zeros(4 * n)
        for blk, (lam, sig) in enumerate(sz):
            sig1 = sig if lam == 1 else 0.0
            sig2 = sig if lam == 2 else 0.0
            v[blk * n:(blk + 1) * n] = -model.xi * np.asarray(s[l - 1], dtype=np.float64) * (sig1 - sig2)
        prod = e @ np.diag(np.exp(-model.dtau * v)) @ prod
    sign, logdet = np.linalg.slogdet(np.eye(4 * n) + prod)
    assert sign > 0
    return float(logdet)


def fermion_weight_fock(model, s) -> float:
    """prod_f det(1 + B^f ...) as the many-body trace over the 2^(4N) Fock
    states of the four flavours (Jordan-Wigner operators), for N <= 2."""
    from .fock import annihilators
    n, L = model.n_sites, model.n_slices
    modes = 4 * n
    c = annihilators(modes)
    cd = [m.T for m in c]
    k1 = hopping_matrix(model.lx, model.ly, model.t, model.mu)
    hk = np.zeros((2 ** modes, 2 ** modes))
    for blk in range(4):
        for i in range(n):
            for j in range(n):
                if k1[i, j] != 0.0:
                    hk += k1[i, j] * cd[blk * n + i] @ c[blk * n + j]
    w, q = np.linalg.eigh(hk)
    ek = (q * np.exp(-model.dtau * w)) @ q.T
    num = [np.diag(cd[m] @ c[m]) for m in range(modes)]
    sigz = [1.0, -1.0, 1.0, -1.0]
    layer = [1, 1, 2, 2]
    u = np.eye(2 ** modes)
    for l in range(1, L + 1):
        hv = np.zeros(2 ** modes)
        for blk in range(4):
            sign_layer = 1.0 if layer[blk] == 1 else -1.0
            for i in range(n):
                hv += -model.xi * float(s[l - 1][i]) * sigz[blk] * sign_layer * num[blk * n + i]
        u = ek @ (np.exp(-model.dtau * hv)[:, None] * u)
    return float(np.trace(u))


def green_pair(model, s):
    """(G^a, G^b): Green's functions of the fields s and -s (chain B_L ... B_1)."""
    s = np.asarray(s)
    _, _, ga = stable.green(model, s)
    _, _, gb = stable.green(model, -s)
    return ga, gb


def sweep(model, J: float, h: float, s, ga, gb, logw, *, seed: int, sweep_index: int, chain: int = 0,
          want_trace=False):
    """One local-update sweep of the bilayer weight, in place on s, ga, gb.
    Sites ascending within slices 1..L; u = Philox (seed, TAG_LOCAL) at counter
    (i, l-1, sweep, chain); recompute of both G every n_stab slices.  Returns
    (logw, accepts, max_drift[, trace])."""
    e, einv = kinetic_propagators(model.lx, model.ly, model.t, model.mu, model.dtau)
    n, L = model.n_sites, model.n_slices
    a = model.dtau * model.xi
    kt = bare_coupling(model.dtau, h)
    nbr = [[] for _ in range(n)]
    for i, j in bonds(model.lx, model.ly):
        nbr[i].append(j)
        nbr[j].append(i)
    accepts, drift = 0, 0.0
    trace = [] if want_trace else None
    key = (seed, TAG_LOCAL)
    for l in range(1, L + 1):
        for i in range(n):
            si = float(s[l - 1, i])
            hloc = model.dtau * J * sum(float(s[l - 1, j]) for j in nbr[i]) + \
                kt * (float(s[l % L, i]) + float(s[(l - 2) % L, i]))
            bare = math.exp(-2.0 * si * hloc)
            da = math.exp(2.0 * a * si) - 1.0
            db = math.exp(-2.0 * a * si) - 1.0
            ra = 1.0 + da * (1.0 - ga[i, i])
            rb = 1.0 + db * (1.0 - gb[i, i])
            r = bare * (ra * rb) ** 2
            u = uniform((i, l - 1, sweep_index, chain), key)
            acc = u < r
            if want_trace:
                trace.append((l, i, r, u, acc))
            if acc:
                for g, dd, rr in ((ga, da, ra), (gb, db, rb)):
                    col = -g[:, i].copy()
                    col[i] += 1.0
                    g -= (dd / rr) * np.outer(col, g[i, :])
                s[l - 1, i] = -s[l - 1, i]
                logw += math.log(r)
                accepts += 1
        for g, sgn in ((ga, 1), (gb, -1)):
            d = field_diagonal(sgn * s[l - 1], model.dtau, model.xi)
            g[:, :] = e @ ((d[:, None] * g) / d[None, :]) @ einv
        if l % model.n_stab == 0:
            for g, sgn in ((ga, 1), (gb, -1)):
                fresh = stable.green_at_slice(model, sgn * s, l)
                drift = max(drift, float(np.max(np.abs(g - fresh))))
                g[:, :] = fresh
    if want_trace:
        return logw, accepts, drift, trace
    return logw, accepts, drift
