"""Seeded synthetic inputs shared by the HIP path's tests/bench and by the oracle.

This module holds workload descriptions (lattice sizes, couplings, slice counts)
and seeded generators of Ising auxiliary fields.  It contains none of the
method's arithmetic: no hopping matrix, no propagator, no determinant, no
effective action.  Everything here is plain parameter bookkeeping and draws
from ``numpy.random.Generator(Philox(key))``.

Field layout everywhere: int8 array ``s[l-1, i]`` for time slice ``l = 1..L``
and site ``i = x + Lx*y`` (slice-major), values +1/-1.
"""
from __future__ import annotations

from dataclasses import dataclass, asdict, replace
import numpy as np


@dataclass(frozen=True)
class Model:
    """Single-flavour lattice fermions coupled to an Ising field.

    lx, ly      periodic square lattice, N = lx*ly sites
    n_slices    number of imaginary-time slices L (L*dtau = beta)
    t, mu       nearest-neighbour hopping and chemical potential
    dtau, xi    slice width and Ising-fermion coupling
    n_stab      slices multiplied between two QR stabilisations
    """

    lx: int
    ly: int
    n_slices: int
    t: float = 1.0
    mu: float = 0.0
    dtau: float = 0.1
    xi: float = 1.0
    n_stab: int = 10

    @property
    def n_sites(self) -> int:
        return self.lx * self.ly

    @property
    def beta(self) -> float:
        return self.n_slices * self.dtau

    def with_(self, **kw) -> "Model":
        return replace(self, **kw)

    def asdict(self) -> dict:
        return asdict(self)


# The five workloads.  The ones that leave t, mu or the stabilisation interval
# unstated use t=1, mu=-0.5, n_stab=10 (the values of the 20x20 workload).
SMALL_4x4 = Model(4, 4, 20, t=1.0, mu=0.0, dtau=0.1, xi=1.0, n_stab=10)
DQMC_20x20 = Model(20, 20, 80, t=1.0, mu=-0.5, dtau=0.1, xi=1.5, n_stab=10)
MIXED_40x40 = Model(40, 40, 100, t=1.0, mu=-0.5, dtau=0.1, xi=1.5, n_stab=10)
LEARNED_48x48 = Model(48, 48, 100, t=1.0, mu=-0.5, dtau=0.1, xi=1.5, n_stab=10)

# The paper's own workload ("Results"): bilayer, beta = 1, dtau = 0.05 (M = 20
# slices), xi = 1, at the finite-temperature critical field h = 2.774 quoted
# for J = 1.  t and mu are not given; t = 1, mu = -0.5 as elsewhere here.
BILAYER_J = 1.0
BILAYER_H = 2.774


def bilayer_model(linear: int, n_stab: int = 10) -> "Model":
    """linear x linear layers, L = 20 slices of dtau = 0.05, xi = 1."""
    return Model(linear, linear, 20, t=1.0, mu=-0.5, dtau=0.05, xi=1.0, n_stab=n_stab)


WORKLOADS = {
    "small_4x4": SMALL_4x4,
    "dqmc_20x20": DQMC_20x20,
    "mixed_40x40": MIXED_40x40,
    "learned_48x48": LEARNED_48x48,
}


def rng(key: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=key))


def iid_field(model: Model, key: int) -> np.ndarray:
    """Independent uniform +-1 spins, int8 [L][N]."""
    g = rng(key)
    return (2 * g.integers(0, 2, size=(model.n_slices, model.n_sites)) - 1).astype(np.int8)


def iid_fields(model: Model, count: int, key: int) -> np.ndarray:
    """``count`` independent iid fields, int8 [count][L][N]."""
    g = rng(key)
    return (2 * g.integers(0, 2, size=(count, model.n_slices, model.n_sites)) - 1).astype(np.int8)


def domain_field(model: Model, key: int, flip_p: float = 0.10) -> np.ndarray:
    """Two ordered spatial domains split by a straight wall along x, constant in
    imaginary time, random overall sign, then each spin flipped with prob flip_p."""
    g = rng(key)
    wall = int(g.integers(1, model.lx))
    sgn = 1 if g.integers(0, 2) else -1
    x = np.arange(model.n_sites) % model.lx
    base = np.where(x < wall, sgn, -sgn).astype(np.int8)
    s = np.broadcast_to(base, (model.n_slices, model.n_sites)).copy()
    flips = g.random((model.n_slices, model.n_sites)) < flip_p
    s[flips] = -s[flips]
    return s


def mixed_batch(model: Model, count: int, key: int) -> np.ndarray:
    """Half iid fields, half ordered-domain fields with 10% flips."""
    half = count // 2
    out = np.empty((count, model.n_slices, model.n_sites), np.int8)
    for b in range(count):
        out[b] = iid_field(model, key + b) if b < half else domain_field(model, key + b)
    return out


def uneven_models(count: int = 64, key: int = 4000, base: Model | None = None) -> list[Model]:
    """Chains of uneven size: Lx=Ly drawn from {8,12,16,20,24}, L from {40,60,80,100}."""
    base = base or Model(8, 8, 40, t=1.0, mu=-0.5, dtau=0.1, xi=1.5, n_stab=10)
    out = []
    for c in range(count):
        g = rng(key + c)
        lin = int(g.choice([8, 12, 16, 20, 24]))
        ls = int(g.choice([40, 60, 80, 100]))
        out.append(base.with_(lx=lin, ly=lin, n_slices=ls))
    return out


def default_terms(n_slices: int) -> list[tuple[int, int]]:
    """Terms (spatial shell r, time separation dl) of the effective action: the
    one-body term (0, 0), then 2 spatial, L/2 temporal and 4 space-time
    couplings (1 + 16 at L=20)."""
    return ([(0, 0), (1, 0), (2, 0)] + [(0, dl) for dl in range(1, n_slices // 2 + 1)]
            + [(1, 1), (1, 2), (2, 1), (2, 2)])


NET_PARAMS = 8 * 27 + 8 + 8 * 8 * 27 + 8 + 8 + 1


def net_init(key: int, scale: float = 1.0) -> np.ndarray:
    """Seeded initial parameters of the learned action's network (1969 FP64
    values in the order W1, b1, W2, b2, w3, b3): normal weights with fan-in
    scaling, zero biases, small readout weights."""
    g = rng(key)
    w1 = g.normal(scale=scale / np.sqrt(27.0), size=8 * 27)
    w2 = g.normal(scale=scale / np.sqrt(8 * 27.0), size=8 * 8 * 27)
    w3 = g.normal(scale=0.01, size=8)
    return np.concatenate([w1, np.zeros(8), w2, np.zeros(8), w3, [0.0]])
