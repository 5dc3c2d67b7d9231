"""Write the stored fixtures under tests/golden/ from the oracle alone.

negative_weights_2x2_L4.json: every auxiliary field of the 2x2, L=4 lattice at
(t=1, mu=-1, dtau=1, xi=3) whose fermion weight, computed by the brute-force
Fock-space trace, is negative.  The trace runs over all 2^16 fields, batched.
Run from the repository root:  python tests/golden/make_golden.py
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import fock, lattice  # noqa: E402
from slq_inputs import Model  # noqa: E402


def all_fields(n_sites, n_slices):
    codes = np.arange(2 ** (n_sites * n_slices))
    bits = (codes[:, None] >> np.arange(n_sites * n_slices)[None, :]) & 1
    return codes, (2 * bits - 1).astype(np.int8).reshape(-1, n_slices, n_sites)


def fock_weights(model, fields):
    """Tr of the ordered slice-operator product for every field (batched)."""
    n = model.n_sites
    c = fock.annihilators(n)
    cd = [m.T for m in c]
    k = lattice.hopping_matrix(model.lx, model.ly, model.t, model.mu)
    hk = sum(k[i, j] * cd[i] @ c[j] for i in range(n) for j in range(n))
    w, q = np.linalg.eigh(hk)
    ek = (q * np.exp(-model.dtau * w)) @ q.T
    occ = np.array([[np.diag(cd[i] @ c[i])[a] for i in range(n)] for a in range(2 ** n)])  # [state][site]
    u = np.broadcast_to(np.eye(2 ** n), (len(fields), 2 ** n, 2 ** n)).copy()
    for l in range(model.n_slices):
        v = np.exp(-model.dtau * model.xi * (fields[:, l, :].astype(np.float64) @ occ.T))  # [field][state]
        u = np.einsum("ab,fb,fbc->fac", ek, v, u)
    return np.trace(u, axis1=1, axis2=2)


def main():
    model = Model(2, 2, 4, t=1.0, mu=-1.0, dtau=1.0, xi=3.0, n_stab=2)
    codes, fields = all_fields(model.n_sites, model.n_slices)
    w = np.concatenate([fock_weights(model, fields[i:i + 8192]) for i in range(0, len(fields), 8192)])
    neg = np.nonzero(w < 0)[0]
    out = {
        "source": "oracle.fock trace over all 2^16 fields; bit b of code is spin (slice b // 4, site b % 4), 1 -> +1",
        "model": model.asdict(),
        "n_fields": int(len(codes)),
        "negative_codes": [int(codes[i]) for i in neg],
        "negative_weights": [float(w[i]) for i in neg],
    }
    path = os.path.join(ROOT, "tests", "golden", "negative_weights_2x2_L4.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"{len(neg)} negative weights of {len(codes)} -> {path}")


if __name__ == "__main__":
    main()
