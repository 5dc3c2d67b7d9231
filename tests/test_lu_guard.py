"""CPU build of the LU kernel's panel-interchange bookkeeping
(paper_1612_03804_amd/csrc/lu_interchange.h, compiled here with g++).

The determinant of the final step (the O(N^3) cost the paper attributes to
"calculating the determinant") is taken from an LU factorisation with partial
pivoting.  The kernel turns a panel's sequence of row swaps into one gather:
rows srow[k] receive the entries of rows ssrc[k].  These tests check that the
gather equals the swaps applied one after another, and that a pivot index
outside [j0 + c, N) is refused (no interchange, reported) so that every row
index the gather touches stays inside the matrix.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HDR_DIR = os.path.join(os.path.dirname(HERE), "paper_1612_03804_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <cstdint>
#include <vector>
#include "lu_interchange.h"
int main() {
  int cases;
  if (scanf("%d", &cases) != 1) return 2;
  for (int t = 0; t < cases; ++t) {
    int N, j0, nbw;
    if (scanf("%d %d %d", &N, &j0, &nbw) != 3) return 2;
    std::vector<uint16_t> ipiv(N, 0);
    for (int c = 0; c < nbw; ++c) { unsigned v; if (scanf("%u", &v) != 1) return 2; ipiv[j0 + c] = (uint16_t)v; }
    std::vector<int> srow(2 * nbw, -7), ssrc(2 * nbw, -7);
    int ns = -1;
    int bad = slq::lu_panel_permutation(N, j0, nbw, ipiv.data(), srow.data(), ssrc.data(), &ns);
    printf("%d %d", bad, ns);
    for (int k = 0; k < ns; ++k) printf(" %d %d", srow[k], ssrc[k]);
    for (int c = 0; c < nbw; ++c) printf(" %d", (int)ipiv[j0 + c]);
    printf("\n");
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def driver():
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    d = tempfile.mkdtemp(prefix="lu_guard_")
    src = os.path.join(d, "drv.cpp")
    exe = os.path.join(d, "drv")
    with open(src, "w") as f:
        f.write(DRIVER)
    # the header is HIP source; on the host its attributes mean nothing
    r = subprocess.run([gxx, "-O1", "-std=c++17", "-D__host__=", "-D__device__=", "-I", HDR_DIR, src, "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def run(exe, cases):
    inp = [str(len(cases))]
    for N, j0, piv in cases:
        inp.append(f"{N} {j0} {len(piv)} " + " ".join(str(int(p)) for p in piv))
    r = subprocess.run([exe], input="\n".join(inp) + "\n", capture_output=True, text=True, check=True)
    out = []
    for line, (N, j0, piv) in zip(r.stdout.strip().split("\n"), cases):
        v = [int(x) for x in line.split()]
        bad, ns = v[0], v[1]
        pairs = v[2:2 + 2 * ns]
        srow, ssrc = pairs[0::2], pairs[1::2]
        ipiv_out = v[2 + 2 * ns:]
        out.append((bad, srow, ssrc, ipiv_out))
    return out


def swaps_applied(N, j0, piv):
    """Row order after applying the swaps (j0 + c <-> piv[c]) in sequence:
    order[r] = original row now at position r."""
    order = np.arange(N)
    for c, p in enumerate(piv):
        a = j0 + c
        order[[a, p]] = order[[p, a]]
    return order


def gather_applied(N, srow, ssrc):
    order = np.arange(N)
    new = order.copy()
    for r, src in zip(srow, ssrc):
        new[r] = order[src]
    return new


def test_gather_equals_sequential_swaps(driver):
    g = np.random.default_rng(7)
    cases = []
    for _ in range(300):
        N = int(g.integers(1, 200))
        nbw = int(g.integers(1, min(16, N) + 1))
        j0 = int(g.integers(0, N - nbw + 1))
        piv = [int(g.integers(j0 + c, N)) for c in range(nbw)]
        cases.append((N, j0, piv))
    for (N, j0, piv), (bad, srow, ssrc, ipiv_out) in zip(cases, run(driver, cases)):
        assert bad == 0 and ipiv_out == piv
        assert len(srow) <= 2 * len(piv)
        assert srow[:len(piv)] == list(range(j0, j0 + len(piv)))
        assert all(j0 <= r < N for r in srow + ssrc)
        np.testing.assert_array_equal(gather_applied(N, srow, ssrc), swaps_applied(N, j0, piv))


def test_out_of_range_pivots_are_refused(driver):
    """Pivots above the matrix (an unset 16-bit index, 65535) or above the
    diagonal are replaced by 'no interchange' and reported; the remaining
    swaps still apply exactly."""
    g = np.random.default_rng(11)
    cases, fixed = [], []
    for _ in range(300):
        N = int(g.integers(2, 200))
        nbw = int(g.integers(1, min(16, N) + 1))
        j0 = int(g.integers(0, N - nbw + 1))
        piv, ok = [], []
        for c in range(nbw):
            kind = g.integers(0, 4)
            if kind == 0:
                p = int(g.integers(N, 65536))            # beyond the last row
            elif kind == 1 and j0 + c > 0:
                p = int(g.integers(0, j0 + c))           # above the diagonal
            else:
                p = int(g.integers(j0 + c, N))
            piv.append(p)
            ok.append(p if j0 + c <= p < N else j0 + c)
        cases.append((N, j0, piv))
        fixed.append(ok)
    for (N, j0, piv), ok, (bad, srow, ssrc, ipiv_out) in zip(cases, fixed, run(driver, cases)):
        assert bad == int(ok != piv)
        assert ipiv_out == ok
        assert all(j0 <= r < N for r in srow + ssrc)
        np.testing.assert_array_equal(gather_applied(N, srow, ssrc), swaps_applied(N, j0, ok))


def test_uninitialised_panel_pivots(driver):
    """The case of a factorisation whose panel never wrote its pivots: every
    entry arbitrary.  The gather stays inside rows [j0, N)."""
    g = np.random.default_rng(3)
    cases = [(400, j0, [int(x) for x in g.integers(0, 65536, 16)]) for j0 in range(0, 384, 16)]
    for (N, j0, piv), (bad, srow, ssrc, _) in zip(cases, run(driver, cases)):
        assert bad == 1
        assert all(j0 <= r < N for r in srow + ssrc)
