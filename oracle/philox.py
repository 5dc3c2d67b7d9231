"""Philox4x64-10 counter-based generator, written from its published definition
(J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random numbers:
as easy as 1, 2, 3", SC'11).  Pure-Python integers; test infrastructure only.

The paper does not say which random numbers it draws; the convention here
(shared with the GPU side, which implements the same definition independently):

    key = (seed, stream_tag), counter = 4 x uint64 chosen per decision,
    uniform u = (word0 >> 11) * 2^-53 in [0, 1),
    small integer in [0, n) = ((word0 >> 32) * n) >> 32.
"""
from __future__ import annotations

MASK64 = (1 << 64) - 1
# Round multipliers and Weyl key increments of Philox4x64.
MUL0 = 0xD2E7470EE14C6C93
MUL1 = 0xCA5A826395121157
WEYL0 = 0x9E3779B97F4A7C15
WEYL1 = 0xBB67AE8584CAA73B

TAG_LOCAL = 1        # local DQMC flip acceptance
TAG_EFFECTIVE = 2    # colour-class choice and effective-model Metropolis
TAG_CUMULATIVE = 3   # cumulative-update acceptance


def philox4x64_10(ctr, key):
    """Ten Philox rounds on a 4-word counter with a 2-word key."""
    c0, c1, c2, c3 = (int(v) & MASK64 for v in ctr)
    k0, k1 = (int(v) & MASK64 for v in key)
    for r in range(10):
        if r:
            k0 = (k0 + WEYL0) & MASK64
            k1 = (k1 + WEYL1) & MASK64
        p0 = MUL0 * c0
        p1 = MUL1 * c2
        c0, c1, c2, c3 = ((p1 >> 64) ^ c1 ^ k0, p1 & MASK64,
                          (p0 >> 64) ^ c3 ^ k1, p0 & MASK64)
    return c0, c1, c2, c3


def uniform(ctr, key) -> float:
    """53-bit uniform double in [0, 1) from the first output word."""
    return (philox4x64_10(ctr, key)[0] >> 11) * (2.0 ** -53)


def below(n: int, ctr, key) -> int:
    """Integer in [0, n) by 32-bit multiply-shift of the first output word."""
    return ((philox4x64_10(ctr, key)[0] >> 32) * int(n)) >> 32
