"""Philox4x32-10 counter-based generator (test infrastructure only).

Written from its published definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC'11): a 4 x 32-bit counter and 2 x 32-bit key; each of the 10 rounds multiplies
counter words 0 and 2 by 0xD2511F53 and 0xCD9E8D57, and outputs
    (hi(M1 c2) ^ c1 ^ k0,  lo(M1 c2),  hi(M0 c0) ^ c3 ^ k1,  lo(M0 c0));
the key is bumped by the Weyl constants (0x9E3779B9, 0xBB67AE85) between rounds.

Toy generation uses it so that the library's generator can be compared draw for draw:
candidate i, stream s -> counter (i mod 2^32, i div 2^32, s, 0), key (seed mod 2^32, seed div 2^32).
A uniform double in [0, 1) is built from two words as ((w_a >> 5) * 2^26 + (w_b >> 6)) * 2^-53.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised over counter arrays; returns four uint32 arrays."""
    c = [np.asarray(x, dtype=np.uint64) & MASK for x in (c0, c1, c2, c3)]
    k0 = int(k0) & 0xFFFFFFFF
    k1 = int(k1) & 0xFFFFFFFF
    for rnd in range(10):
        if rnd:
            k0 = (k0 + W0) & 0xFFFFFFFF
            k1 = (k1 + W1) & 0xFFFFFFFF
        p0 = c[0] * M0
        p1 = c[2] * M1
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c = [hi1 ^ c[1] ^ np.uint64(k0), lo1, hi0 ^ c[3] ^ np.uint64(k1), lo0]
    return tuple(x.astype(np.uint32) for x in c)


def to_unit(wa, wb):
    a = np.asarray(wa, dtype=np.uint64) >> np.uint64(5)
    b = np.asarray(wb, dtype=np.uint64) >> np.uint64(6)
    return (a.astype(np.float64) * 67108864.0 + b.astype(np.float64)) * (1.0 / 9007199254740992.0)


def candidate_uniforms(seed: int, first: int, count: int):
    """(u12, u13, v) for candidates first .. first+count-1."""
    idx = np.arange(first, first + count, dtype=np.uint64)
    lo = idx & MASK
    hi = idx >> np.uint64(32)
    zero = np.zeros_like(idx)
    k0, k1 = seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF
    w = philox4x32_10(lo, hi, zero, zero, k0, k1)
    v = philox4x32_10(lo, hi, zero + np.uint64(1), zero, k0, k1)
    return to_unit(w[0], w[1]), to_unit(w[2], w[3]), to_unit(v[0], v[1])
