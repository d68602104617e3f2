"""Starting points drawn by the library when the caller passes none.

Test infrastructure (oracle): plain, slow, obviously correct.

The paper draws x^0 uniformly from [0,1]^n (App. C) without naming a
generator.  When no x0 is given, the library uses the counter-based generator
Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC 2011), written here from that published definition:

  * a round maps the counter (c0, c1, c2, c3) under the key (k0, k1) to
    (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)), with the
    multipliers M0 = 0xD2511F53 and M1 = 0xCD9E8D57 and hi/lo the upper and lower
    32 bits of the 64-bit product;
  * ten rounds, the key raised by the Weyl constants (0x9E3779B9, 0xBB67AE85)
    modulo 2^32 between consecutive rounds.

The library's mapping to starting points (a reading of its own): key =
(seed mod 2^32, seed div 2^32); coordinate i of restart b is word i mod 4 of
the output for the counter (i div 4, b, 0, 0), and x = (word >> 8) * 2^-24, a
multiple of 2^-24 in [0, 1) that float32 and float64 hold exactly.
"""
from __future__ import annotations

import numpy as np

__all__ = ["philox4x32_10", "x0_philox"]

_M0, _M1 = 0xD2511F53, 0xCD9E8D57
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds on arrays of counters.  ctr: four uint32 arrays
    (or ints) of one shape; key: two uint32 values.  Returns four uint32 arrays."""
    c = [np.asarray(v, dtype=np.uint64) & _MASK for v in ctr]
    k0, k1 = int(key[0]) & _MASK, int(key[1]) & _MASK
    for r in range(10):
        if r:
            k0, k1 = (k0 + _W0) & _MASK, (k1 + _W1) & _MASK
        p0 = c[0] * np.uint64(_M0)   # exact: both factors are below 2^32
        p1 = c[2] * np.uint64(_M1)
        c = [(p1 >> np.uint64(32)) ^ c[1] ^ np.uint64(k0), p1 & np.uint64(_MASK),
             (p0 >> np.uint64(32)) ^ c[3] ^ np.uint64(k1), p0 & np.uint64(_MASK)]
    return [v.astype(np.uint32) for v in c]


def x0_philox(seed: int, B: int, n: int) -> np.ndarray:
    """(B, n) float64 starting points of the library's generator for `seed`."""
    i = np.arange(n, dtype=np.uint64)[None, :].repeat(B, 0)
    b = np.arange(B, dtype=np.uint64)[:, None].repeat(n, 1)
    z = np.zeros_like(i)
    words = philox4x32_10((i >> np.uint64(2), b, z, z), (seed & _MASK, (seed >> 32) & _MASK))
    sel = (i & np.uint64(3)).astype(np.int64)
    w = np.choose(sel, words)
    return (w >> np.uint32(8)).astype(np.float64) * 2.0 ** -24
