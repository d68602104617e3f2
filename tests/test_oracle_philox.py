"""The oracle's Philox4x32-10 against the published known-answer vectors, and
its mapping to starting points against the stated rule, element by element."""
import json
import os

import numpy as np

from oracle.philox import philox4x32_10, x0_philox

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.json")


def test_known_answer_vectors():
    for v in json.load(open(GOLD))["vectors"]:
        ctr = [int(h, 16) for h in v["ctr"]]
        key = [int(h, 16) for h in v["key"]]
        out = philox4x32_10(ctr, key)
        assert [int(w) for w in out] == [int(h, 16) for h in v["out"]]


def test_vectorised_equals_scalar_and_counter_independence():
    """Array counters give each lane exactly its scalar result (no mixing
    between lanes), and changing one counter word changes the output."""
    rng = np.random.default_rng(0)
    ctr = [rng.integers(0, 2 ** 32, size=7, dtype=np.uint64) for _ in range(4)]
    key = (0x12345678, 0x9ABCDEF0)
    out = philox4x32_10(ctr, key)
    for j in range(7):
        s = philox4x32_10([int(c[j]) for c in ctr], key)
        assert [int(w) for w in s] == [int(o[j]) for o in out]
    a = philox4x32_10((1, 2, 3, 4), key)
    b = philox4x32_10((1, 2, 3, 5), key)
    assert [int(w) for w in a] != [int(w) for w in b]


def test_x0_mapping():
    seed, B, n = 0x0123456789ABCDEF, 3, 11
    X = x0_philox(seed, B, n)
    assert X.shape == (B, n) and np.all((X >= 0) & (X < 1))
    for b in range(B):
        for i in range(n):
            w = philox4x32_10((i // 4, b, 0, 0), (seed & 0xFFFFFFFF, seed >> 32))[i % 4]
            assert X[b, i] == (int(w) >> 8) / 2.0 ** 24
    # exactly representable in float32
    assert np.array_equal(X.astype(np.float32).astype(np.float64), X)
