"""Pins for the oracle's Philox4x32-10 generator and its uniform/normal maps."""
import math
import os

import numpy as np

from oracle import philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        rows.append([int(w, 16) for w in line.split()])
    return rows


def test_known_answer_vectors():
    rows = _kat()
    assert len(rows) == 3
    for r in rows:
        out = philox.philox4x32_10(*r[:6])
        assert [int(v) for v in out] == r[6:]


def test_vectorised_matches_scalar():
    rng = np.random.default_rng(0)
    c = rng.integers(0, 2 ** 32, size=(4, 50), dtype=np.uint64)
    vec = philox.philox4x32_10(c[0], c[1], c[2], c[3], 0x1234, 0xabcdef)
    for t in range(50):
        one = philox.philox4x32_10(int(c[0, t]), int(c[1, t]), int(c[2, t]), int(c[3, t]),
                                   0x1234, 0xabcdef)
        assert [int(v[t]) for v in vec] == [int(v) for v in one]


def test_uniform53_range_is_half_open_at_zero():
    assert philox.uniform53(0, 0) == 2.0 ** -53
    assert philox.uniform53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0
    # the low 11 bits of the second word are discarded
    assert philox.uniform53(5, 0x7FF) == philox.uniform53(5, 0)


def test_normal_moments_and_uniform_histogram():
    n = 400_000
    k = np.arange(n) % 7
    p = np.arange(n) // 7
    w = philox.philox4x32_10(k, p, 3, 0, 11, 0)
    u = philox.uniform53(w[0], w[1])
    hist = np.bincount(np.minimum((u * 50).astype(int), 49), minlength=50)
    chi2 = np.sum((hist - n / 50) ** 2 / (n / 50))
    assert chi2 < 49 + 6 * math.sqrt(2 * 49)
    z1, z2 = philox.box_muller(u, philox.uniform53(w[2], w[3]))
    for z in (z1, z2):
        assert abs(z.mean()) < 5 / math.sqrt(n)
        assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / n)
    assert abs(np.mean(z1 * z2)) < 5 / math.sqrt(n)
