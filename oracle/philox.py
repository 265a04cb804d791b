"""Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11), vectorised over
counters with NumPy uint64 arithmetic, plus the maps the Monte Carlo
estimator uses: 53-bit uniforms on (0, 1] and the Box-Muller transform.

Stream layout for the perimeter-row estimator: key = (seed mod 2^32,
seed div 2^32); the four counter words are (step, path, knot, 0).
"""
from __future__ import annotations

import math

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)
SHIFT32 = np.uint64(32)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox rounds on 4x32-bit counters with a 2x32-bit key.

    One round: (hi0, lo0) = M0 * c0, (hi1, lo1) = M1 * c2 (full 64-bit
    products); new counter = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); the key
    is bumped by the Weyl constants between rounds.
    """
    c0 = np.asarray(c0, dtype=np.uint64) & MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & MASK32
    k0 = int(k0) & 0xFFFFFFFF
    k1 = int(k1) & 0xFFFFFFFF
    for _ in range(10):
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> SHIFT32, p0 & MASK32
        hi1, lo1 = p1 >> SHIFT32, p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                          hi0 ^ c3 ^ np.uint64(k1), lo0)
        k0 = (k0 + W0) & 0xFFFFFFFF
        k1 = (k1 + W1) & 0xFFFFFFFF
    return c0, c1, c2, c3


def uniform53(w_hi, w_lo):
    """(m + 1) 2^-53 with m = w_hi 2^21 + floor(w_lo / 2^11), exactly in (0, 1]."""
    m = (np.asarray(w_hi, dtype=np.uint64) << np.uint64(21)) | \
        (np.asarray(w_lo, dtype=np.uint64) >> np.uint64(11))
    return (m.astype(np.float64) + 1.0) * 2.0 ** -53


def box_muller(u1, u2):
    """Two independent standard normals from two uniforms on (0, 1]."""
    rad = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * math.pi * u2
    return rad * np.cos(ang), rad * np.sin(ang)


def seed_key(seed):
    seed = int(seed)
    return seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF


def normals(step, path, knot, seed):
    """The two normals a path uses at one Euler step."""
    k0, k1 = seed_key(seed)
    w0, w1, w2, w3 = philox4x32_10(step, path, knot, 0, k0, k1)
    return box_muller(uniform53(w0, w1), uniform53(w2, w3))
