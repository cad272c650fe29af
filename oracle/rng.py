"""Counter-based random numbers for the VMC step, written from the published
definition of Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11).

TEST INFRASTRUCTURE ONLY (the library has its own HIP implementation; the two
are compared bit for bit on the 32-bit outputs).

Stream layout shared with the library (an interface, not arithmetic of the
method): element pair i of stream `stream_id` at step `step` is drawn from
counter (i, stream_id, step_lo, step_hi) under key (seed_lo, seed_hi); the four
32-bit outputs (x0, x1, x2, x3) give two doubles in (0, 1),
    u = (x0 * 2^20 + (x1 >> 12) + 1/2) / 2^52,   u' = the same from (x2, x3),
which are the two uniforms of the pair, or, through Box-Muller
(sqrt(-2 ln u) cos(2 pi u'), sqrt(-2 ln u) sin(2 pi u')), two standard normals.
"""
from __future__ import annotations

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """ctr: 4 uint32 (array-like, broadcastable), key: 2 uint32 -> 4 uint32 arrays."""
    c = [np.asarray(x, dtype=np.uint64) & MASK for x in ctr]
    k0 = np.asarray(key[0], dtype=np.uint64) & MASK
    k1 = np.asarray(key[1], dtype=np.uint64) & MASK
    for r in range(10):
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        hi0, lo0 = (p0 >> 32) & MASK, p0 & MASK
        hi1, lo1 = (p1 >> 32) & MASK, p1 & MASK
        c = [(hi1 ^ c[1] ^ k0) & MASK, lo1, (hi0 ^ c[3] ^ k1) & MASK, lo0]
        if r < 9:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
    return [x.astype(np.uint32) for x in c]


def to_unit(a, b):
    """Two uint32 -> one double in (0, 1) from 52 of their bits (m + 1/2 is exact,
    so the result is never 0 or 1)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    m = (a << np.uint64(20)) | (b >> np.uint64(12))          # 52 bits
    return (m.astype(np.float64) + 0.5) * 2.0 ** -52


def _counters(n_pairs, stream_id, step):
    i = np.arange(n_pairs, dtype=np.uint64)
    return [i & MASK, np.full(n_pairs, stream_id & MASK, dtype=np.uint64),
            np.full(n_pairs, step & MASK, dtype=np.uint64),
            np.full(n_pairs, (step >> 32) & MASK, dtype=np.uint64)]


def uniforms(seed, stream_id, step, n):
    """n doubles in (0, 1): element 2i and 2i+1 from counter pair i."""
    n_pairs = (n + 1) // 2
    x = philox4x32_10(_counters(n_pairs, stream_id, step), (seed & MASK, (seed >> 32) & MASK))
    u = np.empty(2 * n_pairs)
    u[0::2] = to_unit(x[0], x[1])
    u[1::2] = to_unit(x[2], x[3])
    return u[:n]


def normals(seed, stream_id, step, n):
    """n standard normals by Box-Muller on the pairs of `uniforms`."""
    n_pairs = (n + 1) // 2
    x = philox4x32_10(_counters(n_pairs, stream_id, step), (seed & MASK, (seed >> 32) & MASK))
    u1 = to_unit(x[0], x[1])
    u2 = to_unit(x[2], x[3])
    r = np.sqrt(-2.0 * np.log(u1))
    t = 2.0 * np.pi * u2
    z = np.empty(2 * n_pairs)
    z[0::2] = r * np.cos(t)
    z[1::2] = r * np.sin(t)
    return z[:n]
