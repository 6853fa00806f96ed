"""Philox-4x32-10 counter-based generator (Salmon, Moraes, Dror & Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC 2011), written from its published
definition, plus the two derived variates the HMC step uses.  Test
infrastructure: the HIP library has its own implementation.

One round maps counter (c0, c1, c2, c3) and key (k0, k1) to
  (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0))
with M0 = 0xD2511F53, M1 = 0xCD9E8D57; the key is bumped by the Weyl constants
(0x9E3779B9, 0xBB67AE85) between rounds; ten rounds.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """ctr: [..., 4] uint32-valued; key: [..., 2].  Returns [..., 4] uint64 holding 32-bit words."""
    c = np.asarray(ctr, dtype=np.uint64) & MASK
    k = np.asarray(key, dtype=np.uint64) & MASK
    c0, c1, c2, c3 = c[..., 0], c[..., 1], c[..., 2], c[..., 3]
    k0, k1 = np.broadcast_to(k[..., 0], c0.shape).copy(), np.broadcast_to(k[..., 1], c0.shape).copy()
    for r in range(10):
        if r > 0:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & MASK, lo1, (hi0 ^ c3 ^ k1) & MASK, lo0
    return np.stack([c0, c1, c2, c3], axis=-1)


def _u53(a, b):
    """Uniform in [0, 1) with 53 random bits from two 32-bit words (27 + 26 bits)."""
    return ((a >> np.uint64(5)).astype(np.float64) * 67108864.0 + (b >> np.uint64(6)).astype(np.float64)) / 9007199254740992.0


def _ctr(index, stream, counter):
    index = np.asarray(index, dtype=np.uint64)
    cnt = np.uint64(counter)
    c = np.zeros(index.shape + (4,), dtype=np.uint64)
    c[..., 0] = index & MASK
    c[..., 1] = np.uint64(stream)
    c[..., 2] = cnt & MASK
    c[..., 3] = (cnt >> np.uint64(32)) & MASK
    return c


def _key(seed):
    s = np.uint64(seed)
    return np.array([s & MASK, (s >> np.uint64(32)) & MASK], dtype=np.uint64)


def normals(seed, counter, m):
    """m standard normals for one HMC iteration: element k uses counter
    (k, 0, counter_lo, counter_hi); Box-Muller on the first two 53-bit uniforms:
    sqrt(-2 log(1 - u1)) cos(2 pi u2)."""
    r = philox4x32_10(_ctr(np.arange(m), 0, counter), _key(seed))
    u1 = _u53(r[..., 0], r[..., 1])
    u2 = _u53(r[..., 2], r[..., 3])
    return np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)


def accept_uniform(seed, counter):
    """The Metropolis uniform of one iteration: counter (0, 1, counter_lo, counter_hi)."""
    r = philox4x32_10(_ctr(np.zeros(1), 1, counter), _key(seed))
    return float(_u53(r[..., 0], r[..., 1])[0])
