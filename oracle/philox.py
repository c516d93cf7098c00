"""Philox-4x32-10 counter-based generator -- oracle, test infrastructure only.

Published definition: J. Salmon, M. Moraes, R. Dror, D. Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11.  Ten rounds of the Philox S-box on a 128-bit
counter (four 32-bit words) with a 64-bit key bumped by the Weyl constants.

Used wherever the method draws random numbers that cannot simply be passed in:
the start vector of the coarse-level Arnoldi run and the complex-normal
vectors of the training-data generation (eq. 4.3).  The GPU library implements
the same definition independently.

Mapping to floats (this build's convention, shared by both sides):
  u = (word >> 8) * 2^-24 + 2^-25      uniform in (0, 1), exactly representable
  normal pair (Box-Muller): sqrt(-2 ln u0) * (cos 2 pi u1, sin 2 pi u1)
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint32(0x9E3779B9)
W1 = np.uint32(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)


def philox4x32(counter, key):
    """counter: uint32 array [..., 4]; key: (k0, k1).  Returns uint32 [..., 4]."""
    c = np.asarray(counter, np.uint32)
    x0 = c[..., 0].astype(np.uint64)
    x1 = c[..., 1].astype(np.uint64)
    x2 = c[..., 2].astype(np.uint64)
    x3 = c[..., 3].astype(np.uint64)
    k0 = np.uint32(key[0])
    k1 = np.uint32(key[1])
    for rnd in range(10):
        p0 = M0 * x0
        p1 = M1 * x2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        n0 = hi1 ^ x1 ^ np.uint64(k0)
        n1 = lo1
        n2 = hi0 ^ x3 ^ np.uint64(k1)
        n3 = lo0
        x0, x1, x2, x3 = n0 & MASK, n1, n2 & MASK, n3
        if rnd < 9:
            k0 = np.uint32((int(k0) + int(W0)) & 0xFFFFFFFF)
            k1 = np.uint32((int(k1) + int(W1)) & 0xFFFFFFFF)
    return np.stack([x0, x1, x2, x3], axis=-1).astype(np.uint32)


def uniform01(words):
    """(0,1) floats from uint32 words: (w >> 8) * 2^-24 + 2^-25."""
    w = np.asarray(words, np.uint32)
    return (w >> np.uint32(8)).astype(np.float64) * (2.0 ** -24) + 2.0 ** -25


def stream(n, key, stream_id=0):
    """4n uint32 words for counters (i, stream_id, 0, 0), i = 0..n-1."""
    ctr = np.zeros((n, 4), np.uint32)
    ctr[:, 0] = np.arange(n, dtype=np.uint64).astype(np.uint32)
    ctr[:, 1] = np.uint32(stream_id)
    return philox4x32(ctr, key)


def complex_uniform(n, key, stream_id=0):
    """Entry i: (2 u0 - 1) + i (2 u1 - 1) from counter (i, stream_id, 0, 0)."""
    w = stream(n, key, stream_id)
    u = uniform01(w)
    return (2.0 * u[:, 0] - 1.0) + 1j * (2.0 * u[:, 1] - 1.0)


def complex_normal(n, key, stream_id=0):
    """Entry i ~ CN(0,1): Box-Muller on words 0,1 of counter (i, stream_id, 0, 0),
    each part scaled by sqrt(1/2)."""
    w = stream(n, key, stream_id)
    u = uniform01(w)
    rad = np.sqrt(-2.0 * np.log(u[:, 0])) * np.sqrt(0.5)
    ang = 2.0 * np.pi * u[:, 1]
    return rad * np.cos(ang) + 1j * rad * np.sin(ang)
