"""Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller normals.

Oracle-side implementation written from the published definition of the
generator; the GPU library carries its own independent implementation.

Field layout used by both sides (the paper draws x_alpha ~ N(0,1) for every
Cholesky index, walker and step, Eq. 4-5, and requires walker k of both
systems of a pair to see the same x, Sec. II.B):

    counter = (gamma // 4, k, t, stream), key = (seed mod 2^32, seed >> 32)
    r0..r3  = Philox4x32-10(counter, key)
    u = (r0 + 1) 2^-32, v = r1 2^-32   ->  z0 = sqrt(-2 ln u) cos(2 pi v),
                                           z1 = sqrt(-2 ln u) sin(2 pi v)
    (r2, r3) give z2, z3 the same way;  x[t, k, 4b + j] = z_j.

A frozen (dead) walker simply leaves its counters unused, so the draws of all
other walker pairs are unaffected (Sec. II.B).
"""
from __future__ import annotations

import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32 with 10 rounds.  Inputs are uint32-valued arrays
    (broadcastable) and two scalar key words; returns four uint32 arrays."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & _MASK for c in (c0, c1, c2, c3))
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = np.uint64(int(k0) & 0xFFFFFFFF)
    k1 = np.uint64(int(k1) & 0xFFFFFFFF)
    for r in range(10):
        if r > 0:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> _S32, p0 & _MASK
        hi1, lo1 = p1 >> _S32, p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return tuple(c.astype(np.uint32) for c in (c0, c1, c2, c3))


def normals(seed: int, stream: int, t: int, walkers, n_chol: int) -> np.ndarray:
    """Fields x[k, gamma] for one step t, for the given walker indices."""
    walkers = np.asarray(walkers, dtype=np.uint64)
    nb = (n_chol + 3) // 4
    b = np.arange(nb, dtype=np.uint64)[None, :]
    k = walkers[:, None]
    r = philox4x32_10(b, k, np.uint64(t), np.uint64(stream), seed & 0xFFFFFFFF, seed >> 32)
    r = [x.astype(np.float64) for x in r]
    scale = 2.0 ** -32
    out = np.empty((walkers.shape[0], nb, 4))
    for pair in range(2):
        u = (r[2 * pair] + 1.0) * scale
        v = r[2 * pair + 1] * scale
        rad = np.sqrt(-2.0 * np.log(u))
        ang = 2.0 * np.pi * v
        out[:, :, 2 * pair] = rad * np.cos(ang)
        out[:, :, 2 * pair + 1] = rad * np.sin(ang)
    return out.reshape(walkers.shape[0], 4 * nb)[:, :n_chol]
