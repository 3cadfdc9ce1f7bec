"""Counter-based Gaussian test matrix, the oracle's own implementation.

TEST INFRASTRUCTURE ONLY (see oracle/nys_oracle.py).  The library can draw the
sketch's test matrix Omega on the device from a seed; this module computes the
same matrix on the host from the published definitions, so the two are compared
without either reading the other's numbers.

Uniform bits: Philox4x32 with 10 rounds (Salmon, Moraes, Dror and Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC 2011).  A round takes the counter
(c0, c1, c2, c3) and key (k0, k1) to
    (hi(M1 c2) xor c1 xor k0, lo(M1 c2), hi(M0 c0) xor c3 xor k1, lo(M0 c0)),
M0 = 0xD2511F53, M1 = 0xCD9E8D57, and the key grows by (0x9E3779B9, 0xBB67AE85)
after every round.
Normals: element e of the row-major n x r matrix belongs to block b = e // 2
(counter (b mod 2^32, b // 2^32, 0, 0), key (seed mod 2^32, seed // 2^32)); the
words give u = ((w0 2^32 + w1) >> 11 + 1/2) 2^-53 and v from (w2, w3) alike, and the
Box-Muller pair sqrt(-2 ln u) (cos 2 pi v, sin 2 pi v): cosine for even e, sine for
odd e.
"""
from __future__ import annotations

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(counter, key):
    """Philox4x32-10 of uint32 arrays: counter (..., 4), key (..., 2) -> (..., 4)."""
    c = [np.asarray(counter, dtype=np.uint64)[..., i].copy() for i in range(4)]
    k0 = np.asarray(key, dtype=np.uint64)[..., 0].copy()
    k1 = np.asarray(key, dtype=np.uint64)[..., 1].copy()
    for _ in range(10):
        p0 = np.uint64(M0) * c[0]
        p1 = np.uint64(M1) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK)
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
        k0 = (k0 + np.uint64(W0)) & np.uint64(MASK)
        k1 = (k1 + np.uint64(W1)) & np.uint64(MASK)
    return np.stack(c, axis=-1).astype(np.uint32)


def gaussian_test_matrix(n: int, r: int, seed: int) -> np.ndarray:
    """Omega (n x r float64) as the library draws it for a given seed."""
    count = n * r
    nb = (count + 1) // 2
    b = np.arange(nb, dtype=np.uint64)
    ctr = np.zeros((nb, 4), dtype=np.uint64)
    ctr[:, 0] = b & np.uint64(MASK)
    ctr[:, 1] = b >> np.uint64(32)
    key = np.empty((nb, 2), dtype=np.uint64)
    key[:, 0] = seed & MASK
    key[:, 1] = (seed >> 32) & MASK
    w = philox4x32_10(ctr, key).astype(np.uint64)
    xu = ((w[:, 0] << np.uint64(32)) | w[:, 1]) >> np.uint64(11)
    xv = ((w[:, 2] << np.uint64(32)) | w[:, 3]) >> np.uint64(11)
    u = (xu.astype(np.float64) + 0.5) * 2.0 ** -53
    v = (xv.astype(np.float64) + 0.5) * 2.0 ** -53
    rad = np.sqrt(-2.0 * np.log(u))
    ang = 2.0 * 3.141592653589793 * v
    z = np.empty(2 * nb)
    z[0::2] = rad * np.cos(ang)
    z[1::2] = rad * np.sin(ang)
    return z[:count].reshape(n, r)
