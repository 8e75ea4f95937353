"""Counter-based Gaussian generator: the test-side reference.

TEST INFRASTRUCTURE ONLY: imported by tests/ to check the library's on-device
generator (lrpr_randn); it shares no code with it.  Both sides implement the
same published generator from its definition:

* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
  as 1, 2, 3", SC'11): a 4 x 32-bit counter and a 2 x 32-bit key; ten rounds,
  each two 32 x 32 -> 64-bit products (multipliers 0xD2511F53, 0xCD9E8D57)
  whose halves are recombined with the other counter words and the key, the
  key bumped by the Weyl constants (0x9E3779B9, 0xBB67AE85) between rounds.
* Gaussian pair j of stream s under seed k: counter (j mod 2^32, j div 2^32,
  s mod 2^32, s div 2^32), key (k mod 2^32, k div 2^32); words (x0, x1) and
  (x2, x3) give two 53-bit uniforms u = (floor((hi 2^32 + lo) / 2^11) + 1/2)
  2^-53 in (0, 1); Box-Muller: r = sqrt(-2 ln u1), elements 2j and 2j+1 are
  r cos(2 pi u2) and r sin(2 pi u2).
"""
from __future__ import annotations

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
_MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """One block: ctr 4 words, key 2 words (Python ints) -> 4 words."""
    c = [int(x) & _MASK for x in ctr]
    k0, k1 = int(key[0]) & _MASK, int(key[1]) & _MASK
    for _ in range(10):
        p0, p1 = M0 * c[0], M1 * c[2]
        c = [((p1 >> 32) ^ c[1] ^ k0) & _MASK, p1 & _MASK, ((p0 >> 32) ^ c[3] ^ k1) & _MASK, p0 & _MASK]
        k0, k1 = (k0 + W0) & _MASK, (k1 + W1) & _MASK
    return c


def _philox_vec(j, stream, seed):
    """Vectorised over pair indices j (uint64 array): returns 4 uint64 arrays of 32-bit words."""
    j = j.astype(np.uint64)
    m = np.uint64(_MASK)
    c0, c1 = j & m, j >> np.uint64(32)
    c2 = np.full_like(j, np.uint64(stream & _MASK))
    c3 = np.full_like(j, np.uint64((stream >> 32) & _MASK))
    k0, k1 = np.uint64(seed & _MASK), np.uint64((seed >> 32) & _MASK)
    for _ in range(10):
        p0, p1 = np.uint64(M0) * c0, np.uint64(M1) * c2
        c0, c1, c2, c3 = (((p1 >> np.uint64(32)) ^ c1 ^ k0) & m, p1 & m,
                          ((p0 >> np.uint64(32)) ^ c3 ^ k1) & m, p0 & m)
        k0, k1 = (k0 + np.uint64(W0)) & m, (k1 + np.uint64(W1)) & m
    return c0, c1, c2, c3


def randn(count: int, seed: int, stream: int) -> np.ndarray:
    """count standard Gaussians (FP64) of the given seed and stream."""
    npairs = (count + 1) // 2
    x0, x1, x2, x3 = _philox_vec(np.arange(npairs, dtype=np.uint64), stream, seed)
    sh = np.uint64(11)
    u1 = (((x0 << np.uint64(32)) | x1) >> sh).astype(np.float64) + 0.5
    u2 = (((x2 << np.uint64(32)) | x3) >> sh).astype(np.float64) + 0.5
    u1 *= 2.0 ** -53
    u2 *= 2.0 ** -53
    r = np.sqrt(-2.0 * np.log(u1))
    out = np.empty(2 * npairs)
    out[0::2] = r * np.cos(2.0 * np.pi * u2)
    out[1::2] = r * np.sin(2.0 * np.pi * u2)
    return out[:count]
