"""Random words and uniforms (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

The paper leaves the engine's random numbers unspecified (its Monte Carlo
engine is an external one).  This build fixes:

* Philox4x32-10, the counter-based generator of Salmon, Moraes, Dror and
  Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11): a 4x32-bit
  counter and a 2x32-bit key, ten rounds, each round two 32x32->64-bit
  multiplications by the published multipliers, a swap-and-xor with the key,
  and a Weyl-sequence key bump between rounds.
* Stream layout: the key is (seed mod 2^32, seed div 2^32).  A path's random
  words are numbered w = slot * A + asset (A = number of assets); word w is
  element w mod 4 of the Philox block with counter
  (path, w div 4, instance, 0).
* Sobol: unscrambled Sobol points with the Joe-Kuo direction numbers, in
  Gray-code order, as scipy.stats.qmc.Sobol generates them; path i is point
  i (point 0 included); dimension w = slot * A + asset.
* Uniform maps onto exact dyadic rationals inside (0, 1):
  FP64 paths use u = (x + 1/2) 2^-32; FP32 paths use u = (x>>9 + 1/2) 2^-23
  = (2 (x>>9) + 1) 2^-24, an odd multiple of 2^-24 below 1, so it is exact in
  binary32 as well as in binary64.
"""
from __future__ import annotations

import numpy as np

MASK32 = 0xFFFFFFFF
PHILOX_M0, PHILOX_M1 = 0xD2511F53, 0xCD9E8D57     # round multipliers
PHILOX_W0, PHILOX_W1 = 0x9E3779B9, 0xBB67AE85     # key-schedule (Weyl) increments
PHILOX_ROUNDS = 10


def philox4x32_10(ctr, key):
    """One Philox4x32-10 block, plain Python integers.

    ctr = (c0, c1, c2, c3), key = (k0, k1); returns the 4 output words.
    """
    c0, c1, c2, c3 = (int(x) & MASK32 for x in ctr)
    k0, k1 = (int(x) & MASK32 for x in key)
    for _ in range(PHILOX_ROUNDS):
        p0 = PHILOX_M0 * c0                 # 64-bit products
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> 32, p0 & MASK32
        hi1, lo1 = p1 >> 32, p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & MASK32, lo1, (hi0 ^ c3 ^ k1) & MASK32, lo0
        k0 = (k0 + PHILOX_W0) & MASK32
        k1 = (k1 + PHILOX_W1) & MASK32
    return c0, c1, c2, c3


def philox4x32_10_np(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10 over numpy arrays of counters (uint64 math)."""
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) & np.uint64(MASK32) for x in (c0, c1, c2, c3))
    k0 = np.uint64(int(k0) & MASK32)
    k1 = np.uint64(int(k1) & MASK32)
    m32 = np.uint64(MASK32)
    s32 = np.uint64(32)
    for _ in range(PHILOX_ROUNDS):
        p0 = np.uint64(PHILOX_M0) * c0
        p1 = np.uint64(PHILOX_M1) * c2
        n0 = ((p1 >> s32) ^ c1 ^ k0) & m32
        n1 = p1 & m32
        n2 = ((p0 >> s32) ^ c3 ^ k1) & m32
        n3 = p0 & m32
        c0, c1, c2, c3 = n0, n1, n2, n3
        k0 = np.uint64((int(k0) + PHILOX_W0) & MASK32)
        k1 = np.uint64((int(k1) + PHILOX_W1) & MASK32)
    return tuple(x.astype(np.uint32) for x in (c0, c1, c2, c3))


def seed_key(seed: int):
    seed = int(seed)
    return seed & MASK32, (seed >> 32) & MASK32


def philox_path_words(path: int, n_words: int, instance: int = 0, seed: int = 42):
    """Random words 0..n_words-1 of one path (plain Python, small cases)."""
    key = seed_key(seed)
    out = []
    for blk in range((n_words + 3) // 4):
        out.extend(philox4x32_10((path, blk, instance, 0), key))
    return out[:n_words]


def philox_words(paths, n_words: int, instance: int = 0, seed: int = 42):
    """uint32 array [len(paths), n_words] of the paths' random words."""
    paths = np.asarray(paths, dtype=np.uint64)
    k0, k1 = seed_key(seed)
    nblk = (n_words + 3) // 4
    out = np.zeros((paths.size, nblk * 4), dtype=np.uint32)
    for blk in range(nblk):
        w = philox4x32_10_np(paths, np.full_like(paths, blk), np.full_like(paths, instance),
                             np.zeros_like(paths), k0, k1)
        for j in range(4):
            out[:, 4 * blk + j] = w[j]
    return out[:, :n_words]


def sobol_words(paths, n_dims: int):
    """uint32 array [len(paths), n_dims]: Sobol points (scipy, unscrambled,
    Gray-code order) at the given point indices, as 32-bit integers."""
    from scipy.stats import qmc

    paths = np.asarray(paths, dtype=np.int64)
    if paths.size == 0:
        return np.zeros((0, n_dims), dtype=np.uint32)
    hi = int(paths.max()) + 1
    eng = qmc.Sobol(d=n_dims, scramble=False, bits=32)
    pts = eng.random(hi)                       # points 0 .. hi-1, exact dyadics
    ints = np.ldexp(pts, 32).astype(np.uint64)  # exact: k / 2^32 -> k
    return ints[paths].astype(np.uint32)


def uniform_f64(x):
    """u = (x + 1/2) 2^-32 for 32-bit words x (exact in binary64)."""
    return np.ldexp(np.asarray(x, dtype=np.float64) + 0.5, -32)


def uniform_f32(x):
    """u = (x>>9 + 1/2) 2^-23 (exact in binary32 and binary64)."""
    hi = (np.asarray(x, dtype=np.uint64) >> np.uint64(9)).astype(np.float64)
    return np.ldexp(hi + 0.5, -23)
