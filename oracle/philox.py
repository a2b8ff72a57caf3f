"""Counter-based Gaussian numbers for the randomized schemes (oracle, test infrastructure).

The randomized low-rank approximation of Section 4 (Algorithms 8 and 9) and the
random start vector of the Lanczos bidiagonalization (Algorithm 7) draw Gaussian
vectors. The oracle must see the same draws as the library, so both sides
implement one published generator, each in its own code:

  * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
    as 1, 2, 3", SC 2011): 10 rounds over a 4 x 32-bit counter and a 2 x 32-bit
    key, round multipliers 0xD2511F53 / 0xCD9E8D57, key increments (Weyl
    constants) 0x9E3779B9 / 0xBB67AE85;
  * the Box-Muller transform (Box and Muller, 1958), first of the pair.

Convention of the Gaussian matrix Omega (rows = point positions in cluster
order, columns = draws): entry (i, j) takes the counter
(i mod 2^32, j, i div 2^32, 0x0A11CE5) and the key (seed mod 2^32, seed div 2^32).
From the output words (x, y, z, w): a = ((x << 21) xor (y >> 11)) mod 2^53 and
b likewise from (z, w); u1 = (a + 1) 2^-53 in (0, 1], u2 = b 2^-53 in [0, 1);
the entry is sqrt(-2 ln u1) cos(2 pi u2).
"""

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK32 = 0xFFFFFFFF
OMEGA_TAG = 0x0A11CE5


def philox4x32_10(ctr, key):
    """ctr: uint64 array (..., 4) of 32-bit words; key: (k0, k1). Returns (..., 4) uint64."""
    c = np.array(ctr, dtype=np.uint64) & np.uint64(MASK32)
    k0, k1 = np.uint64(key[0] & MASK32), np.uint64(key[1] & MASK32)
    x, y, z, w = c[..., 0], c[..., 1], c[..., 2], c[..., 3]
    for _ in range(10):
        p0 = np.uint64(M0) * x  # < 2^64: exact in uint64
        p1 = np.uint64(M1) * z
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK32)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK32)
        x, y, z, w = hi1 ^ y ^ k0, lo1, hi0 ^ w ^ k1, lo0
        k0 = (k0 + np.uint64(W0)) & np.uint64(MASK32)
        k1 = (k1 + np.uint64(W1)) & np.uint64(MASK32)
    return np.stack([x, y, z, w], axis=-1)


def gaussian_from_words(r):
    """Box-Muller of one Philox output block (..., 4) -> float64 (...)."""
    r = np.asarray(r, dtype=np.uint64)
    m53 = np.uint64((1 << 53) - 1)
    a = ((r[..., 0] << np.uint64(21)) ^ (r[..., 1] >> np.uint64(11))) & m53
    b = ((r[..., 2] << np.uint64(21)) ^ (r[..., 3] >> np.uint64(11))) & m53
    u1 = (a.astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = b.astype(np.float64) * 2.0 ** -53
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def omega(rows, cols, seed):
    """Omega[rows, cols] as a (len(rows), len(cols)) float64 matrix."""
    i = np.asarray(rows, dtype=np.uint64)[:, None]
    j = np.asarray(cols, dtype=np.uint64)[None, :]
    i, j = np.broadcast_arrays(i, j)
    ctr = np.stack([i & np.uint64(MASK32), j, i >> np.uint64(32),
                    np.full(i.shape, OMEGA_TAG, dtype=np.uint64)], axis=-1)
    return gaussian_from_words(philox4x32_10(ctr, (int(seed) & MASK32, (int(seed) >> 32) & MASK32)))
