"""Philox4x32-10 and Box-Muller, written from their published definitions.

Philox4x32-R is the counter-based generator of Salmon, Moraes, Dror and Shaw,
"Parallel Random Numbers: As Easy as 1, 2, 3" (SC'11), Section 4: a 128-bit
counter (x0, x1, x2, x3) and a 64-bit key (k0, k1) go through R rounds of

    (hi0, lo0) = M0 * x0          (32 x 32 -> 64-bit product)
    (hi1, lo1) = M1 * x2
    (x0, x1, x2, x3) <- (hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0)

with M0 = 0xD2511F53, M1 = 0xCD9E8D57, and between rounds the key is bumped by
the Weyl constants (0x9E3779B9, 0xBB67AE85) modulo 2^32.  R = 10 here.

Box-Muller (Box and Muller, 1958) maps two uniforms u1, u2 in (0, 1] to two
independent standard normals sqrt(-2 ln u1) * (cos 2 pi u2, sin 2 pi u2).

Everything is vectorised over numpy uint32 arrays; products are formed in uint64.
"""

from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32(counter, key, rounds: int = 10):
    """Philox4x32-`rounds`.  counter: 4 uint32 arrays (broadcastable); key: 2 ints/arrays.

    Returns four uint32 arrays."""
    x = [np.asarray(c, dtype=np.uint64) & MASK32 for c in counter]
    x = np.broadcast_arrays(*x)
    x = [a.copy() for a in x]
    k0 = np.uint64(int(key[0]) & 0xFFFFFFFF)
    k1 = np.uint64(int(key[1]) & 0xFFFFFFFF)
    for r in range(rounds):
        if r > 0:
            k0 = np.uint64((int(k0) + W0) & 0xFFFFFFFF)
            k1 = np.uint64((int(k1) + W1) & 0xFFFFFFFF)
        p0 = M0 * x[0]
        p1 = M1 * x[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        x = [hi1 ^ x[1] ^ k0, lo1, hi0 ^ x[3] ^ k1, lo0]
    return [a.astype(np.uint32) for a in x]


def uniform_open(bits) -> np.ndarray:
    """Uniform in (0, 1) from a uint32: (2 * (bits >> 9) + 1) * 2^-24.

    The top 23 bits are kept so the value is exactly representable in binary32
    as well as binary64: both precisions then start from the same uniform."""
    b = np.asarray(bits, dtype=np.uint32).astype(np.float64)
    top = np.floor(b / 512.0)
    return (2.0 * top + 1.0) * (2.0 ** -24)


def box_muller(bits_a, bits_b):
    """Two standard normals (a, b) from two uint32 words, in float64."""
    u1 = uniform_open(bits_a)
    u2 = uniform_open(bits_b)
    rho = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * np.pi * u2
    return rho * np.cos(ang), rho * np.sin(ang)
