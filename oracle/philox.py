"""Philox4x32-10 counter-based generator (oracle; test infrastructure only).

Written from its published definition (Salmon, Moraes, Dror, Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11): a 4 x 32-bit counter and a
2 x 32-bit key; each of the 10 rounds replaces (c0, c1, c2, c3) by

    (hi(M1 c2) ^ c1 ^ k0,  lo(M1 c2),  hi(M0 c0) ^ c3 ^ k1,  lo(M0 c0))

with M0 = 0xD2511F53, M1 = 0xCD9E8D57, and the key is advanced by the Weyl
constants (0x9E3779B9, 0xBB67AE85) between rounds.

The draws the solver takes from it (a convention of this project, stated
identically in the GPU library): draw j of stream s for fit f under seed S uses
counter (j, 0, s, f) and key (S mod 2^32, S >> 32); the four output words
(x0, x1, x2, x3) give the uniform

    u = ((x0 << 32 | x1) >> 12 + 0.5) * 2^-52     in (0, 1),

and a standard normal by Box-Muller from the pair (u, u') of draws 2j, 2j+1:
sqrt(-2 ln u) cos(2 pi u').

Parity pins: the known-answer vectors in tests/golden/philox4x32_10_kat.txt;
two normals worked by hand from the first of them and the Box-Muller pairing
(tests/golden/philox_normal_box_muller.txt), which a swap of cos and sin or
of the pair fails.
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """One block: ctr (4 ints), key (2 ints) -> 4 output words (python ints)."""
    c0, c1, c2, c3 = (int(x) & MASK for x in ctr)
    k0, k1 = (int(x) & MASK for x in key)
    for r in range(10):
        if r:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> 32, p0 & MASK
        hi1, lo1 = p1 >> 32, p1 & MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & MASK, lo1, (hi0 ^ c3 ^ k1) & MASK, lo0
    return c0, c1, c2, c3


def _philox_vec(j, stream: int, fit: int, seed: int):
    """Vectorised Philox over counters (j, 0, stream, fit): four uint64 arrays."""
    j = np.asarray(j, dtype=np.uint64)
    c0 = j & np.uint64(MASK)
    c1 = np.zeros_like(c0)
    c2 = np.full_like(c0, np.uint64(stream & MASK))
    c3 = np.full_like(c0, np.uint64(fit & MASK))
    k0 = np.uint64(seed & MASK)
    k1 = np.uint64((seed >> 32) & MASK)
    m0 = np.uint64(M0)
    m1 = np.uint64(M1)
    mask = np.uint64(MASK)
    for r in range(10):
        if r:
            k0 = (k0 + np.uint64(W0)) & mask
            k1 = (k1 + np.uint64(W1)) & mask
        p0 = m0 * c0
        p1 = m1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & mask
        hi1, lo1 = p1 >> np.uint64(32), p1 & mask
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & mask, lo1, (hi0 ^ c3 ^ k1) & mask, lo0
    return c0, c1, c2, c3


def philox_uniform(count: int, stream: int, fit: int, seed: int, start: int = 0) -> np.ndarray:
    """`count` uniforms in (0, 1) for draws start..start+count-1 (module doc)."""
    j = np.arange(start, start + count, dtype=np.uint64)
    x0, x1, _, _ = _philox_vec(j, stream, fit, seed)
    bits = ((x0 << np.uint64(32)) | x1) >> np.uint64(12)
    return (bits.astype(np.float64) + 0.5) * 2.0 ** -52


def philox_normal(count: int, stream: int, fit: int, seed: int) -> np.ndarray:
    """`count` standard normals; normal t uses draws 2t and 2t+1 (module doc)."""
    u = philox_uniform(2 * count, stream, fit, seed)
    u1 = u[0::2]
    u2 = u[1::2]
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
