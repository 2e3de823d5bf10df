"""Counter-based random numbers for stochastic dynamics (test infrastructure).

The paper makes its stochastic integrators reproducible by handing the random
generator to every function that draws (Sec. II, code-design paragraph). Here
the numbers are a pure function of (seed, step, atom): Philox4x64-10 (Salmon,
Moraes, Dror, Shaw, SC'11), one 4-word block per atom and step, with the
counter (atom, step, 0, 0) and the key (seed_lo, seed_hi). The GPU side
implements the same published definition independently.

Uniforms u = (top 24 bits + 1) / 2^24 in (0, 1] (exact in float32 and float64);
normals by Box-Muller: sqrt(-2 ln u1) (cos, sin)(2 pi u2), and from (u3, u4) a
third (the cosine branch).
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B
MASK = (1 << 64) - 1


def philox4x64_10(ctr, key):
    """Pure-Python reference of one block: ctr 4 ints, key 2 ints (< 2^64)."""
    c = [int(v) & MASK for v in ctr]
    k0, k1 = int(key[0]) & MASK, int(key[1]) & MASK
    for r in range(10):
        if r:
            k0, k1 = (k0 + W0) & MASK, (k1 + W1) & MASK
        p0, p1 = M0 * c[0], M1 * c[2]
        hi0, lo0 = p0 >> 64, p0 & MASK
        hi1, lo1 = p1 >> 64, p1 & MASK
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return c


def _mulhilo(a, b):
    """64 x 64 -> (hi, lo) on uint64 arrays, from 32-bit halves."""
    m32 = np.uint64(0xFFFFFFFF)
    s32 = np.uint64(32)
    a_lo, a_hi = a & m32, a >> s32
    b_lo, b_hi = b & m32, b >> s32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> s32) + (lh & m32) + (hl & m32)
    lo = (ll & m32) | ((mid & m32) << s32)
    hi = hh + (lh >> s32) + (hl >> s32) + (mid >> s32)
    return hi, lo


def philox_blocks(atoms, step, seed):
    """Blocks for counters (atom, step, 0, 0), key (seed_lo, seed_hi): uint64 [4, n]."""
    with np.errstate(over="ignore"):
        a = np.asarray(atoms, np.uint64)
        c = [a, np.full_like(a, np.uint64(step)), np.zeros_like(a), np.zeros_like(a)]
        k0 = np.uint64(int(seed) & MASK)
        k1 = np.uint64((int(seed) >> 64) & MASK)
        for r in range(10):
            if r:
                k0 = np.uint64((int(k0) + W0) & MASK)
                k1 = np.uint64((int(k1) + W1) & MASK)
            hi0, lo0 = _mulhilo(np.uint64(M0), c[0])
            hi1, lo1 = _mulhilo(np.uint64(M1), c[2])
            c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack(c)


def uniforms24(words):
    """(top 24 bits + 1) / 2^24 in (0, 1], float64."""
    return ((words >> np.uint64(40)).astype(np.float64) + 1.0) / 16777216.0


def normals3(atoms, step, seed):
    """Three standard normals per atom (float64 [3, n])."""
    u = uniforms24(philox_blocks(atoms, step, seed))
    r1 = np.sqrt(-2.0 * np.log(u[0]))
    r2 = np.sqrt(-2.0 * np.log(u[2]))
    return np.stack([r1 * np.cos(2 * np.pi * u[1]), r1 * np.sin(2 * np.pi * u[1]),
                     r2 * np.cos(2 * np.pi * u[3])])
