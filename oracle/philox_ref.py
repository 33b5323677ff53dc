"""Philox4x64-10 counter-based generator and the Gaussian draws built on it
(test infrastructure only; shares no code with the GPU library).

Philox4x64-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC 2011): a 256-bit counter (four 64-bit words) and a 128-bit key
go through ten rounds; each round multiplies counter words 0 and 2 by fixed
64-bit constants, swaps and XORs the high halves with the other two words and
the key, and the key is advanced by two Weyl constants between rounds.

Gaussian noise: each 64-bit output word w gives a uniform u = (floor(w / 2^40)
+ 1/2) / 2^24 in (0, 1) (its top 24 bits); consecutive pairs (u1, u2) give
two standard normals by the Box-Muller transform
sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2).
"""
from __future__ import annotations

import math

import numpy as np

MASK = (1 << 64) - 1
MUL = (0xD2E7470EE14C6C93, 0xCA5A826395121157)
WEYL = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)


def _mulhilo(a: int, b: int):
    p = a * b
    return p >> 64, p & MASK


def philox4x64_10(ctr, key):
    """One block: four 64-bit words from counter words ctr[0..3] and key words key[0..1]."""
    c = [int(v) & MASK for v in ctr]
    k0, k1 = int(key[0]) & MASK, int(key[1]) & MASK
    for r in range(10):
        if r:
            k0 = (k0 + WEYL[0]) & MASK
            k1 = (k1 + WEYL[1]) & MASK
        hi0, lo0 = _mulhilo(MUL[0], c[0])
        hi1, lo1 = _mulhilo(MUL[1], c[2])
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return c


def counter_add(ctr, n: int):
    """256-bit counter plus n (word 0 least significant)."""
    v = sum(int(w) << (64 * i) for i, w in enumerate(ctr)) + n
    v &= (1 << 256) - 1
    return [(v >> (64 * i)) & MASK for i in range(4)]


def raw_blocks(key, ctr, n_blocks: int) -> np.ndarray:
    """Blocks for counters ctr, ctr+1, ... as uint64 [n_blocks, 4]."""
    out = np.zeros((n_blocks, 4), dtype=np.uint64)
    for b in range(n_blocks):
        out[b] = philox4x64_10(counter_add(ctr, b), key)
    return out


def uniform24(words: np.ndarray) -> np.ndarray:
    return ((words >> np.uint64(40)).astype(np.float64) + 0.5) / float(1 << 24)


def normals(key, ctr, n: int) -> np.ndarray:
    """n standard normals: block b (counter ctr + b) gives normals 4b .. 4b+3."""
    nb = (n + 3) // 4
    u = uniform24(raw_blocks(key, ctr, nb))
    r1 = np.sqrt(-2.0 * np.log(u[:, 0]))
    r2 = np.sqrt(-2.0 * np.log(u[:, 2]))
    z = np.stack([r1 * np.cos(2 * math.pi * u[:, 1]), r1 * np.sin(2 * math.pi * u[:, 1]),
                  r2 * np.cos(2 * math.pi * u[:, 3]), r2 * np.sin(2 * math.pi * u[:, 3])], axis=1)
    return z.reshape(-1)[:n]
