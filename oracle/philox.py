"""Philox4x64-10 and Box-Muller normals for the sketch test matrix (test infrastructure).

The sketch of Sec. 2.2 uses a standard normal test matrix Omega.  The GPU
library draws it from a counter-based generator so that any element can be
produced independently; this module restates the same published generator
(Philox4x64 with 10 rounds, Salmon, Moraes, Dror, Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11) and the Box-Muller transform in plain
Python integers, so the oracle can rebuild Omega for a given (seed, stream).

Element (i, j) of the n x s column-major Omega has linear index e = j n + i.
Block c = e // 4 is Philox4x64-10 of counter (c, 0, 0, 0) under key
(seed, stream); lane l = e % 4 takes the pair p = l // 2 of 64-bit outputs
(o[2p], o[2p+1]) and
    U1 = ((o[2p] >> 11) + 1/2) 2^-53,   U2 = (o[2p+1] >> 11) 2^-53,
    R = sqrt(-2 ln U1),  theta = 2 pi U2,
    Omega = R cos(theta) for even l, R sin(theta) for odd l,
computed in FP64 and rounded once to FP32.

Pinned by numpy.random.Philox (the same published generator; numpy advances
its counter by one before producing a block, so its first block is counter
(1, 0, 0, 0)), and by the first two moments of the normals.
"""
import math

import numpy as np

_M0 = 0xD2E7470EE14C6C93
_M1 = 0xCA5A826395121157
_W0 = 0x9E3779B97F4A7C15
_W1 = 0xBB67AE8584CAA73B
_MASK = (1 << 64) - 1


def philox4x64_10(counter, key):
    """One Philox4x64-10 block: counter (4 x u64), key (2 x u64) -> 4 x u64."""
    c0, c1, c2, c3 = (int(v) & _MASK for v in counter)
    k0, k1 = (int(v) & _MASK for v in key)
    for _ in range(10):
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> 64, p0 & _MASK
        hi1, lo1 = p1 >> 64, p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + _W0) & _MASK
        k1 = (k1 + _W1) & _MASK
    return (c0, c1, c2, c3)


def normal_pair(o_a, o_b):
    u1 = ((o_a >> 11) + 0.5) * 2.0 ** -53
    u2 = (o_b >> 11) * 2.0 ** -53
    r = math.sqrt(-2.0 * math.log(u1))
    t = 2.0 * math.pi * u2
    return r * math.cos(t), r * math.sin(t)


def gaussian_matrix(n, s, seed, stream=0):
    """n x s FP32 test matrix (column-major element order as described above)."""
    total = n * s
    flat = np.empty(total, dtype=np.float64)
    nblocks = (total + 3) // 4
    for c in range(nblocks):
        o = philox4x64_10((c, 0, 0, 0), (seed, stream))
        z0, z1 = normal_pair(o[0], o[1])
        z2, z3 = normal_pair(o[2], o[3])
        vals = (z0, z1, z2, z3)
        for l in range(4):
            e = 4 * c + l
            if e < total:
                flat[e] = vals[l]
    return flat.reshape(s, n).T.astype(np.float32)
