"""Philox4x32-10 counter-based random number generator, vectorised in numpy.

Written from the published definition (Salmon, Moraes, Dror & Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11, Sec. 3 and Table 2):
a 4x32-bit counter block is mixed by ten rounds, each round multiplying two
of the words by fixed 32-bit multipliers and mixing the high and low halves of
the 64-bit products with the remaining words and the key; the two-word key is
bumped by two Weyl constants between rounds.

This module holds no arithmetic of the simulation method; it only turns a
(key, counter) pair into uniform variates for the seeded synthetic loads.
"""
import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint32(0x9E3779B9)
_W1 = np.uint32(0xBB67AE85)
_MASK32 = np.uint64(0xFFFFFFFF)
_SH32 = np.uint64(32)


def philox4x32(ctr, key, rounds=10):
    """Apply Philox4x32 to counter blocks.

    ctr: uint32 array of shape (..., 4); key: uint32 array of shape (..., 2)
    broadcastable against ctr[..., :2]. Returns uint32 array of shape (..., 4).
    """
    ctr = np.asarray(ctr, dtype=np.uint32)
    key = np.asarray(key, dtype=np.uint32)
    c0 = ctr[..., 0].astype(np.uint64)
    c1 = ctr[..., 1].astype(np.uint32)
    c2 = ctr[..., 2].astype(np.uint64)
    c3 = ctr[..., 3].astype(np.uint32)
    k0 = np.broadcast_to(key[..., 0], ctr.shape[:-1]).astype(np.uint32)
    k1 = np.broadcast_to(key[..., 1], ctr.shape[:-1]).astype(np.uint32)
    with np.errstate(over="ignore"):
        for r in range(rounds):
            if r > 0:
                k0 = k0 + _W0
                k1 = k1 + _W1
            p0 = _M0 * c0
            p1 = _M1 * c2
            hi0 = (p0 >> _SH32).astype(np.uint32)
            lo0 = (p0 & _MASK32).astype(np.uint32)
            hi1 = (p1 >> _SH32).astype(np.uint32)
            lo1 = (p1 & _MASK32).astype(np.uint32)
            n0 = hi1 ^ c1 ^ k0
            n1 = lo1
            n2 = hi0 ^ c3 ^ k1
            n3 = lo0
            c0 = n0.astype(np.uint64)
            c1 = n1
            c2 = n2.astype(np.uint64)
            c3 = n3
    out = np.empty(ctr.shape, dtype=np.uint32)
    out[..., 0] = c0.astype(np.uint32)
    out[..., 1] = c1
    out[..., 2] = c2.astype(np.uint32)
    out[..., 3] = c3
    return out


def u01_pair(words):
    """Two doubles in the open interval (0, 1) from a (..., 4) uint32 block.

    Each double takes 53 random bits from two words: 27 from the first and 26
    from the second, plus one half unit in the last place so that 0 never
    occurs.
    """
    w = words.astype(np.uint64)
    a = ((w[..., 0] >> np.uint64(5)) << np.uint64(26)) | (w[..., 1] >> np.uint64(6))
    b = ((w[..., 2] >> np.uint64(5)) << np.uint64(26)) | (w[..., 3] >> np.uint64(6))
    scale = 1.0 / 9007199254740992.0  # 2**-53
    return (a.astype(np.float64) + 0.5) * scale, (b.astype(np.float64) + 0.5) * scale


class Stream:
    """Per-item uniform variates: item index and draw number form the counter.

    key = (seed low 32 bits, seed high 32 bits xor tag); counter =
    (item low 32 bits, item high 32 bits, draw block, 0). One draw block
    yields two uniforms, so any item can draw as many variates as it needs
    without touching the counters of other items.
    """

    def __init__(self, seed, tag):
        seed = int(seed) & 0xFFFFFFFFFFFFFFFF
        self.key = np.array(
            [seed & 0xFFFFFFFF, ((seed >> 32) ^ (int(tag) * 0x85EBCA6B)) & 0xFFFFFFFF],
            dtype=np.uint32,
        )

    def uniforms(self, items, block):
        items = np.asarray(items, dtype=np.int64)
        ctr = np.empty(items.shape + (4,), dtype=np.uint32)
        ctr[..., 0] = (items & 0xFFFFFFFF).astype(np.uint32)
        ctr[..., 1] = (items >> 32).astype(np.uint32)
        ctr[..., 2] = np.uint32(block)
        ctr[..., 3] = 0
        return u01_pair(philox4x32(ctr, self.key))
