"""Oracle Philox4x32-10 counter-based generator (pure Python integers).

Test infrastructure only (see ``oracle/__init__``).

Philox4x32 with 10 rounds as defined by Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3" (SC'11): each round multiplies
words 0 and 2 by two fixed odd constants, producing 64-bit products whose
halves are permuted and XORed with the other words and the round key; the
key is advanced by two Weyl constants between rounds.

Stream layout used by the sampler (both sides implement it independently):
key = (seed_lo, seed_hi); counter = (chain_uid, t, tag, block) with tag 0 for
momenta (blocks 0 and 1 -> 8 words -> 4 Box-Muller pairs, first 6 normals
used), tag 1 for the Metropolis uniform (word 0 of block 0), tag 2 for the
chain-start jitter, tag 3 for the step-size jitter (word 0 of block 0).
"""
from __future__ import annotations

import math

import numpy as np

MASK = 0xFFFFFFFF
PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85

TAG_MOMENTUM = 0
TAG_ACCEPT = 1
TAG_INIT = 2
TAG_JITTER = 3


def philox4x32_10(counter, key):
    x0, x1, x2, x3 = [c & MASK for c in counter]
    k0, k1 = key[0] & MASK, key[1] & MASK
    for r in range(10):
        if r > 0:
            k0 = (k0 + PHILOX_W0) & MASK
            k1 = (k1 + PHILOX_W1) & MASK
        p0 = PHILOX_M0 * x0
        p1 = PHILOX_M1 * x2
        hi0, lo0 = (p0 >> 32) & MASK, p0 & MASK
        hi1, lo1 = (p1 >> 32) & MASK, p1 & MASK
        x0, x1, x2, x3 = (hi1 ^ x1 ^ k0), lo1, (hi0 ^ x3 ^ k1), lo0
    return (x0, x1, x2, x3)


def seed_key(seed: int):
    seed &= 0xFFFFFFFFFFFFFFFF
    return (seed & MASK, (seed >> 32) & MASK)


def uniform_from_word(w: int) -> float:
    """Top 23 bits mapped to the open interval (0, 1).

    Every value is an odd multiple of 2^-24 below 1, hence exactly
    representable in float32 (24-bit significand); with 24 bits the largest
    value 1 - 2^-25 would not be."""
    return ((w >> 9) + 0.5) * (2.0 ** -23)


def box_muller(u0: float, u1: float):
    r = math.sqrt(-2.0 * math.log(u0))
    a = 2.0 * math.pi * u1
    return r * math.cos(a), r * math.sin(a)


def momentum_normals(seed: int, chain_uid: int, t: int) -> np.ndarray:
    key = seed_key(seed)
    words = list(philox4x32_10((chain_uid, t, TAG_MOMENTUM, 0), key)) + \
        list(philox4x32_10((chain_uid, t, TAG_MOMENTUM, 1), key))
    z = []
    for j in range(4):
        z.extend(box_muller(uniform_from_word(words[2 * j]), uniform_from_word(words[2 * j + 1])))
    return np.array(z[:6])


def accept_uniform(seed: int, chain_uid: int, t: int) -> float:
    w = philox4x32_10((chain_uid, t, TAG_ACCEPT, 0), seed_key(seed))
    return uniform_from_word(w[0])


def jitter_uniform(seed: int, chain_uid: int, t: int) -> float:
    w = philox4x32_10((chain_uid, t, TAG_JITTER, 0), seed_key(seed))
    return uniform_from_word(w[0])


# ---- NUTS stream (tag 4) ------------------------------------------------------
# counter (chain_uid, t, 4, block): block d < 64, word 0 -> direction of doubling
# d (uniform < 1/2: backward), word 1 -> the uniform of the merge after doubling
# d; block 64 + n // 4, word n % 4 -> the uniform of the n-th leaf of the
# iteration (counted over the whole trajectory) in its subtree's sampling.
TAG_NUTS = 4


def nuts_direction(seed: int, chain_uid: int, t: int, d: int) -> int:
    w = philox4x32_10((chain_uid, t, TAG_NUTS, d), seed_key(seed))
    return -1 if uniform_from_word(w[0]) < 0.5 else 1


def nuts_merge_uniform(seed: int, chain_uid: int, t: int, d: int) -> float:
    w = philox4x32_10((chain_uid, t, TAG_NUTS, d), seed_key(seed))
    return uniform_from_word(w[1])


def nuts_leaf_uniform(seed: int, chain_uid: int, t: int, n: int) -> float:
    w = philox4x32_10((chain_uid, t, TAG_NUTS, 64 + n // 4), seed_key(seed))
    return uniform_from_word(w[n % 4])
