"""Philox4x32-10 counter-based generator and the sampler's draws (CPU oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Philox4x32 is defined in Salmon, Moraes, Dror & Shaw, "Parallel random
numbers: as easy as 1, 2, 3" (SC 2011): a 128-bit counter (c0, c1, c2, c3)
and a 64-bit key (k0, k1) go through R rounds of

    (hi0, lo0) = M0 * c0,  (hi1, lo1) = M1 * c2       (32x32 -> 64-bit products)
    c' = (hi1 ^ c1 ^ k0,  lo1,  hi0 ^ c3 ^ k1,  lo0)

with the key advanced by the Weyl constants (W0, W1) between rounds;
Philox4x32-10 uses R = 10.  Written here with Python integers, one round at
a time, as the paper describes it.

The sampler's streams (documented with the library's MCMC entry points):
counter = (index, chain, iteration, purpose), key = (seed low word, seed high
word).  A uniform is ((64-bit word >> 11) + 1/2) * 2^-53 of words (0,1) and
(2,3); a normal pair is Box-Muller (r cos 2 pi u1, r sin 2 pi u1) with
r = sqrt(-2 ln u0).
"""
import math

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF

PROPOSAL, MIXTURE, ACCEPT, MINIBATCH, INIT = 1, 2, 3, 4, 5


def philox4x32(counter, key, rounds=10):
    """The Philox4x32-R bijection of `counter` (4 words) under `key` (2 words)."""
    c0, c1, c2, c3 = (int(x) & MASK for x in counter)
    k0, k1 = (int(x) & MASK for x in key)
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> 32, p0 & MASK
        hi1, lo1 = p1 >> 32, p1 & MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def u01(hi, lo):
    """Uniform in (0, 1) from two 32-bit words: 53 high bits plus one half ulp."""
    x = (hi << 32) | lo
    return ((x >> 11) + 0.5) / 9007199254740992.0


def uniform2(seed, purpose, it, chain, index):
    r = philox4x32((index, chain, it, purpose), (seed & MASK, (seed >> 32) & MASK))
    return u01(r[0], r[1]), u01(r[2], r[3])


def normal2(seed, purpose, it, chain, index):
    a, b = uniform2(seed, purpose, it, chain, index)
    r = math.sqrt(-2.0 * math.log(a))
    return r * math.cos(2.0 * math.pi * b), r * math.sin(2.0 * math.pi * b)


def normals(seed, purpose, it, chain, n):
    """n standard normals of one (iteration, chain, purpose) stream, index = pair."""
    out = []
    for i in range((n + 1) // 2):
        out.extend(normal2(seed, purpose, it, chain, i))
    return out[:n]
