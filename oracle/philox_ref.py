"""Pure-Python Philox4x32-10 and Box-Muller (test infrastructure only).

A second, independent restatement of the generator from its publication
(Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC'11) using Python's unbounded integers, so that a slip in the C oracle's
32-bit arithmetic (a lost carry, a swapped half) shows up as a mismatch.
"""
import math

_MASK = (1 << 32) - 1
_MUL = (0xD2511F53, 0xCD9E8D57)   # round multipliers for words 0 and 2
_WEYL = (0x9E3779B9, 0xBB67AE85)  # key increments between rounds


def philox4x32_10(key, ctr):
    """key: (k0, k1); ctr: (c0, c1, c2, c3); returns the 4 output words."""
    k0, k1 = key[0] & _MASK, key[1] & _MASK
    c0, c1, c2, c3 = (x & _MASK for x in ctr)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + _WEYL[0]) & _MASK
            k1 = (k1 + _WEYL[1]) & _MASK
        prod0 = _MUL[0] * c0
        prod1 = _MUL[1] * c2
        c0, c1, c2, c3 = ((prod1 >> 32) ^ c1 ^ k0, prod1 & _MASK,
                          (prod0 >> 32) ^ c3 ^ k1, prod0 & _MASK)
    return [c0, c1, c2, c3]


def key_of(seed):
    return (seed & _MASK, (seed >> 32) & _MASK)


def block(seed, tag, a, b, blk):
    return philox4x32_10(key_of(seed), (blk & _MASK, a, b, tag))


def gaussians(words):
    """Box-Muller on (w0, w1) and (w2, w3) with 24-bit uniforms."""
    out = []
    for i in (0, 2):
        u1 = ((words[i] >> 8) + 1) / 16777216.0
        u2 = (words[i + 1] >> 8) / 16777216.0
        rho = math.sqrt(-2.0 * math.log(u1))
        out += [rho * math.cos(2.0 * math.pi * u2), rho * math.sin(2.0 * math.pi * u2)]
    return out
