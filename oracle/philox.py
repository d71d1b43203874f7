"""Pure-Python Philox4x32-10 (test infrastructure; second implementation).

Written from the definition in Salmon, Moraes, Dror and Shaw, "Parallel random
numbers: as easy as 1, 2, 3" (SC'11): a 4x32-bit counter, a 2x32-bit key, ten
rounds of two 32x32->64-bit products whose high halves are XORed with the
other two words and the round key; the key is bumped by the Weyl constants
between rounds.  Used by tests to name the exact uniform that the contract
assigns to one site, and to cross-check the C oracle.
"""
_MASK = 0xFFFFFFFF
_MUL = (0xD2511F53, 0xCD9E8D57)
_WEYL = (0x9E3779B9, 0xBB67AE85)


def philox4x32_10(ctr, key):
    a, b, c, d = (int(v) & _MASK for v in ctr)
    k0, k1 = (int(v) & _MASK for v in key)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + _WEYL[0]) & _MASK
            k1 = (k1 + _WEYL[1]) & _MASK
        pa = _MUL[0] * a
        pc = _MUL[1] * c
        a, b, c, d = ((pc >> 32) ^ b ^ k0) & _MASK, pc & _MASK, ((pa >> 32) ^ d ^ k1) & _MASK, pa & _MASK
    return [a, b, c, d]


def seed_key(seed):
    seed = int(seed)
    return (seed & _MASK, (seed >> 32) & _MASK)


def sweep_uniform(seed, replica, t, colour, Lx, x, y):
    """The 32-bit uniform the contract assigns to site (x, y) in sweep t."""
    h = (y * Lx + x) >> 1
    return philox4x32_10((h >> 2, t, replica, colour), seed_key(seed))[h & 3]


def bitsliced_uniform(seed, replica, t, colour, Lx, x, y):
    """The 32-bit uniform of site (x, y) in sweep t under the bit-sliced
    contract: with h the site's compact index, group g = h >> 5 has words
    W_k = sweep stream word 32 g + k (k = 0..31), and bit 31 - k of the
    uniform is bit h & 31 of W_k."""
    h = (y * Lx + x) >> 1
    g, b = h >> 5, h & 31
    u = 0
    for k in range(32):
        i = 32 * g + k
        w = philox4x32_10((i >> 2, t, replica, colour), seed_key(seed))[i & 3]
        u |= ((w >> b) & 1) << (31 - k)
    return u


def init_uniform(seed, replica, Lx, x, y):
    """The 32-bit uniform deciding the random initial spin of site (x, y)."""
    g = y * Lx + x
    return philox4x32_10((g >> 2, 0, replica, 2), seed_key(seed))[g & 3]
