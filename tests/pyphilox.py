"""Pure-Python Philox4x32-10, written independently of the C oracle from the
definition in Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
1, 2, 3" (SC'11): 4x32-bit counter, 2x32-bit key, ten rounds of two 32x32->64
multiplications (by 0xD2511F53 on word 0 and 0xCD9E8D57 on word 2) with the
key bumped by the golden-ratio and sqrt(3)-1 Weyl constants between rounds.

Used only by tests, as a second implementation that the oracle's Philox and its
noise mapping are compared against.
"""
MASK = (1 << 32) - 1
MULT = (0xD2511F53, 0xCD9E8D57)
WEYL = (0x9E3779B9, 0xBB67AE85)


def block(counter, key):
    x = [c & MASK for c in counter]
    k = [key[0] & MASK, key[1] & MASK]
    for r in range(10):
        if r:
            k = [(k[0] + WEYL[0]) & MASK, (k[1] + WEYL[1]) & MASK]
        prod_a = MULT[0] * x[0]
        prod_b = MULT[1] * x[2]
        x = [(prod_b >> 32) ^ x[1] ^ k[0], prod_b & MASK,
             (prod_a >> 32) ^ x[3] ^ k[1], prod_a & MASK]
    return x


def uniform_pm1(seed, t, idx):
    """The noise value r(seed, t, idx) in (-1, 1): word idx%4 of the block at
    counter (idx//4 as 64 bits, t as 64 bits) and key (seed as 64 bits), read as
    a signed 32-bit integer w, mapped to (w + 1/2) / 2^31."""
    q = idx // 4
    w = block([q & MASK, q >> 32, t & MASK, (t >> 32) & MASK], [seed & MASK, (seed >> 32) & MASK])[idx % 4]
    if w >= 1 << 31:
        w -= 1 << 32
    return (w + 0.5) / 2.0 ** 31
