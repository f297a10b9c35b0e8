"""Pure-Python Philox4x32-10, written from its published definition.

TEST INFRASTRUCTURE. Nothing in the product path may import this module; only
the tests, the smoke check and the CPU-baseline leg of the benchmark use it.

Definition followed: Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
as easy as 1, 2, 3", SC'11, section on the Philox family.  A Philox-4x32
round takes a 4-word counter (c0, c1, c2, c3) and a 2-word key (k0, k1),
forms the two 64-bit products M0*c0 and M1*c2, and returns
(hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0)).  Between
rounds the key is bumped by the Weyl constants (golden ratio and sqrt(3)-1
scaled to 32 bits).  The -10 variant applies ten rounds.

This is the third, independent implementation (besides the C oracle and the
HIP device code) used to pin the generator bit for bit.
"""

MASK32 = 0xFFFFFFFF
PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9  # floor(2^32 * (golden ratio - 1))
PHILOX_W1 = 0xBB67AE85  # floor(2^32 * (sqrt(3) - 1))


def _round(ctr, key):
    p0 = PHILOX_M0 * ctr[0]
    p1 = PHILOX_M1 * ctr[2]
    hi0, lo0 = (p0 >> 32) & MASK32, p0 & MASK32
    hi1, lo1 = (p1 >> 32) & MASK32, p1 & MASK32
    return [hi1 ^ ctr[1] ^ key[0], lo1, hi0 ^ ctr[3] ^ key[1], lo0]


def philox4x32_10(ctr, key):
    """Return the four 32-bit output words for a 4-word counter and 2-word key."""
    c = [int(v) & MASK32 for v in ctr]
    k = [int(v) & MASK32 for v in key]
    for r in range(10):
        if r > 0:
            k = [(k[0] + PHILOX_W0) & MASK32, (k[1] + PHILOX_W1) & MASK32]
        c = _round(c, k)
    return c
