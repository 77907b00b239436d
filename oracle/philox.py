"""Philox4x32-10 counter-based generator, written with Python integers.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU
baseline of the benchmark, never by the product path.

Definition followed: Salmon, Moraes, Dror and Shaw, "Parallel Random Numbers:
As Easy as 1, 2, 3" (SC'11), Philox with four 32-bit words and ten rounds.
One round multiplies counter words 0 and 2 by two fixed odd 32-bit
multipliers, keeps the high and low halves of each 64-bit product, XORs the
high halves with the other two counter words and the two key words, and
permutes the words; between rounds the key is advanced by two Weyl
increments (the golden ratio and sqrt(3)-1 scaled to 32 bits).

Pinned in tests/test_oracle_philox.py against the three known-answer cases
published with the generator (tests/golden/philox4x32_10_kat.json), and for
the statistical properties the decomposition relies on (uniformity,
independence across counters).
"""
from __future__ import annotations

MASK32 = 0xFFFFFFFF
MULT0 = 0xD2511F53
MULT1 = 0xCD9E8D57
WEYL0 = 0x9E3779B9
WEYL1 = 0xBB67AE85


def _one_round(c, k0, k1):
    prod0 = MULT0 * c[0]
    prod1 = MULT1 * c[2]
    hi0, lo0 = prod0 >> 32, prod0 & MASK32
    hi1, lo1 = prod1 >> 32, prod1 & MASK32
    return (hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0)


def philox4x32_10(counter, key):
    """Return the four 32-bit output words for a 4-word counter and 2-word key."""
    c = tuple(int(w) & MASK32 for w in counter)
    k0, k1 = (int(w) & MASK32 for w in key)
    for r in range(10):
        if r:
            k0 = (k0 + WEYL0) & MASK32
            k1 = (k1 + WEYL1) & MASK32
        c = _one_round(c, k0, k1)
    return c


def draw_u128(seed: int, j: int, step: int = 0, tensor: int = 0) -> int:
    """128-bit uniform integer for draw j.

    Key = (seed mod 2^32, seed >> 32); counter = (j mod 2^32, j >> 32, step,
    tensor); the four output words are joined little-endian.
    """
    x = philox4x32_10((j & MASK32, (j >> 32) & MASK32, step & MASK32, tensor & MASK32),
                      (seed & MASK32, (seed >> 32) & MASK32))
    return x[0] | (x[1] << 32) | (x[2] << 64) | (x[3] << 96)
