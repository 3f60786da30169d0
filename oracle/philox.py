"""Philox4x64-10 counter-based generator, written from its published
definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC'11).  Pure Python integers; used for the Metropolis uniforms.

The method section samples configurations by Markov-chain Monte Carlo; the
paper does not fix a generator.  Reading: one uniform per proposal slot,
  counter = (chain, global_sweep, slot, stream), key = (seed, 0),
  u = (w0 >> 11) * 2^-53   (w0 = first output word),
so every draw is positional and independent of how many proposals were
actually evaluated.
"""
from __future__ import annotations

MASK64 = (1 << 64) - 1
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15  # golden ratio
PHILOX_W1 = 0xBB67AE8584CAA73B  # sqrt(3) - 1


def philox4x64_10(ctr, key):
    """Ten Philox rounds on a 4 x 64-bit counter with a 2 x 64-bit key."""
    c0, c1, c2, c3 = (int(x) & MASK64 for x in ctr)
    k0, k1 = (int(x) & MASK64 for x in key)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + PHILOX_W0) & MASK64
            k1 = (k1 + PHILOX_W1) & MASK64
        p0 = PHILOX_M0 * c0
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def uniform(seed, chain, gsweep, slot, stream=0):
    """Uniform double in [0, 1) owned by one proposal slot."""
    w0 = philox4x64_10((chain, gsweep, slot, stream), (seed, 0))[0]
    return (w0 >> 11) * (2.0 ** -53)
