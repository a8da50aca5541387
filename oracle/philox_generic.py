"""Word-size-generic Philox4xW-R (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC'11) in plain Python integers -- TEST INFRASTRUCTURE ONLY.

One round maps the counter (c0, c1, c2, c3) with round key (k0, k1) to
    (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0))
and the key is bumped by the Weyl constants (W0, W1) between rounds.

The 64-bit instance is pinned against NumPy's Philox4x64 bit generator, which checks the
round structure and key schedule; the 32-bit instance (different constants only) then pins
the C++ oracle's Philox4x32-10, which in turn pins the renderer's.
"""
from __future__ import annotations

CONSTANTS = {
    32: dict(M0=0xD2511F53, M1=0xCD9E8D57, W0=0x9E3779B9, W1=0xBB67AE85),
    64: dict(M0=0xD2E7470EE14C6C93, M1=0xCA5A826395121157, W0=0x9E3779B97F4A7C15, W1=0xBB67AE8584CAA73B),
}


def philox4(ctr, key, width=32, rounds=10):
    c = CONSTANTS[width]
    mask = (1 << width) - 1
    c0, c1, c2, c3 = (int(x) & mask for x in ctr)
    k0, k1 = (int(x) & mask for x in key)
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + c["W0"]) & mask
            k1 = (k1 + c["W1"]) & mask
        p0 = c["M0"] * c0
        p1 = c["M1"] * c2
        c0, c1, c2, c3 = ((p1 >> width) ^ c1 ^ k0) & mask, p1 & mask, ((p0 >> width) ^ c3 ^ k1) & mask, p0 & mask
    return (c0, c1, c2, c3)


def uniform24(x: int) -> float:
    """Top 24 bits of a 32-bit word scaled by 2^-24: exact in FP32 and FP64."""
    return (int(x) >> 8) * 2.0**-24
