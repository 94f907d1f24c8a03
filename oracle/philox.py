"""Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11,
"Parallel random numbers: as easy as 1, 2, 3"), written from the published
definition.

The paper fixes no random stream (it only publishes seeds with its code).
The sampler's draws use (a reading recorded in the design notes):

    block = Philox4x64_10(counter=(op_index, chain, 0, 0), key=(seed, 0))
    u     = (block[0] >> 11) * 2**-53          # uniform in [0, 1), 53 bits

Pinned against ``numpy.random.Philox`` (a library implementation of the same
published generator) in ``tests/test_oracle_philox.py``.
"""
from __future__ import annotations

import numpy as np

# Round multipliers and Weyl key increments of Philox4x64 (published constants).
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15
PHILOX_W1 = 0xBB67AE8584CAA73B
MASK64 = (1 << 64) - 1


def philox4x64_scalar(ctr, key, rounds: int = 10):
    """Plain Python-integer version: returns the 4-word output block."""
    c0, c1, c2, c3 = (int(v) & MASK64 for v in ctr)
    k0, k1 = (int(v) & MASK64 for v in key)
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + PHILOX_W0) & MASK64
            k1 = (k1 + PHILOX_W1) & MASK64
        p0 = PHILOX_M0 * c0
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return (c0, c1, c2, c3)


def _mulhilo(a: np.ndarray, m: int):
    """64x64 -> (hi, lo) for uint64 arrays, by 32-bit halves."""
    a = a.astype(np.uint64)
    m_lo = np.uint64(m & 0xFFFFFFFF)
    m_hi = np.uint64(m >> 32)
    mask = np.uint64(0xFFFFFFFF)
    s32 = np.uint64(32)
    a_lo = a & mask
    a_hi = a >> s32
    ll = a_lo * m_lo
    hl = a_hi * m_lo
    lh = a_lo * m_hi
    hh = a_hi * m_hi
    cross = (ll >> s32) + (hl & mask) + (lh & mask)
    hi = hh + (hl >> s32) + (lh >> s32) + (cross >> s32)
    lo = a * np.uint64(m)          # wraps modulo 2**64
    return hi, lo


def philox4x64(ctr0, ctr1, key0, rounds: int = 10, ctr2=0, ctr3=0, key1=0):
    """Vectorised Philox4x64-10 over broadcastable uint64 counter words."""
    with np.errstate(over="ignore"):
        c0 = np.asarray(ctr0, dtype=np.uint64)
        c1 = np.asarray(ctr1, dtype=np.uint64)
        c0, c1 = np.broadcast_arrays(c0, c1)
        c0 = c0.copy()
        c1 = c1.copy()
        c2 = np.full_like(c0, np.uint64(ctr2))
        c3 = np.full_like(c0, np.uint64(ctr3))
        k0 = np.uint64(int(key0) & MASK64)
        k1 = np.uint64(int(key1) & MASK64)
        w0 = np.uint64(PHILOX_W0)
        w1 = np.uint64(PHILOX_W1)
        for r in range(rounds):
            if r > 0:
                k0 = k0 + w0
                k1 = k1 + w1
            hi0, lo0 = _mulhilo(c0, PHILOX_M0)
            hi1, lo1 = _mulhilo(c2, PHILOX_M1)
            c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return c0, c1, c2, c3


def uniform53(op_index, chains, seed):
    """u in [0,1) for (op_index, chain) pairs: (word0 >> 11) * 2**-53."""
    w0, _, _, _ = philox4x64(np.uint64(op_index), np.asarray(chains, dtype=np.uint64), seed)
    return (w0 >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
