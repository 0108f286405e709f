"""Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC'11), written from its published definition (oracle; test
infrastructure only).

One round maps counter (c0, c1, c2, c3) and key (k0, k1) to
    (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0))
and the key is bumped by the Weyl constants between rounds; ten rounds.

Streams used by the motif library (the same convention is implemented,
separately, on the device):
    key = (seed, (domain << 32) | sub)
    domain 1  stratified hyperedge sampling; sub = stratum size j;
              counter = (i, 0, 0, 0) for draw i; index = hi64(word0 * |E_j|)
    domain 2  null-model copy; sub = copy index; counter = (t, round, lane, 0)
    domain 3  proposal (score-proportional) sampling; sub = stratum size j;
              counter = (i, 0, 0, 0) for draw i
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B
MASK64 = (1 << 64) - 1

DOMAIN_SAMPLE = 1
DOMAIN_NULL = 2
DOMAIN_PROPOSAL = 3


def philox4x64_10(counter, key):
    """Scalar form with Python integers."""
    c = [int(x) & MASK64 for x in counter]
    k = [int(x) & MASK64 for x in key]
    for _ in range(10):
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        c = [(p1 >> 64) ^ c[1] ^ k[0], p1 & MASK64, (p0 >> 64) ^ c[3] ^ k[1], p0 & MASK64]
        k = [(k[0] + W0) & MASK64, (k[1] + W1) & MASK64]
    return c


def _mulhilo(a: int, b: np.ndarray):
    """Full 64x64 -> 128-bit product of a constant and a uint64 vector, as (hi, lo)."""
    b = b.astype(np.uint64)
    a_lo, a_hi = np.uint64(a & 0xFFFFFFFF), np.uint64(a >> 32)
    m32 = np.uint64(0xFFFFFFFF)
    b_lo, b_hi = b & m32, b >> np.uint64(32)
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> np.uint64(32)) + (lh & m32) + (hl & m32)
    lo = (ll & m32) | ((mid & m32) << np.uint64(32))
    hi = hh + (lh >> np.uint64(32)) + (hl >> np.uint64(32)) + (mid >> np.uint64(32))
    return hi, lo


def philox_vec(c0, c1, c2, c3, k0: int, k1: int):
    """Vectorised Philox4x64-10 over counters given as uint64 arrays (or scalars)."""
    n = max(np.size(x) for x in (c0, c1, c2, c3))
    c = [np.broadcast_to(np.asarray(x, dtype=np.uint64), (n,)).copy() for x in (c0, c1, c2, c3)]
    ka, kb = k0 & MASK64, k1 & MASK64
    with np.errstate(over="ignore"):
        for _ in range(10):
            hi0, lo0 = _mulhilo(M0, c[0])
            hi1, lo1 = _mulhilo(M1, c[2])
            c = [hi1 ^ c[1] ^ np.uint64(ka), lo1, hi0 ^ c[3] ^ np.uint64(kb), lo0]
            ka = (ka + W0) & MASK64
            kb = (kb + W1) & MASK64
    return c


def stream_key(seed: int, domain: int, sub: int):
    return (int(seed) & MASK64, ((domain << 32) | (sub & 0xFFFFFFFF)) & MASK64)


def bounded(words: np.ndarray, n: int) -> np.ndarray:
    """hi64(word * n): a value in [0, n) from a uniform 64-bit word (Lemire's multiply-high)."""
    hi, _ = _mulhilo(int(n), np.asarray(words, dtype=np.uint64))
    return hi


def stratum_draws(seed: int, j: int, n_j: int, count: int) -> np.ndarray:
    """Indices of ``count`` with-replacement draws from a stratum of ``n_j`` hyperedges."""
    if count == 0 or n_j == 0:
        return np.zeros(count, dtype=np.int64)
    k0, k1 = stream_key(seed, DOMAIN_SAMPLE, j)
    w = philox_vec(np.arange(count, dtype=np.uint64), 0, 0, 0, k0, k1)[0]
    return bounded(w, n_j).astype(np.int64)
