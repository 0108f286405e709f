"""Order-5 motifs (oracle; test infrastructure only): Python front of
``motif5_oracle.c``.

Section 6.4 runs the sampling algorithm of Section 5 at order 5, where the
exact algorithms do not reach.  A class is reported by its canonical pattern:
the smallest 26-bit fill-in pattern (one bit per subset of the five local
positions with at least two members, ascending subset-mask order; local
positions follow ascending node id) over the 120 relabellings.  Its maxcard
(largest hyperedge size) and countmax (how many hyperedges have that size)
follow from the pattern, and the estimate of a class is
raw * |E_maxcard| / (S_maxcard * countmax), as at orders 3 and 4.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import build as _build
from .core import Normalised, normalise

_lib = None
N_SUB = 26
SUB_MASKS = [m for m in range(32) if bin(m).count("1") >= 2]


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(_build.ensure_built(_build.LIB5))
        u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
        i64 = ctypes.c_int64
        _lib.oracle5_canonical.argtypes = [ctypes.c_uint32]
        _lib.oracle5_canonical.restype = ctypes.c_uint32
        _lib.oracle5_connected.argtypes = [ctypes.c_uint32]
        _lib.oracle5_connected.restype = ctypes.c_int
        _lib.oracle5_maxcard.argtypes = [ctypes.c_uint32, ctypes.POINTER(ctypes.c_int)]
        _lib.oracle5_maxcard.restype = ctypes.c_int
        _lib.oracle5_exact_brute.argtypes = [ctypes.c_uint32, u32p, i64, u32p, i64, u32p, i64, u32p, i64, u32p, i64p,
                                             i64]
        _lib.oracle5_exact_brute.restype = i64
        _lib.oracle5_sampled_raw.argtypes = [ctypes.c_uint32, u32p, i64, u32p, i64, u32p, i64, u32p, i64,
                                             i64p, i64, i64p, i64, i64p, i64, i64p, i64, u32p, i64p, i64]
        _lib.oracle5_sampled_raw.restype = i64
    return _lib


def canonical(pattern: int) -> int:
    return int(lib().oracle5_canonical(pattern))


def connected(pattern: int) -> bool:
    return bool(lib().oracle5_connected(pattern))


def maxcard(pattern: int):
    """(maxcard, countmax) of a pattern."""
    cm = ctypes.c_int(0)
    mc = lib().oracle5_maxcard(pattern, ctypes.byref(cm))
    return mc, cm.value


def _flat(nh, j):
    return np.ascontiguousarray(nh.edges(j).reshape(-1), dtype=np.uint32)


def _dict(n, canon, cnt):
    if n < 0:
        raise RuntimeError("order-5 oracle failed")
    return {int(canon[i]): int(cnt[i]) for i in range(n)}


def exact_brute(h, cap: int = 1 << 16) -> dict:
    """Every connected induced 5-node sub-hypergraph, by class: {canonical: count}."""
    nh = h if isinstance(h, Normalised) else normalise(h)
    canon = np.zeros(cap, dtype=np.uint32)
    cnt = np.zeros(cap, dtype=np.int64)
    n = lib().oracle5_exact_brute(nh.n_nodes, _flat(nh, 2), nh.count(2), _flat(nh, 3), nh.count(3), _flat(nh, 4),
                                  nh.count(4), _flat(nh, 5), nh.count(5), canon, cnt, cap)
    return _dict(n, canon, cnt)


def sampled_raw(h, samples: dict, cap: int = 1 << 16) -> dict:
    """Raw counts of Algorithm 4 at order 5 for explicit sample lists {j: indices}."""
    nh = h if isinstance(h, Normalised) else normalise(h)
    s = {j: np.ascontiguousarray(np.asarray(samples.get(j, []), dtype=np.int64)) for j in (2, 3, 4, 5)}
    canon = np.zeros(cap, dtype=np.uint32)
    cnt = np.zeros(cap, dtype=np.int64)
    n = lib().oracle5_sampled_raw(nh.n_nodes, _flat(nh, 2), nh.count(2), _flat(nh, 3), nh.count(3), _flat(nh, 4),
                                  nh.count(4), _flat(nh, 5), nh.count(5), s[2], len(s[2]), s[3], len(s[3]),
                                  s[4], len(s[4]), s[5], len(s[5]), canon, cnt, cap)
    return _dict(n, canon, cnt)


def scale(raw: dict, n_by_size: dict, s_by_size: dict) -> dict:
    """raw * |E_j| / (S_j * countmax), j = maxcard, in float64 (0 when S_j = 0)."""
    out = {}
    for c, r in raw.items():
        j, cm = maxcard(c)
        S = s_by_size.get(j, 0)
        out[c] = float(r) * float(n_by_size.get(j, 0)) / (float(S) * cm) if S else 0.0
    return out
