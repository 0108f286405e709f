"""Python front of the C oracle (test infrastructure only).

``normalise`` applies the definitions of Section 3 to a raw hyperedge list:
a hypergraph's hyperedges form a *set* (duplicates collapse, first occurrence
kept), the empty set and singletons are ignored by fill-in (Section 4.3), and
a hyperedge is a set of nodes (a repeated node is an input error).  The
per-size lists keep first-occurrence order, which is the stratum order the
sampler indexes (Section 5, Algorithm 4).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import build as _build
from .classes import table

_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(_build.ensure_built())
        u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
        i64 = ctypes.c_int64
        _lib.oracle_count_exact.argtypes = [ctypes.c_int, ctypes.c_uint32, u32p, i64, u32p, i64, u32p, i64, i64p]
        _lib.oracle_count_exact.restype = ctypes.c_int
        _lib.oracle_count_exact_threads.argtypes = [ctypes.c_int, ctypes.c_uint32, u32p, i64, u32p, i64, u32p, i64,
                                                    ctypes.c_int, i64p]
        _lib.oracle_count_exact_threads.restype = ctypes.c_int
        _lib.oracle_count_baseline.argtypes = [ctypes.c_int, ctypes.c_uint32, u32p, i64p, i64, u32p, i64, u32p, i64,
                                               u32p, i64, i64p, i64p]
        _lib.oracle_count_baseline.restype = ctypes.c_int
        _lib.oracle_sampled_raw.argtypes = [ctypes.c_int, ctypes.c_uint32, u32p, i64, u32p, i64, u32p, i64,
                                            i64p, i64, i64p, i64, i64p, i64, i64p]
        _lib.oracle_sampled_raw.restype = ctypes.c_int
        _lib.oracle_class_canon.argtypes = [ctypes.c_int, u32p]
        _lib.oracle_class_canon.restype = ctypes.c_int
        _lib.oracle_pattern_class.argtypes = [ctypes.c_int, ctypes.c_uint32]
        _lib.oracle_pattern_class.restype = ctypes.c_int
    return _lib


class InputError(ValueError):
    pass


@dataclass
class Normalised:
    n_nodes: int
    by_size: dict            # size j -> int64 array (n_j, j), ascending rows, first-occurrence order
    n_dropped_singletons: int
    n_duplicates: int
    order: list              # every unique hyperedge (ascending tuple), first-occurrence order

    def edges(self, j: int) -> np.ndarray:
        return self.by_size.get(j, np.zeros((0, j), dtype=np.int64))

    def count(self, j: int) -> int:
        return len(self.edges(j))


def normalise(h) -> Normalised:
    """Set semantics of Section 3 applied to a ``workloads.Hypergraph``."""
    off = h.offsets.astype(np.int64)
    mem = h.members.astype(np.int64)
    seen = {}
    lists = {}
    order = []
    singles = dups = 0
    for i in range(len(off) - 1):
        e = mem[off[i]:off[i + 1]].tolist()
        if len(e) == 0:
            raise InputError(f"hyperedge {i} is empty")
        if any(v < 0 or v >= h.n_nodes for v in e):
            raise InputError(f"hyperedge {i} has a node id outside [0, {h.n_nodes})")
        if len(set(e)) != len(e):
            raise InputError(f"hyperedge {i} repeats a node")
        if len(e) == 1:
            singles += 1
            continue
        key = tuple(sorted(e))
        if key in seen:
            dups += 1
            continue
        seen[key] = i
        order.append(key)
        lists.setdefault(len(key), []).append(key)
    by_size = {j: np.array(v, dtype=np.int64).reshape(-1, j) for j, v in lists.items()}
    return Normalised(h.n_nodes, by_size, singles, dups, order)


def _flat(nh: Normalised, j: int) -> np.ndarray:
    return np.ascontiguousarray(nh.edges(j).reshape(-1), dtype=np.uint32)


def count_exact(h, k: int) -> np.ndarray:
    """Exact counts per class (Algorithm 2 for k=3, Algorithm 3 for k=4)."""
    nh = h if isinstance(h, Normalised) else normalise(h)
    out = np.zeros(table(k).n_classes, dtype=np.int64)
    rc = lib().oracle_count_exact(k, nh.n_nodes, _flat(nh, 2), nh.count(2), _flat(nh, 3), nh.count(3),
                                  _flat(nh, 4), nh.count(4), out)
    if rc != 0:
        raise RuntimeError("oracle_count_exact failed")
    return out


def count_exact_threads(h, k: int, n_threads: int = 0):
    """count_exact with each step of Algorithm 2 / 3 spread over host threads
    (0: every core).  Returns (counts, threads used)."""
    nh = h if isinstance(h, Normalised) else normalise(h)
    out = np.zeros(table(k).n_classes, dtype=np.int64)
    used = lib().oracle_count_exact_threads(k, nh.n_nodes, _flat(nh, 2), nh.count(2), _flat(nh, 3), nh.count(3),
                                            _flat(nh, 4), nh.count(4), int(n_threads), out)
    if used < 0:
        raise RuntimeError("oracle_count_exact_threads failed")
    return out, used


def count_baseline(h, k: int):
    """Exact counts by the baseline of Section 4.1 (Algorithm 1): ESU on the
    clique projection of every hyperedge, keeping the candidates whose induced
    sub-hypergraph is connected.  Returns (counts, candidates, discarded)."""
    nh = h if isinstance(h, Normalised) else normalise(h)
    members = np.ascontiguousarray([v for e in nh.order for v in e], dtype=np.uint32)
    offsets = np.zeros(len(nh.order) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([len(e) for e in nh.order], dtype=np.int64)
    out = np.zeros(table(k).n_classes, dtype=np.int64)
    stats = np.zeros(2, dtype=np.int64)
    rc = lib().oracle_count_baseline(k, nh.n_nodes, members, offsets, len(nh.order), _flat(nh, 2), nh.count(2),
                                     _flat(nh, 3), nh.count(3), _flat(nh, 4), nh.count(4), out, stats)
    if rc != 0:
        raise RuntimeError("oracle_count_baseline failed")
    return out, int(stats[0]), int(stats[1])


def sampled_raw(h, k: int, samples: dict) -> np.ndarray:
    """Raw per-class counts of Algorithm 4 for explicit sample lists.

    ``samples[j]`` lists indices into the size-j hyperedges (first-occurrence
    order), with repetition for draws with replacement.
    """
    nh = h if isinstance(h, Normalised) else normalise(h)
    s = {j: np.ascontiguousarray(np.asarray(samples.get(j, []), dtype=np.int64)) for j in (2, 3, 4)}
    out = np.zeros(table(k).n_classes, dtype=np.int64)
    rc = lib().oracle_sampled_raw(k, nh.n_nodes, _flat(nh, 2), nh.count(2), _flat(nh, 3), nh.count(3),
                                  _flat(nh, 4), nh.count(4), s[2], len(s[2]), s[3], len(s[3]),
                                  s[4], len(s[4]), out)
    if rc != 0:
        raise RuntimeError("oracle_sampled_raw failed")
    return out


def scale_estimate(raw: np.ndarray, k: int, n_by_size: dict, s_by_size: dict) -> np.ndarray:
    """Correction of Algorithm 4: c * |E_maxcard| / (S_maxcard * countmax), in float64.

    A class whose stratum was not sampled (S_j = 0) is reported as 0.
    """
    t = table(k)
    est = np.zeros(t.n_classes, dtype=np.float64)
    for m in range(t.n_classes):
        j = t.maxcard[m]
        if s_by_size.get(j, 0) > 0:
            est[m] = float(raw[m]) * float(n_by_size.get(j, 0)) / (float(s_by_size[j]) * t.countmax[m])
    return est


def estimator_moments(h, k: int, s_by_size: dict):
    """Variance and excess kurtosis, per class, of Algorithm 4's corrected
    estimate with S_j draws with replacement from each stratum (Section 5).

    A class m is estimated from the stratum j of its largest hyperedges:
    est_m = |E_j| / (S_j countmax_m) * sum over the S_j draws of n_m(e), with
    n_m(e) the raw count of one sample e and the draws independent and
    uniform on E_j.  So Var(est_m) = |E_j|^2 / (S_j countmax_m^2) * v_m, v_m the
    variance of n_m(e) over E_j, and the excess kurtosis of the sum is that
    of n_m(e) divided by S_j.  n_m(e) comes from sampled_raw with e as the
    only sample.  Returns (var, kurt), float64; 0 where v_m = 0 or S_j = 0.
    """
    nh = h if isinstance(h, Normalised) else normalise(h)
    t = table(k)
    var = np.zeros(t.n_classes)
    kurt = np.zeros(t.n_classes)
    for j in range(2, k + 1):
        n_j, S = nh.count(j), s_by_size.get(j, 0)
        if n_j == 0 or S == 0:
            continue
        per = np.array([sampled_raw(nh, k, {j: [e]}) for e in range(n_j)], dtype=np.float64)
        for m in range(t.n_classes):
            if t.maxcard[m] != j:
                continue
            x = per[:, m]
            v = x.var()
            if v == 0.0:
                continue
            var[m] = float(n_j) ** 2 * v / (float(S) * t.countmax[m] ** 2)
            kurt[m] = (((x - x.mean()) ** 4).mean() / v ** 2 - 3.0) / S
    return var, kurt


def class_canon_c(k: int) -> list:
    buf = np.zeros(256, dtype=np.uint32)
    n = lib().oracle_class_canon(k, buf)
    return buf[:n].tolist()


def pattern_class_c(k: int, pattern: int) -> int:
    return lib().oracle_pattern_class(k, pattern)


ALLOC_PROPORTIONAL = 0
ALLOC_PAPER = 1


def sample_sizes(n_by_size: dict, k: int, fraction: float, allocation: int = ALLOC_PROPORTIONAL) -> dict:
    """Number of draws per stratum (Section 5: S_j samples from the hyperedges of size j).

    Proportional: S_j = ceil(fraction * |E_j|).  Paper split for k = 4
    (appendix: S_3 = 3 S_2, S_4 = 2 S_2): S = ceil(fraction * sum_j |E_j|),
    S_2 = floor(S / 6), S_3 = floor(S / 2), S_4 = S - S_2 - S_3, and a stratum
    with hyperedges gets at least one draw under this split (otherwise the
    classes of a stratum left undrawn would be estimated as 0, which the
    unbiasedness of Section 5 rules out).  An empty stratum gets no draw.
    """
    import math
    if allocation == ALLOC_PAPER and k == 4:
        s = math.ceil(fraction * float(sum(n_by_size.get(j, 0) for j in (2, 3, 4))))
        S = {2: s // 6, 3: s // 2}
        S[4] = s - S[2] - S[3]
        S = {j: max(S[j], 1) for j in S}
    else:
        S = {j: math.ceil(fraction * float(n_by_size.get(j, 0))) for j in range(2, k + 1)}
    return {j: (S.get(j, 0) if n_by_size.get(j, 0) > 0 else 0) for j in range(2, k + 1)}
