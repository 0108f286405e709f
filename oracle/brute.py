"""Brute force over all k-node subsets: the plain definition (oracle; test infrastructure only).

For every k-subset V' of the nodes, build the vertex-induced sub-hypergraph
H[V'] = (V', {e in E : e subset of V'}) (Definition of the vertex-induced
sub-hypergraph, Section 3), keep it when it is connected (higher-order motif
of order k, Section 3) and add one to its isomorphism class (Definition of
hypergraph isomorphism, Section 3).  Only feasible for tiny inputs.
"""
from __future__ import annotations

from itertools import combinations

import numpy as np

from .classes import table
from .core import Normalised, normalise


def count_brute(h, k: int, nodes=None) -> np.ndarray:
    nh = h if isinstance(h, Normalised) else normalise(h)
    t = table(k)
    present = set()
    for j, arr in nh.by_size.items():
        if j <= k:
            present.update(tuple(r) for r in arr.tolist())
    if nodes is None:
        touched = sorted({v for e in present for v in e})
    else:
        touched = sorted(nodes)
    counts = np.zeros(t.n_classes, dtype=np.int64)
    for V in combinations(touched, k):
        def has(mask, V=V):
            return tuple(V[i] for i in range(k) if (mask >> i) & 1) in present
        cls = t.class_of[t.pattern_of(has)]
        if cls >= 0:
            counts[cls] += 1
    return counts


def connected_sets_brute(h, k: int) -> int:
    """Number of k-node sets whose induced sub-hypergraph is connected."""
    return int(count_brute(h, k).sum())
