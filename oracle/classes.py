"""Isomorphism classes of k-node sub-hypergraph patterns (oracle; test infrastructure only).

Follows Section 4.3 (Fig. 3a): every pattern of interactions among k nodes is
generated under every relabelling of the nodes, and relabellings of one
pattern form one class.  Only connected patterns are motifs (Definition of
higher-order motifs, Section 3).

Encoding of a pattern (a reading fixed here, since the paper numbers no
classes): the k nodes of a candidate set take local positions 0..k-1 in
ascending node-id order.  The candidate sub-hyperedges are the subsets of
{0..k-1} of size >= 2 (the empty set and singletons are ignored, as the
fill-in step of Section 4.3 allows), listed in ascending order of their bit
mask; pattern bit i is set when the i-th subset is a hyperedge.  For k=4 the
subset masks are 3,5,6,7,9,10,11,12,13,14,15; for k=3 they are 3,5,6,7.

The canonical form of a pattern is the smallest pattern value over all k!
relabellings; class ids rank the distinct canonical forms of connected
patterns in ascending order.
"""
from __future__ import annotations

from functools import lru_cache
from itertools import permutations


def subset_masks(k: int) -> list[int]:
    """Subsets of {0..k-1} with at least two members, ascending by mask value."""
    return [m for m in range(1 << k) if bin(m).count("1") >= 2]


def _relabel_subset(mask: int, perm) -> int:
    out = 0
    for i, target in enumerate(perm):
        if (mask >> i) & 1:
            out |= 1 << target
    return out


def relabel(pattern: int, perm, k: int) -> int:
    """Pattern after moving local node i to position perm[i]."""
    masks = subset_masks(k)
    index = {m: i for i, m in enumerate(masks)}
    out = 0
    for i, m in enumerate(masks):
        if (pattern >> i) & 1:
            out |= 1 << index[_relabel_subset(m, perm)]
    return out


def hyperedges_of(pattern: int, k: int) -> list[int]:
    masks = subset_masks(k)
    return [m for i, m in enumerate(masks) if (pattern >> i) & 1]


def is_connected(pattern: int, k: int) -> bool:
    """True when every one of the k nodes lies in one component of the pattern's hyperedges."""
    parent = list(range(k))

    def find(x):
        while parent[x] != x:
            x = parent[x]
        return x
    covered = 0
    for m in hyperedges_of(pattern, k):
        covered |= m
        nodes = [i for i in range(k) if (m >> i) & 1]
        for v in nodes[1:]:
            a, b = find(nodes[0]), find(v)
            if a != b:
                parent[a] = b
    if covered != (1 << k) - 1:
        return False
    return len({find(i) for i in range(k)}) == 1


def canonical(pattern: int, k: int) -> int:
    return min(relabel(pattern, p, k) for p in permutations(range(k)))


class ClassTable:
    """All patterns of k nodes, their canonical forms and class ids."""

    def __init__(self, k: int):
        if k not in (3, 4):
            raise ValueError("k must be 3 or 4")
        self.k = k
        self.masks = subset_masks(k)
        self.n_bits = len(self.masks)
        n_patterns = 1 << self.n_bits
        canon = [canonical(p, k) for p in range(n_patterns)]
        conn = [is_connected(p, k) for p in range(n_patterns)]
        self.canon_masks = sorted({canon[p] for p in range(n_patterns) if conn[p]})
        rank = {c: i for i, c in enumerate(self.canon_masks)}
        self.class_of = [rank[canon[p]] if conn[p] else -1 for p in range(n_patterns)]
        self.n_classes = len(self.canon_masks)
        self.orbit_size = [0] * self.n_classes
        for p in range(n_patterns):
            if self.class_of[p] >= 0:
                self.orbit_size[self.class_of[p]] += 1
        self.maxcard = []
        self.countmax = []
        self.n_hyperedges = []
        for c in self.canon_masks:
            sizes = [bin(m).count("1") for m in hyperedges_of(c, k)]
            mc = max(sizes)
            self.maxcard.append(mc)
            self.countmax.append(sizes.count(mc))
            self.n_hyperedges.append(len(sizes))

    def pattern_of(self, present) -> int:
        """Pattern from a predicate over subset masks (fill-in result)."""
        p = 0
        for i, m in enumerate(self.masks):
            if present(m):
                p |= 1 << i
        return p


@lru_cache(maxsize=None)
def table(k: int) -> ClassTable:
    return ClassTable(k)
