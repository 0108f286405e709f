"""Pins of the oracle's class table against closed forms and textbook facts.

Section 4.3 (and Fig. 1's caption) gives 6 classes of order 3; the order-4
class count follows from Burnside's lemma below.  Nothing here re-runs the
table's own canonicalisation.
"""
from itertools import permutations
from math import comb

import networkx as nx
import pytest

from oracle import core
from oracle.classes import subset_masks, table, is_connected


def _labelled_patterns(n):
    """Patterns (sets of subsets of size >= 2) on n labelled nodes: 2^(2^n - n - 1)."""
    return 2 ** (2 ** n - n - 1)


def _connected_labelled(n_max):
    """Connected labelled patterns by the exponential-formula recursion:
    a(n) = sum_{k=1..n} C(n-1, k-1) c(k) a(n-k), solved for c(n)."""
    a = {0: 1}
    for n in range(1, n_max + 1):
        a[n] = _labelled_patterns(n)
    c = {}
    for n in range(1, n_max + 1):
        c[n] = a[n] - sum(comb(n - 1, k - 1) * c[k] * a[n - k] for k in range(1, n))
    return c


def _burnside_classes(k, subsets):
    """Number of unlabelled patterns over the given subsets (all, connected or not):
    the mean over the k! permutations of 2^(cycles of the permutation on the subsets)."""
    total = 0
    perms = list(permutations(range(k)))
    for perm in perms:
        image = {}
        for m in subsets:
            img = 0
            for i in range(k):
                if (m >> i) & 1:
                    img |= 1 << perm[i]
            image[m] = img
        seen, cycles = set(), 0
        for m in subsets:
            if m in seen:
                continue
            cycles += 1
            x = m
            while x not in seen:
                seen.add(x)
                x = image[x]
        total += 2 ** cycles
    assert total % len(perms) == 0
    return total // len(perms)


def test_subset_encoding():
    assert subset_masks(3) == [3, 5, 6, 7]
    assert subset_masks(4) == [3, 5, 6, 7, 9, 10, 11, 12, 13, 14, 15]


@pytest.mark.parametrize("k", [3, 4])
def test_connected_labelled_pattern_count(k):
    c = _connected_labelled(4)
    assert (c[1], c[2], c[3], c[4]) == (1, 1, 12, 1990)
    t = table(k)
    assert sum(t.orbit_size) == c[k]
    assert sum(1 for x in t.class_of if x >= 0) == c[k]


def test_class_counts_by_burnside():
    # all unlabelled patterns: u(3) = 8, u(4) by Burnside; disconnected ones are
    # products of smaller connected classes (c_u(1) = c_u(2) = 1, c_u(3) = 6)
    u3 = _burnside_classes(3, subset_masks(3))
    u4 = _burnside_classes(4, subset_masks(4))
    assert u3 == 8
    assert u3 - 1 - 1 == 6 == table(3).n_classes           # minus {3-set: 2+1, 1+1+1}
    disconnected4 = 6 + 1 + 1 + 1                            # 3+1, 2+2, 2+1+1, 1+1+1+1
    assert u4 - disconnected4 == 171 == table(4).n_classes
    # with the 4-set itself present every pattern is connected: classes with maxcard 4
    others = [m for m in subset_masks(4) if m != 15]
    assert _burnside_classes(4, others) == sum(1 for mc in table(4).maxcard if mc == 4) == 90


@pytest.mark.parametrize("k", [3, 4])
def test_orbits_divide_group_order(k):
    t = table(k)
    fact = 6 if k == 3 else 24
    assert all(fact % o == 0 for o in t.orbit_size)


def test_order3_classes_are_the_six_of_the_paper():
    t = table(3)
    # path, triangle, 3-edge alone, 3-edge + 1 / 2 / 3 pairs
    assert t.canon_masks == [3, 7, 8, 9, 11, 15]
    assert t.n_hyperedges == [2, 3, 1, 2, 3, 4]
    assert list(zip(t.maxcard, t.countmax)) == [(2, 2), (2, 3), (3, 1), (3, 1), (3, 1), (3, 1)]


def test_pairs_only_order4_classes_are_the_connected_graphs():
    t = table(4)
    pair_bits = [i for i, m in enumerate(subset_masks(4)) if bin(m).count("1") == 2]
    atlas = [g for g in nx.graph_atlas_g() if g.number_of_nodes() == 4 and nx.is_connected(g)]
    assert len(atlas) == 6
    found = []
    for cls, c in enumerate(t.canon_masks):
        if t.maxcard[cls] != 2:
            continue
        g = nx.Graph()
        g.add_nodes_from(range(4))
        for i in pair_bits:
            if (c >> i) & 1:
                m = subset_masks(4)[i]
                g.add_edge(*[v for v in range(4) if (m >> v) & 1])
        matches = [j for j, a in enumerate(atlas) if nx.is_isomorphic(a, g)]
        assert len(matches) == 1
        found.append(matches[0])
    assert sorted(found) == list(range(6))
    # and 38 connected labelled graphs on 4 nodes
    assert sum(t.orbit_size[c] for c in range(t.n_classes) if t.maxcard[c] == 2) == 38


def test_maxcard_countmax_histogram():
    from collections import Counter
    t = table(4)
    assert Counter(t.maxcard) == {2: 6, 3: 75, 4: 90}
    # every class with maxcard 4 has exactly one 4-set hyperedge
    assert all(cm == 1 for mc, cm in zip(t.maxcard, t.countmax) if mc == 4)
    # maxcard 3 classes: countmax between 1 and 4 (the 4 triples of 4 nodes)
    assert set(cm for mc, cm in zip(t.maxcard, t.countmax) if mc == 3) == {1, 2, 3, 4}


@pytest.mark.parametrize("k", [3, 4])
def test_c_oracle_class_list_agrees(k):
    t = table(k)
    assert core.class_canon_c(k) == t.canon_masks
    for p in range(1 << t.n_bits):
        assert core.pattern_class_c(k, p) == t.class_of[p]


def test_connectivity_of_small_patterns():
    # a single pair leaves two of four nodes uncovered; a 4-edge alone is connected
    assert not is_connected(1, 4)
    assert is_connected(1 << 10, 4)
    # two disjoint pairs {0,1},{2,3}: disconnected; adding {1,2} connects them
    p = (1 << 0) | (1 << 7)
    assert not is_connected(p, 4)
    assert is_connected(p | (1 << 2), 4)
