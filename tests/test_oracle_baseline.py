"""Pins of the oracle's baseline count (Algorithm 1, Section 4.1): ESU on the
clique projection, keeping the candidates whose induced sub-hypergraph is
connected.  Its counts must be the plain definition's (brute force over all
k-node sets) and Algorithm 2/3's; its candidates must be the connected k-node
sets of the projection, counted here with networkx."""
from itertools import combinations

import networkx as nx
import numpy as np
import pytest

import workloads as W
from oracle import brute, core
from oracle.classes import table


def _projection_connected_sets(h, k: int) -> int:
    nh = core.normalise(h)
    G = nx.Graph()
    for e in nh.order:
        G.add_edges_from(combinations(e, 2))
    return sum(1 for V in combinations(sorted(G.nodes), k) if nx.is_connected(G.subgraph(V)))


def test_one_hyperedge_above_the_order_is_all_discarded():
    # the projection of a 4-node hyperedge is K4: its four triangles are
    # candidates at order 3, and none holds a hyperedge (Section 4.1, the
    # failure of the projection)
    h = W.from_lists([[0, 1, 2, 3]])
    counts, cand, disc = core.count_baseline(h, 3)
    assert cand == 4 and disc == 4 and not counts.any()
    counts, cand, disc = core.count_baseline(h, 4)
    assert cand == 1 and disc == 0 and counts.sum() == 1
    assert np.array_equal(counts, brute.count_brute(h, 4))


def test_pair_and_triangle_hyperedge():
    # {0,1} and {1,2,3}: the projection has the connected triples 012, 013 and
    # 123; only 123 induces a connected sub-hypergraph
    h = W.from_lists([[0, 1], [1, 2, 3]])
    counts, cand, disc = core.count_baseline(h, 3)
    assert (cand, disc) == (3, 2)
    assert np.array_equal(counts, brute.count_brute(h, 3))
    assert counts.sum() == 1


def test_five_node_hyperedge_bridges_nothing():
    # a 5-node hyperedge joins its members in the projection but never lies
    # inside a 4-node set: only the pairwise path 0-1-2-3 is a motif
    h = W.from_lists([[0, 1], [1, 2], [2, 3], [0, 4, 5, 6, 7]])
    counts, cand, disc = core.count_baseline(h, 4)
    assert counts.sum() == 1
    assert cand == _projection_connected_sets(h, 4)
    assert disc == cand - 1


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("k", [3, 4])
def test_matches_definition_and_projection(seed, k):
    h = W.random_small(300 + seed, 14, 24, {1: 0.05, 2: 0.4, 3: 0.3, 4: 0.15, 5: 0.05, 6: 0.05}, allow_dups=True)
    counts, cand, disc = core.count_baseline(h, k)
    assert np.array_equal(counts, brute.count_brute(h, k))
    assert cand == _projection_connected_sets(h, k)
    assert disc == cand - int(counts.sum())
    assert len(counts) == table(k).n_classes


@pytest.mark.parametrize("k", [3, 4])
def test_matches_algorithms_2_and_3(k):
    h = W.random_small(11, 40, 200, {1: 0.05, 2: 0.5, 3: 0.3, 4: 0.1, 5: 0.05}, allow_dups=True)
    counts, cand, disc = core.count_baseline(h, k)
    assert np.array_equal(counts, core.count_exact(h, k))
    assert cand > counts.sum() and disc == cand - int(counts.sum())
