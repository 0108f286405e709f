"""Pins of the oracle's exact counts (Algorithms 2 and 3) against the plain
definition, hand-derived fixtures, closed forms and graph identities."""
import json
import os
from itertools import combinations
from math import comb

import networkx as nx
import numpy as np
import pytest

import workloads as W
from oracle import brute, core
from oracle.classes import subset_masks, table


def _pattern(nodes, inside, k):
    pos = {v: i for i, v in enumerate(sorted(nodes))}
    masks = subset_masks(k)
    p = 0
    for e in inside:
        m = 0
        for v in e:
            m |= 1 << pos[v]
        p |= 1 << masks.index(m)
    return p


def _expected_from_hand(entries, k):
    t = table(k)
    out = np.zeros(t.n_classes, dtype=np.int64)
    for occ in entries:
        cls = t.class_of[_pattern(occ["nodes"], occ["inside"], k)]
        assert cls >= 0, "hand fixture lists a disconnected set"
        out[cls] += 1
    return out


def _hand_examples(golden_dir):
    with open(os.path.join(golden_dir, "hand_examples.json")) as f:
        return json.load(f)["examples"]


@pytest.mark.parametrize("k", [3, 4])
def test_hand_examples(golden_dir, k):
    for ex in _hand_examples(golden_dir):
        h = W.from_lists(ex["edges"], ex["n_nodes"])
        want = _expected_from_hand(ex[f"k{k}"], k)
        assert np.array_equal(core.count_exact(h, k), want), ex["name"]
        assert np.array_equal(brute.count_brute(h, k), want), ex["name"]


SIZE_MIXES = [
    {2: 0.6, 3: 0.3, 4: 0.1},
    {1: 0.05, 2: 0.45, 3: 0.3, 4: 0.15, 5: 0.05},
    {2: 0.2, 3: 0.5, 4: 0.3},
    {2: 1.0},
]


@pytest.mark.parametrize("seed", range(24))
def test_algorithms_match_brute_force(seed):
    mix = SIZE_MIXES[seed % len(SIZE_MIXES)]
    n = 10 + seed % 7
    h = W.random_small(seed, n, 12 + 3 * (seed % 9), mix, allow_dups=bool(seed % 2))
    for k in (3, 4):
        assert np.array_equal(core.count_exact(h, k), brute.count_brute(h, k)), (seed, k)


def _count_connected_sets(h, k):
    """k-sets whose induced sub-hypergraph is connected, via networkx on the
    graph linking nodes that share a hyperedge inside the set."""
    nh = core.normalise(h)
    edges = [e for j, arr in nh.by_size.items() if j <= k for e in arr.tolist()]
    nodes = sorted({v for e in edges for v in e})
    total = 0
    for V in combinations(nodes, k):
        s = set(V)
        g = nx.Graph()
        g.add_nodes_from(V)
        for e in edges:
            if set(e) <= s:
                g.add_edges_from((e[0], x) for x in e[1:])
        total += nx.is_connected(g)
    return total


@pytest.mark.parametrize("seed", range(6))
def test_sum_equals_connected_sets(seed):
    h = W.random_small(100 + seed, 12, 20, {2: 0.5, 3: 0.35, 4: 0.15})
    for k in (3, 4):
        assert core.count_exact(h, k).sum() == _count_connected_sets(h, k)


def _relabel(h, perm):
    return W.Hypergraph(h.n_nodes, perm[h.members.astype(np.int64)].astype(np.uint32), h.offsets.copy())


@pytest.mark.parametrize("seed", range(4))
def test_relabelling_invariance(seed):
    h = W.random_small(200 + seed, 40, 160, {2: 0.5, 3: 0.3, 4: 0.2})
    perm = np.random.default_rng(seed).permutation(h.n_nodes)
    for k in (3, 4):
        assert np.array_equal(core.count_exact(h, k), core.count_exact(_relabel(h, perm), k))


def test_disjoint_union_is_additive():
    a = W.random_small(300, 30, 120, {2: 0.5, 3: 0.3, 4: 0.2})
    b = W.random_small(301, 25, 90, {2: 0.4, 3: 0.4, 4: 0.2})
    edges = a.edges() + [[v + a.n_nodes for v in e] for e in b.edges()]
    u = W.from_lists(edges, a.n_nodes + b.n_nodes)
    for k in (3, 4):
        assert np.array_equal(core.count_exact(u, k), core.count_exact(a, k) + core.count_exact(b, k))


def test_larger_hyperedges_singletons_and_repeats_change_nothing():
    h = W.random_small(400, 30, 120, {2: 0.5, 3: 0.3, 4: 0.2})
    rng = np.random.default_rng(0)
    extra = [sorted(rng.choice(30, size=s, replace=False).tolist()) for s in (5, 6, 7, 5)]
    singles = [[int(v)] for v in rng.choice(30, size=5, replace=False)]
    repeats = h.edges()[:10]
    base3, base4 = core.count_exact(h, 3), core.count_exact(h, 4)
    h4 = W.from_lists(h.edges() + extra + singles + repeats, 30)
    assert np.array_equal(core.count_exact(h4, 4), base4)
    four_edges = [sorted(rng.choice(30, size=4, replace=False).tolist()) for _ in range(3)]
    h3 = W.from_lists(h.edges() + extra + four_edges + singles + repeats, 30)
    # 4-node hyperedges cannot lie inside a 3-node set
    assert np.array_equal(core.count_exact(h3, 3), core.count_exact(W.from_lists(h.edges() + four_edges, 30), 3))
    assert np.array_equal(core.count_exact(W.from_lists(h.edges() + four_edges, 30), 3), base3)


@pytest.mark.parametrize("n", [4, 7, 11])
def test_complete_graph(n):
    h = W.from_lists([list(e) for e in combinations(range(n), 2)], n)
    t3, t4 = table(3), table(4)
    c3, c4 = core.count_exact(h, 3), core.count_exact(h, 4)
    tri = t3.class_of[_pattern([0, 1, 2], [[0, 1], [0, 2], [1, 2]], 3)]
    k4 = t4.class_of[_pattern([0, 1, 2, 3], [list(e) for e in combinations(range(4), 2)], 4)]
    assert c3[tri] == comb(n, 3) and c3.sum() == comb(n, 3)
    assert c4[k4] == comb(n, 4) and c4.sum() == comb(n, 4)


@pytest.mark.parametrize("n", [4, 6, 9])
def test_complete_hypergraph(n):
    for k in (3, 4):
        edges = [list(e) for s in range(2, k + 1) for e in combinations(range(n), s)]
        c = core.count_exact(W.from_lists(edges, n), k)
        full = table(k).class_of[(1 << table(k).n_bits) - 1]
        assert c[full] == comb(n, k) and c.sum() == comb(n, k)


@pytest.mark.parametrize("leaves", [3, 5, 12])
def test_star(leaves):
    h = W.from_lists([[0, v] for v in range(1, leaves + 1)], leaves + 1)
    path = table(3).class_of[_pattern([0, 1, 2], [[0, 1], [0, 2]], 3)]
    star = table(4).class_of[_pattern([0, 1, 2, 3], [[0, 1], [0, 2], [0, 3]], 4)]
    c3, c4 = core.count_exact(h, 3), core.count_exact(h, 4)
    assert c3[path] == comb(leaves, 2) and c3.sum() == comb(leaves, 2)
    assert c4[star] == comb(leaves, 3) and c4.sum() == comb(leaves, 3)


def test_single_four_edge():
    h = W.from_lists([[3, 1, 2, 0]], 4)
    c4 = core.count_exact(h, 4)
    assert c4[table(4).class_of[1 << 10]] == 1 and c4.sum() == 1
    assert core.count_exact(h, 3).sum() == 0


def _graph_edges(seed, n, p):
    g = nx.gnp_random_graph(n, p, seed=seed)
    return g, [list(e) for e in g.edges()]


@pytest.mark.parametrize("seed,n,p", [(0, 30, 0.2), (1, 50, 0.12), (2, 40, 0.35)])
def test_graph_only_order3_by_matrix_algebra(seed, n, p):
    g, edges = _graph_edges(seed, n, p)
    A = nx.to_numpy_array(g, nodelist=range(n), dtype=np.int64)
    d = A.sum(axis=1)
    tri = int(np.trace(A @ A @ A)) // 6
    wedges = int(sum(comb(int(x), 2) for x in d)) - 3 * tri
    c = core.count_exact(W.from_lists(edges, n), 3)
    t = table(3)
    assert c[t.class_of[_pattern([0, 1, 2], [[0, 1], [0, 2], [1, 2]], 3)]] == tri
    assert c[t.class_of[_pattern([0, 1, 2], [[0, 1], [0, 2]], 3)]] == wedges
    assert c.sum() == tri + wedges


@pytest.mark.parametrize("seed,n,p", [(0, 30, 0.2), (1, 45, 0.15), (2, 28, 0.4)])
def test_graph_only_order4_by_matrix_algebra(seed, n, p):
    """Induced 4-node graphlet counts from subgraph counts that matrix powers give."""
    g, edges = _graph_edges(seed, n, p)
    A = nx.to_numpy_array(g, nodelist=range(n), dtype=np.int64)
    A2 = A @ A
    A3 = A2 @ A
    d = A.sum(axis=1)
    m = len(edges)
    T = int(np.trace(A3)) // 6
    K4 = sum(1 for c in nx.enumerate_all_cliques(g) if len(c) == 4)
    star_non = sum(comb(int(x), 3) for x in d)
    path_non = sum(int((d[u] - 1) * (d[v] - 1)) for u, v in edges) - 3 * T
    c4_non = (int(np.trace(A2 @ A2)) - 2 * m - 2 * int((d * (d - 1)).sum())) // 8
    paw_non = int(sum((A3[v, v] // 2) * (d[v] - 2) for v in range(n)))
    diamond_non = sum(comb(int(A2[u, v]), 2) for u, v in edges)
    diamond = diamond_non - 6 * K4
    C4 = c4_non - diamond - 3 * K4
    paw = paw_non - 4 * diamond - 12 * K4
    star = star_non - paw - 2 * diamond - 4 * K4
    P4 = path_non - 2 * paw - 4 * C4 - 6 * diamond - 12 * K4
    t = table(4)
    shapes = {
        "P4": ([[0, 1], [1, 2], [2, 3]], P4),
        "star": ([[0, 1], [0, 2], [0, 3]], star),
        "C4": ([[0, 1], [1, 2], [2, 3], [0, 3]], C4),
        "paw": ([[0, 1], [0, 2], [1, 2], [0, 3]], paw),
        "diamond": ([[0, 1], [0, 2], [1, 2], [0, 3], [1, 3]], diamond),
        "K4": ([list(e) for e in combinations(range(4), 2)], K4),
    }
    c = core.count_exact(W.from_lists(edges, n), 4)
    for name, (inside, want) in shapes.items():
        assert c[t.class_of[_pattern([0, 1, 2, 3], inside, 4)]] == want, name
    assert c.sum() == sum(v for _, v in shapes.values())


def test_workload_order3_matches_brute_force_on_a_node_subset():
    """The order-3 workload restricted to its 60 busiest nodes, both routes."""
    h = W.cfg0_facetoface_k3()
    keep = set(range(60))
    sub = W.from_lists([e for e in h.edges() if set(e) <= keep], 60)
    assert np.array_equal(core.count_exact(sub, 3), brute.count_brute(sub, 3))


def test_input_errors():
    with pytest.raises(core.InputError):
        core.normalise(W.from_lists([[0, 1], [2, 2]], 3))
    with pytest.raises(core.InputError):
        core.normalise(W.from_lists([[0, 5]], 3))
    with pytest.raises(core.InputError):
        core.normalise(W.Hypergraph(3, np.array([0, 1], np.uint32), np.array([0, 0, 2], np.uint64)))


@pytest.mark.parametrize("seed", range(12))
def test_threaded_algorithms_match_brute_force(seed):
    """Algorithms 2 and 3 spread over host threads give the single-thread
    counts and brute force's (set semantics of `visited`)."""
    mix = SIZE_MIXES[seed % len(SIZE_MIXES)]
    h = W.random_small(500 + seed, 10 + seed % 9, 20 + 5 * (seed % 7), mix, allow_dups=bool(seed % 2))
    for k in (3, 4):
        want = brute.count_brute(h, k)
        for threads in (1, 3, 8):
            got, used = core.count_exact_threads(h, k, threads)
            assert used == threads
            assert np.array_equal(got, want), (seed, k, threads)


def test_threaded_matches_single_thread_on_workloads(golden_dir):
    with open(os.path.join(golden_dir, "workload_counts.json")) as f:
        cases = {(c["workload"], c["k"]): np.array(c["counts"]) for c in json.load(f)["cases"] if "copy" not in c}
    h = W.cfg0_facetoface_k3(0)
    assert np.array_equal(core.count_exact_threads(h, 3)[0], cases[("facetoface_N200_E2000", 3)])
    h = W.scaled_communication(0.004, 0)
    assert np.array_equal(core.count_exact_threads(h, 4)[0], cases[("communication_scaled_0.004", 4)])
