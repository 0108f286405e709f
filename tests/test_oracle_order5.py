"""Pins of the order-5 oracle: the canonical form is invariant under
relabelling and separates the two-hyperedge shapes exactly as their
(sizes, overlap) types do; connectivity and maxcard on hand-worked
patterns; brute force agrees with an independent pure-Python brute force;
the census identity (every hyperedge sampled once gives countmax x exact)."""
import itertools
import random

import numpy as np
import pytest

import workloads as W
from oracle import core, order5


def _py_pattern(V, edges_set):
    p = 0
    for b, m in enumerate(order5.SUB_MASKS):
        sub = tuple(V[i] for i in range(5) if (m >> i) & 1)
        if sub in edges_set:
            p |= 1 << b
    return p


def _py_relabel(p, perm):
    out = 0
    for b, m in enumerate(order5.SUB_MASKS):
        if (p >> b) & 1:
            img = 0
            for i in range(5):
                if (m >> i) & 1:
                    img |= 1 << perm[i]
            out |= 1 << order5.SUB_MASKS.index(img)
    return out


def _py_canonical(p):
    return min(_py_relabel(p, perm) for perm in itertools.permutations(range(5)))


def test_canonical_invariant_under_relabelling():
    rng = random.Random(1)
    for _ in range(300):
        p = rng.getrandbits(26)
        perm = list(range(5))
        rng.shuffle(perm)
        c = order5.canonical(p)
        assert order5.canonical(_py_relabel(p, perm)) == c
        assert c <= p
    for p in (0b1, 1 << 25, (1 << 26) - 1, 0b1010110):
        assert order5.canonical(p) == _py_canonical(p)


def test_two_hyperedge_classes_are_their_overlap_types():
    """Two distinct hyperedges inside five nodes: their isomorphism types are
    the triples (smaller size a, larger size b, overlap i) with a + b - i <= 5
    and i < a when a = b; the canonical forms of all 325 two-bit patterns
    must number exactly these."""
    types = set()
    for x, y in itertools.combinations(order5.SUB_MASKS, 2):
        a, b = sorted((bin(x).count("1"), bin(y).count("1")))
        types.add((a, b, bin(x & y).count("1")))
    forms = {order5.canonical((1 << i) | (1 << j)) for i, j in itertools.combinations(range(26), 2)}
    want = {(a, b, i) for a in range(2, 6) for b in range(a, 6) for i in range(0, a + 1)
            if a + b - i <= 5 and not (a == b and i == a) and i <= b}
    assert types == want
    assert len(forms) == len(want)
    assert len({order5.canonical(1 << i) for i in range(26)}) == 4     # one hyperedge: its size


def test_connectivity_and_maxcard_hand_cases():
    def pat(*subsets):
        return sum(1 << order5.SUB_MASKS.index(sum(1 << v for v in s)) for s in subsets)
    assert order5.connected(pat((0, 1), (1, 2), (2, 3), (3, 4)))            # a path
    assert not order5.connected(pat((0, 1), (2, 3, 4)))
    assert not order5.connected(pat((0, 1, 2, 3)))                           # node 4 alone
    assert order5.connected(pat((0, 1, 2, 3, 4)))
    assert order5.maxcard(pat((0, 1), (1, 2, 3), (2, 3, 4), (0, 4))) == (3, 2)
    assert order5.maxcard(pat((0, 1, 2, 3, 4), (0, 1))) == (5, 1)


@pytest.mark.parametrize("seed", range(6))
def test_brute_force_matches_python(seed):
    h = W.random_small(800 + seed, 8 + seed % 3, 14 + 2 * seed, {2: 0.45, 3: 0.3, 4: 0.15, 5: 0.1},
                       allow_dups=bool(seed % 2))
    nh = core.normalise(h)
    edges = {tuple(e) for e in nh.order if len(e) <= 5}
    want = {}
    for V in itertools.combinations(range(h.n_nodes), 5):
        p = _py_pattern(V, edges)
        if p and order5.connected(p):
            c = _py_canonical(p)
            want[c] = want.get(c, 0) + 1
    assert order5.exact_brute(h) == want


@pytest.mark.parametrize("seed", range(6))
def test_census_is_countmax_times_exact(seed):
    """Each hyperedge of size 2..5 sampled once: a 5-set of class m is found
    once from each of its countmax largest hyperedges (Section 5)."""
    h = W.random_small(850 + seed, 10 + seed, 22 + 3 * seed, {2: 0.4, 3: 0.3, 4: 0.2, 5: 0.1})
    nh = core.normalise(h)
    exact = order5.exact_brute(h)
    raw = order5.sampled_raw(h, {j: np.arange(nh.count(j)) for j in (2, 3, 4, 5)})
    assert set(raw) == set(exact)
    for c, n in exact.items():
        assert raw[c] == order5.maxcard(c)[1] * n
    est = order5.scale(raw, {j: nh.count(j) for j in (2, 3, 4, 5)}, {j: nh.count(j) for j in (2, 3, 4, 5)})
    assert all(abs(est[c] - exact[c]) < 1e-9 for c in exact)


def test_relabelling_invariance():
    h = W.random_small(870, 11, 30, {2: 0.5, 3: 0.3, 4: 0.1, 5: 0.1})
    perm = np.random.default_rng(2).permutation(h.n_nodes)
    hp = W.Hypergraph(h.n_nodes, perm[h.members.astype(np.int64)].astype(np.uint32), h.offsets.copy())
    assert order5.exact_brute(hp) == order5.exact_brute(h)
