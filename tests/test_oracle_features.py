"""Pins of the features oracle (the learned proposal's 16 inputs per
hyperedge): values worked out by hand on a five-node example, invariance
under node relabelling, indifference to duplicate and oversized hyperedges,
and the per-stratum standardisation."""
import math

import numpy as np

import workloads as W
from oracle import features

L = math.log


def _hand():
    # pairs {0,1} {0,2} {1,2} {3,4}, the triple {0,1,3}, the quadruple {0,1,2,3}
    return W.from_lists([(0, 1), (0, 2), (1, 2), (3, 4), (0, 1, 3), (0, 1, 2, 3)], 5)


def test_hand_example():
    """Degrees: d2 = 2,2,2,1,1; d3 = 1,1,0,1,0; d4 = 1,1,1,1,0 for nodes 0..4."""
    X = features.raw_features(_hand(), 4)
    want = np.array([
        # pair {0,1}: member pairs joined 1/1, wedges C(2,2)+C(2,2) = 2, d2 d3 sum 4, d2 d2 product 4
        [1, 0, 0, L(3), L(3), L(3), L(2), L(2), L(2), L(2), 1.0, 0.5 * L(3), 0.5 * L(5), 0.5 * L(5), 0, 1],
        [1, 0, 0, L(3), L(3), L(3), L(1.5), L(2), L(2), L(2), 1.0, 0.5 * L(3), 0.5 * L(3), 0.5 * L(5), 0, 1],
        [1, 0, 0, L(3), L(3), L(3), L(1.5), L(2), L(2), L(2), 1.0, 0.5 * L(3), 0.5 * L(3), 0.5 * L(5), 0, 1],
        # pair {3,4}: d2 1,1; d3 1,0; d4 1,0
        [1, 0, 0, L(2), L(2), L(2), L(1.5), L(2), L(1.5), L(2), 1.0, 0.0, 0.5 * L(2), 0.5 * L(2), 0, 1],
        # triple {0,1,3}: mean d2 5/3; pairs joined 1 of 3; d2 products 4+2+2
        [0, 1, 0, L(8 / 3), L(3), L(2), L(2), L(2), L(2), L(2), 1 / 3, 0.5 * L(3), 0.5 * L(6), L(3), 0, 1],
        # quadruple {0,1,2,3}: mean d2 7/4, mean d3 3/4; pairs joined 3 of 6; d2 products 18
        [0, 0, 1, L(11 / 4), L(3), L(2), L(7 / 4), L(2), L(2), L(2), 0.5, L(2), 0.5 * L(6), 0.5 * L(19), 0, 1],
    ])
    np.testing.assert_allclose(X, want, rtol=0, atol=1e-15)


def test_stars_count_pairwise_triples():
    """Column 14 is log(1 + sum C(d2, 3)) / 3: a star centre with 5 leaves has C(5,3) = 10."""
    h = W.from_lists([(0, i) for i in range(1, 6)], 6)
    X = features.raw_features(h, 3)
    assert np.allclose(X[:, 14], L(11) / 3)
    assert np.allclose(X[:, 11], 0.5 * L(1 + 10))      # C(5,2) at the centre, 0 at the leaf


def test_relabelling_and_set_semantics():
    """Rows follow first occurrence; relabelling nodes, repeating a hyperedge
    or adding one of size 5 changes no feature."""
    h = W.random_small(77, 25, 120, {2: 0.5, 3: 0.3, 4: 0.2})
    X = features.features(h, 4)
    perm = np.random.default_rng(1).permutation(h.n_nodes)
    hp = W.Hypergraph(h.n_nodes, perm[h.members], h.offsets.copy())
    np.testing.assert_allclose(features.features(hp, 4), X, atol=1e-12)
    edges = h.edges()
    hx = W.from_lists(edges + [edges[0], [0, 1, 2, 3, 4]], h.n_nodes)
    np.testing.assert_allclose(features.features(hx, 4), X, atol=1e-12)


def test_standardisation():
    h = W.random_small(78, 40, 300, {2: 0.5, 3: 0.3, 4: 0.2})
    b = features.strata_bounds(h, 4)
    Z = features.features(h, 4)
    for s in range(3):
        blk = Z[b[s]:b[s + 1]]
        for f in features.STANDARDISED:
            col = blk[:, f]
            if np.all(col == 0):
                continue
            assert abs(col.mean()) < 1e-9 and abs(col.std() - 1) < 1e-9
