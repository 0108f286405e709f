"""Pins of the configuration-model null and of the motif-profile measures
(Section 6.3): the chain keeps degrees and sizes and repeats no node, its
draws are uniform over every hypergraph with the same degree and size
sequences (enumerated by brute force on a tiny one), and the profile and
accuracy measures agree with hand-worked values and their defining
properties."""
import itertools
from collections import Counter

import numpy as np
import pytest
from scipy import stats as sps

import workloads as W
from oracle import core, nulls, profiles


@pytest.mark.parametrize("seed", range(4))
def test_config_model_keeps_degrees_and_sizes(seed):
    h = W.random_small(700 + seed, 25, 90, {2: 0.4, 3: 0.3, 4: 0.2, 6: 0.1})
    m, o = profiles.config_model(h, sweeps=6, seed=seed, copy=3)
    nulls.check_null_invariants(h, m, o)
    m2, o2 = profiles.config_model(h, sweeps=6, seed=seed, copy=3)
    assert np.array_equal(m, m2) and np.array_equal(o, o2)
    m3, _ = profiles.config_model(h, sweeps=6, seed=seed, copy=4)
    assert not np.array_equal(m, m3)
    # every hyperedge stored ascending
    off = o.astype(np.int64)
    for i in range(len(off) - 1):
        e = m[off[i]:off[i + 1]]
        assert np.all(np.diff(e.astype(np.int64)) > 0)


def _states(sizes, degree):
    """Every assignment of node sets (in hyperedge order) with these sizes and degrees."""
    n = len(degree)
    out = []
    for combo in itertools.product(*[itertools.combinations(range(n), s) for s in sizes]):
        d = np.zeros(n, dtype=int)
        for e in combo:
            d[list(e)] += 1
        if np.array_equal(d, degree):
            out.append(combo)
    return out


def test_config_model_draws_are_uniform():
    """Symmetric moves keep the uniform distribution: on a tiny hypergraph,
    3,000 independent chains land on each of the 90 valid hypergraphs about
    equally often (chi-square), and reach every one of them."""
    edges = [(0, 1), (1, 2), (2, 3), (0, 3)]
    h = W.from_lists(edges, 4)
    nh = core.normalise(h)
    sizes = [len(e) for e in nh.order]
    deg = nulls.degree_sequence(np.array([v for e in nh.order for v in e]),
                                np.cumsum([0] + sizes), 4)
    states = _states(sizes, deg)
    assert len(states) == 90
    seen = Counter()
    runs = 3000
    for c in range(runs):
        m, o = profiles.config_model(h, sweeps=8, seed=9, copy=c)
        off = o.astype(np.int64)
        seen[tuple(tuple(m[off[i]:off[i + 1]].tolist()) for i in range(len(sizes)))] += 1
    assert set(seen) == set(states)
    obs = np.array([seen[s] for s in states])
    p = sps.chisquare(obs).pvalue
    assert p > 1e-3, (p, obs)


def test_relative_abundance_hand_example():
    real = np.array([10.0, 0.0, 6.0])
    null = np.array([[2.0, 0.0, 6.0], [4.0, 0.0, 6.0]])      # mean 3, 0, 6
    d = profiles.relative_abundance(real, null)
    assert np.allclose(d, [(10 - 3) / (10 + 3 + 4), 0.0, 0.0])
    sp = profiles.significance_profile(d)
    assert np.isclose(np.sum(sp ** 2), 1.0) and np.isclose(sp[0], 1.0)
    assert np.all(profiles.significance_profile(np.zeros(3)) == 0)


def test_quality_measures():
    a = np.array([0.1, -0.4, 0.3, 0.0, 0.9])
    assert np.isclose(profiles.quality(a, a)[0], 1.0)
    assert np.isclose(profiles.quality(-a, a)[0], -1.0)
    assert np.isclose(profiles.quality(2 * a + 3, a)[0], 1.0)
    b = a + np.array([0.0, 0.1, -0.2, 0.0, 0.05])
    rho, mx, mae = profiles.quality(b, a)
    assert np.isclose(mx, 0.2) and np.isclose(mae, 0.35 / 5)
    # Pearson's rho by its definition on a hand case: x = (1, 2, 3), y = (1, 3, 2)
    assert np.isclose(profiles.quality([1, 2, 3], [1, 3, 2])[0], 0.5)


def test_stratum_sizes_rule():
    """S = 60 split 1 : 3 : 2 gives 10 / 30 / 20; rounding and the k = 3 form."""
    assert profiles.stratum_sizes(60, 3, 2) == {2: 10, 3: 30, 4: 20}
    assert profiles.stratum_sizes(10, 1, 1) == {2: 3, 3: 3, 4: 4}          # 10/3 = 3.33 -> 3
    assert profiles.stratum_sizes(7, 0.5, 0.0) == {2: 5, 3: 2, 4: 0}       # 7/1.5 = 4.67 -> 5; 2.5 -> 3, capped at 2
    assert profiles.stratum_sizes(9, 2, 0, k=3) == {2: 3, 3: 6}


def test_stratum_search_consistency():
    """Algorithm 4 is consistent: with many draws in every cell the
    estimated profiles approach the exact one and every cell's mean
    correlation approaches 1; with few draws it is lower somewhere."""
    h = W.random_small(710, 30, 200, {2: 0.6, 3: 0.3, 4: 0.1})
    exact = core.count_exact(h, 4)
    null = np.array([core.count_exact(W.Hypergraph(h.n_nodes, *profiles.config_model(h, 3, 1, c)), 4)
                     for c in range(4)])
    prof = profiles.relative_abundance(exact, null)
    big = profiles.stratum_search(h, 4, 6000, [1.0, 3.0], [1.0, 2.0], 2, 5, null, prof)
    small = profiles.stratum_search(h, 4, 40, [1.0, 3.0], [1.0, 2.0], 2, 5, null, prof)
    assert big.shape == (2, 2) and np.all(big > 0.97) and np.all(big <= 1 + 1e-12)
    assert small.min() < big.min()
