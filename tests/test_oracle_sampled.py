"""Pins of the oracle's sampled estimator (Algorithm 4, Section 5), its RNG
and the null model."""
from itertools import combinations

import numpy as np
import pytest

import workloads as W
from oracle import brute, core, nulls, philox, stats
from oracle.classes import table


# ---------------------------------------------------------------- Philox RNG
@pytest.mark.parametrize("key", [(0, 0), (5, 7), (2**64 - 1, 12345), (0xDEADBEEF, (1 << 32) | 4)])
@pytest.mark.parametrize("ctr", [0, 1, 41, 2**40])
def test_philox_matches_numpy_bit_generator(key, ctr):
    # numpy's generator advances its counter before each block, so its first
    # block for state counter c is the Philox function at counter c + 1
    g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array([ctr, 0, 0, 0], dtype=np.uint64))
    want = g.random_raw(4).tolist()
    assert philox.philox4x64_10([ctr + 1, 0, 0, 0], key) == want
    vec = philox.philox_vec(np.array([ctr + 1], np.uint64), 0, 0, 0, *key)
    assert [int(v[0]) for v in vec] == want


def test_philox_full_counter():
    g = np.random.Philox(key=np.array([9, 3], dtype=np.uint64), counter=np.array([2**64 - 1, 6, 7, 8], dtype=np.uint64))
    want = g.random_raw(4).tolist()   # counter carries into the second word
    assert philox.philox4x64_10([0, 7, 7, 8], [9, 3]) == want
    vec = philox.philox_vec(np.array([0], np.uint64), 7, 7, 8, 9, 3)
    assert [int(v[0]) for v in vec] == want


def test_bounded_draws():
    w = np.array([0, 2**63, 2**64 - 1], dtype=np.uint64)
    assert philox.bounded(w, 10).tolist() == [0, 5, 9]
    idx = philox.stratum_draws(7, 2, 1000, 200_000)
    assert idx.min() >= 0 and idx.max() < 1000
    counts = np.bincount(idx, minlength=1000)
    chi2 = ((counts - 200.0) ** 2 / 200.0).sum()
    assert chi2 < 1000 + 6 * np.sqrt(2 * 1000)


# ---------------------------------------------------------------- Algorithm 4
def _strata(nh, k):
    return {j: nh.count(j) for j in range(2, k + 1)}


@pytest.mark.parametrize("seed", range(8))
def test_census_reproduces_exact_counts(seed):
    """Sampling every hyperedge once: each occurrence is found once per
    hyperedge of maximal size in it, so raw = countmax * exact and the
    corrected estimate equals the exact count."""
    h = W.random_small(500 + seed, 14, 45, {1: 0.05, 2: 0.5, 3: 0.3, 4: 0.15, 5: 0.05})
    nh = core.normalise(h)
    for k in (3, 4):
        t = table(k)
        exact = core.count_exact(nh, k)
        samples = {j: np.arange(nh.count(j)) for j in range(2, k + 1)}
        raw = core.sampled_raw(nh, k, samples)
        assert np.array_equal(raw, exact * np.array(t.countmax))
        est = core.scale_estimate(raw, k, _strata(nh, k), {j: nh.count(j) for j in range(2, k + 1)})
        assert np.array_equal(est, exact.astype(np.float64))


def _raw_by_definition(nh, k, samples):
    """Per sampled hyperedge e: every k-set V containing e, connected, whose
    largest inside hyperedge has |e| nodes, by brute force over all k-sets."""
    t = table(k)
    present = {tuple(r) for j, arr in nh.by_size.items() if j <= k for r in arr.tolist()}
    nodes = sorted({v for e in present for v in e})
    raw = np.zeros(t.n_classes, dtype=np.int64)
    for j, idx in samples.items():
        for i in idx:
            e = set(nh.edges(j)[i].tolist())
            for V in combinations(nodes, k):
                if not e <= set(V):
                    continue
                inside = [x for x in present if set(x) <= set(V)]
                if max(len(x) for x in inside) != j:
                    continue
                p = t.pattern_of(lambda m, V=V: tuple(V[b] for b in range(k) if (m >> b) & 1) in present)
                if t.class_of[p] >= 0:
                    raw[t.class_of[p]] += 1
    return raw


@pytest.mark.parametrize("seed", range(6))
def test_sampled_raw_matches_definition(seed):
    h = W.random_small(600 + seed, 11, 30, {2: 0.5, 3: 0.3, 4: 0.2})
    nh = core.normalise(h)
    rng = np.random.default_rng(seed)
    for k in (3, 4):
        samples = {j: rng.integers(0, nh.count(j), size=5) for j in range(2, k + 1) if nh.count(j)}
        assert np.array_equal(core.sampled_raw(nh, k, samples), _raw_by_definition(nh, k, samples))


def test_estimator_is_unbiased():
    """Mean of the corrected estimate over many seeds is within 4 standard
    errors of the exact count for every class (the unbiasedness of Section 5)."""
    h = W.random_small(700, 16, 70, {2: 0.5, 3: 0.3, 4: 0.2})
    nh = core.normalise(h)
    k = 4
    exact = core.count_exact(nh, k)
    n_j = _strata(nh, k)
    S = {j: max(1, n_j[j] // 4) for j in n_j}
    runs = []
    for seed in range(300):
        samples = {j: philox.stratum_draws(seed, j, n_j[j], S[j]) for j in n_j}
        raw = core.sampled_raw(nh, k, samples)
        runs.append(core.scale_estimate(raw, k, n_j, S))
    runs = np.array(runs)
    z = stats.bias_z(runs, exact)
    assert np.all(np.abs(z) < 4.5), z[np.abs(z) >= 4.5]
    assert stats.mean_relative_error(runs, exact) < 0.5


def test_estimator_variance_matches_closed_form():
    """The spread of the corrected estimate over seeds is that of S_j
    independent uniform draws with replacement (Section 5): for every class
    the sample variance over 3000 seeds agrees with |E_j|^2 v_m / (S_j
    countmax_m^2) within 5 standard errors of a variance estimate
    (sqrt(2 / (R - 1) + kurtosis / R) relative), and is 0 where v_m is.  With
    half of each stratum drawn, draws without replacement would shrink the
    variance by about half (by (|E_j| - S_j) / (|E_j| - 1)), several times
    the tolerance; a biased index or a wrong S_j in the correction would
    change it too."""
    h = W.random_small(700, 16, 70, {2: 0.5, 3: 0.3, 4: 0.2})
    nh = core.normalise(h)
    k = 4
    n_j = _strata(nh, k)
    S = {j: max(1, n_j[j] // 2) for j in n_j}
    var, kurt = core.estimator_moments(nh, k, S)
    R = 3000
    runs = []
    for seed in range(R):
        samples = {j: philox.stratum_draws(seed, j, n_j[j], S[j]) for j in n_j}
        runs.append(core.scale_estimate(core.sampled_raw(nh, k, samples), k, n_j, S))
    s2 = np.array(runs).var(axis=0, ddof=1)
    assert np.all(s2[var == 0] == 0)
    on = var > 0
    assert on.sum() >= 10
    rel = s2[on] / var[on] - 1.0
    tol = 5.0 * np.sqrt(2.0 / (R - 1) + np.maximum(kurt[on], 0.0) / R)
    assert np.all(np.abs(rel) < tol), (rel[np.abs(rel) >= tol], tol[np.abs(rel) >= tol])


def test_unsampled_stratum_reports_zero():
    h = W.from_lists([[0, 1, 2, 3], [0, 1], [1, 2], [2, 3]], 4)
    raw = core.sampled_raw(h, 4, {2: [0]})
    est = core.scale_estimate(raw, 4, {2: 3, 3: 0, 4: 1}, {2: 1, 3: 0, 4: 0})
    assert est.sum() == 0   # the only occurrence has maxcard 4


# ---------------------------------------------------------------- null model
def test_stub_matching_invariants_and_determinism():
    h = W.random_small(800, 60, 300, {2: 0.5, 3: 0.3, 4: 0.15, 5: 0.05})
    m1, o1 = nulls.stub_matching(h, seed=3, copy=0)
    nulls.check_null_invariants(h, m1, o1)
    m2, o2 = nulls.stub_matching(h, seed=3, copy=0)
    assert np.array_equal(m1, m2) and np.array_equal(o1, o2)
    m3, _ = nulls.stub_matching(h, seed=3, copy=1)
    assert not np.array_equal(m1, m3)
    m4, _ = nulls.stub_matching(h, seed=4, copy=0)
    assert not np.array_equal(m1, m4)


def test_stub_matching_checker_rejects_changes():
    h = W.random_small(801, 20, 40, {2: 0.6, 3: 0.4})
    m, o = nulls.stub_matching(h, seed=0, copy=0)
    bad = m.copy()
    bad[0] = (bad[0] + 1) % 20          # one stub moved to another node: degrees change
    with pytest.raises(AssertionError):
        nulls.check_null_invariants(h, bad, o)


def test_zscores_closed_form():
    real = np.array([10, 5, 7, 3])
    nulls_ = np.array([[8, 5, 7, 3], [12, 5, 7, 3], [10, 5, 7, 3]])
    # class 0: mean 10, sd 2 -> z 0; classes 1-3: sd 0 and x == mean -> 0
    assert nulls.zscores(real, nulls_).tolist() == [0.0, 0.0, 0.0, 0.0]
    real = np.array([14, 6, 6, 3])
    z = nulls.zscores(real, nulls_)
    assert z[0] == 2.0 and z[1] == np.inf and z[2] == -np.inf and z[3] == 0.0


def test_mre_definition():
    exact = np.array([100.0, 0.0, 50.0])
    runs = np.array([[110.0, 0.0, 40.0], [90.0, 3.0, 50.0]])
    assert stats.mean_relative_error(runs, exact) == pytest.approx(((10 + 10) / 150 + (10 + 3) / 150) / 2)


def test_sample_sizes_rule():
    n = {2: 12258, 3: 11313, 4: 4549}
    assert core.sample_sizes(n, 4, 0.01) == {2: 123, 3: 114, 4: 46}
    s = 28120 // 100 + 1                           # ceil(0.01 * 28120) = 282
    assert core.sample_sizes(n, 4, 0.01, core.ALLOC_PAPER) == {2: s // 6, 3: s // 2, 4: s - s // 6 - s // 2}
    assert core.sample_sizes({2: 10, 3: 0}, 3, 0.5) == {2: 5, 3: 0}
    assert core.sample_sizes(n, 3, 1.0, core.ALLOC_PAPER) == {2: 12258, 3: 11313}
