"""Sampled counting (Algorithm 4) through the C ABI against the oracle.

Draws come from the same published counter-based generator on both sides
(Philox4x64-10); raw counts must match bit-exactly and the corrected
estimates exactly (both are formed in fp64 and rounded once to fp32)."""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import core, philox, stats

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def hm():
    import torch
    import paper_2209_10241_amd as hm
    assert torch.cuda.is_available()
    return hm


def _golden(name, k):
    with open(os.path.join(ROOT, "tests", "golden", "workload_counts.json")) as f:
        for c in json.load(f)["cases"]:
            if c["workload"] == name and c["k"] == k:
                return np.array(c["counts"], dtype=np.int64)
    raise KeyError(name)


def _graph(hm, h, bit_rows=True):
    hm.hm_set_option(hm.HM_OPT_BITSET_MAX_NODES, 8192 if bit_rows else 0)
    try:
        return hm.hm_graph_create(h.members, h.offsets, h.n_nodes)
    finally:
        hm.hm_set_option(hm.HM_OPT_BITSET_MAX_NODES, 8192)


def _oracle_sampled(nh, k, fraction, seed, allocation=0):
    n = {j: nh.count(j) for j in range(2, k + 1)}
    S = core.sample_sizes(n, k, fraction, allocation)
    samples = {j: philox.stratum_draws(seed, j, n[j], S[j]) for j in S}
    raw = core.sampled_raw(nh, k, samples)
    est = core.scale_estimate(raw, k, n, S).astype(np.float32)
    return raw, est, S, samples


@pytest.mark.parametrize("allocation", [0, 1])
def test_draws_match_oracle(hm, allocation):
    h = W.cfg1_facetoface_k4(0)
    nh = core.normalise(h)
    with _graph(hm, h) as g:
        got = hm.hm_sample_draw(g, 4, 0.05, 12345, allocation)
        S = hm.hm_sample_sizes(g, 4, 0.05, allocation)
    n = {j: nh.count(j) for j in (2, 3, 4)}
    assert S == core.sample_sizes(n, 4, 0.05, allocation)
    for j in (2, 3, 4):
        want = philox.stratum_draws(12345, j, n[j], S[j])
        assert np.array_equal(got[j].cpu().numpy().astype(np.int64), want)


@pytest.mark.parametrize("bit_rows", [True, False], ids=["bits", "hash"])
@pytest.mark.parametrize("seed", range(16))
def test_random_small_matches_oracle(hm, seed, bit_rows):
    mixes = [{2: 0.6, 3: 0.3, 4: 0.1}, {1: 0.05, 2: 0.45, 3: 0.3, 4: 0.15, 5: 0.05}, {2: 0.3, 3: 0.4, 4: 0.3}]
    h = W.random_small(4000 + seed, 15 + (seed * 11) % 50, 40 + (seed * 53) % 300, mixes[seed % 3],
                       allow_dups=bool(seed % 2))
    nh = core.normalise(h)
    with _graph(hm, h, bit_rows) as g:
        for k in (3, 4):
            for fraction in (0.3, 1.0):
                est, raw = hm.count_sampled(g, k, fraction, seed * 7 + 1, 0)
                want_raw, want_est, _, _ = _oracle_sampled(nh, k, fraction, seed * 7 + 1)
                assert np.array_equal(raw.cpu().numpy(), want_raw), (k, fraction)
                assert np.array_equal(est.cpu().numpy(), want_est), (k, fraction)


@pytest.mark.parametrize("bit_rows", [True, False], ids=["bits", "hash"])
def test_facetoface_order4_one_percent(hm, bit_rows):
    """The benchmark's workload at 1%: raw counts against the oracle's Algorithm 4."""
    h = W.cfg1_facetoface_k4(0)
    nh = core.normalise(h)
    want_raw, want_est, _, _ = _oracle_sampled(nh, 4, 0.01, 99)
    with _graph(hm, h, bit_rows) as g:
        est, raw = hm.count_sampled(g, 4, 0.01, 99, 0)
    assert np.array_equal(raw.cpu().numpy(), want_raw)
    assert np.array_equal(est.cpu().numpy(), want_est)


def test_facetoface_order3_paper_allocation(hm):
    h = W.cfg0_facetoface_k3(0)
    nh = core.normalise(h)
    want_raw, want_est, _, _ = _oracle_sampled(nh, 3, 0.1, 5, 1)
    with _graph(hm, h) as g:
        est, raw = hm.count_sampled(g, 3, 0.1, 5, 1)
    assert np.array_equal(raw.cpu().numpy(), want_raw)
    assert np.array_equal(est.cpu().numpy(), want_est)


@pytest.mark.parametrize("bit_rows", [True, False], ids=["bits", "hash"])
@pytest.mark.parametrize("name,k,maker", [("facetoface_N200_E2000", 3, W.cfg0_facetoface_k3),
                                          ("facetoface_N400_E30000", 4, W.cfg1_facetoface_k4),
                                          ("communication_scaled_0.004", 4,
                                           lambda seed: W.scaled_communication(0.004, seed))])
def test_census_reproduces_exact(hm, name, k, maker, bit_rows):
    """Every hyperedge sampled once: raw = countmax * exact and the estimate is the exact count."""
    h = maker(0)
    exact = _golden(name, k)
    with _graph(hm, h, bit_rows) as g:
        st = g.stats()
        samples = {j: np.arange(st[f"n{j}"]) for j in range(2, k + 1)}
        est, raw = hm.count_sampled_indices(g, k, samples)
        countmax = np.array([hm.hm_class_info(k, c)[2] for c in range(len(exact))])
    assert np.array_equal(raw.cpu().numpy(), exact * countmax)
    assert np.array_equal(est.cpu().numpy(), exact.astype(np.float32))


@pytest.mark.parametrize("bit_rows", [True, False], ids=["bits", "hash"])
def test_heavy_tailed_matches_oracle(hm, bit_rows):
    """Hubs, pairs inside many 3-node hyperedges: raw counts of 20% draws against the oracle."""
    h = W.scaled_communication(0.004, 0)
    nh = core.normalise(h)
    want_raw, want_est, _, _ = _oracle_sampled(nh, 4, 0.2, 31)
    with _graph(hm, h, bit_rows) as g:
        est, raw = hm.count_sampled(g, 4, 0.2, 31, 0)
    assert np.array_equal(raw.cpu().numpy(), want_raw)
    assert np.array_equal(est.cpu().numpy(), want_est)


def test_explicit_indices_match_oracle(hm):
    h = W.random_small(4100, 40, 300, {2: 0.5, 3: 0.3, 4: 0.2})
    nh = core.normalise(h)
    rng = np.random.default_rng(3)
    samples = {j: rng.integers(0, nh.count(j), size=25) for j in (2, 3, 4)}
    with _graph(hm, h) as g:
        _, raw = hm.count_sampled_indices(g, 4, samples)
    assert np.array_equal(raw.cpu().numpy(), core.sampled_raw(nh, 4, samples))


def test_bad_arguments(hm):
    h = W.random_small(4200, 20, 60, {2: 0.6, 3: 0.4})
    with _graph(hm, h) as g:
        n2 = g.stats()["n2"]
        with pytest.raises(hm.HMError):
            hm.count_sampled_indices(g, 4, {2: np.array([0, n2])})
        with pytest.raises(hm.HMError):
            hm.count_sampled(g, 4, 0.0, 1)
        with pytest.raises(hm.HMError):
            hm.count_sampled(g, 4, 1.5, 1)
        with pytest.raises(hm.HMError):
            hm.count_sampled(g, 5, 0.5, 1)


def test_unbiased_over_32_seeds(hm):
    """Mean over 32 seeds within 4 standard errors of the exact count for every class,
    and the mean relative error at 10% sampling stated numerically."""
    h = W.cfg1_facetoface_k4(0)
    exact = _golden("facetoface_N400_E30000", 4)
    runs = []
    with _graph(hm, h) as g:
        for seed in range(32):
            est, _ = hm.count_sampled(g, 4, 0.10, 1000 + seed, 0)
            runs.append(est.cpu().numpy().astype(np.float64))
    runs = np.array(runs)
    z = stats.bias_z(runs, exact)
    assert np.all(np.abs(z) < 4.5), np.abs(z).max()
    mre = stats.mean_relative_error(runs, exact)
    print(f"mean relative error over 32 seeds at 10%: {mre:.4f}")
    assert mre < 0.05


def test_variance_matches_closed_form(hm):
    """The spread of the sampler's estimate over 3000 seeds is that of S_j
    independent uniform draws with replacement from each stratum (Section 5):
    the per-class sample variance agrees with the oracle's |E_j|^2 v_m /
    (S_j countmax_m^2) within 5 standard errors of a variance estimate, and
    is 0 where that is.  Half of each stratum is drawn, so draws without
    replacement would show as a variance about half as large."""
    import torch
    h = W.random_small(700, 16, 70, {2: 0.5, 3: 0.3, 4: 0.2})
    nh = core.normalise(h)
    k, R = 4, 3000
    n_j = {j: nh.count(j) for j in range(2, k + 1)}
    S = core.sample_sizes(n_j, k, 0.5)
    var, kurt = core.estimator_moments(nh, k, S)
    n = hm.hm_num_classes(k)
    est = torch.empty((R, n), dtype=torch.float32, device="cuda")
    raw = torch.empty((R, n), dtype=torch.int64, device="cuda")
    with _graph(hm, h) as g:
        for seed in range(R):
            hm.count_sampled(g, k, 0.5, 7000 + seed, 0, est=est[seed], raw=raw[seed])
        runs = est.cpu().numpy().astype(np.float64)
    s2 = runs.var(axis=0, ddof=1)
    assert np.all(s2[var == 0] == 0)
    on = var > 0
    assert on.sum() >= 10
    rel = s2[on] / var[on] - 1.0
    tol = 5.0 * np.sqrt(2.0 / (R - 1) + np.maximum(kurt[on], 0.0) / R)
    print(f"variance over {R} seeds: max |rel| / tol {np.abs(rel / tol).max():.2f}")
    assert np.all(np.abs(rel) < tol), (rel[np.abs(rel) >= tol], tol[np.abs(rel) >= tol])


@pytest.fixture
def queued(hm):
    """No bit rows and the smallest work chunks: the long walks of every sample
    go through the work queue and its drain launch."""
    hm.hm_set_option(hm.HM_OPT_SAMPLE_CHUNK_SCALE, 1024)
    try:
        yield
    finally:
        hm.hm_set_option(hm.HM_OPT_SAMPLE_CHUNK_SCALE, 1)


@pytest.mark.parametrize("seed", range(8))
def test_work_queue_matches_oracle(hm, queued, seed):
    mixes = [{2: 0.6, 3: 0.3, 4: 0.1}, {2: 0.3, 3: 0.4, 4: 0.3}]
    h = W.random_small(4500 + seed, 20 + (seed * 13) % 40, 120 + (seed * 71) % 300, mixes[seed % 2])
    nh = core.normalise(h)
    with _graph(hm, h, False) as g:
        for fraction in (0.3, 1.0):
            est, raw = hm.count_sampled(g, 4, fraction, seed * 3 + 2, 0)
            want_raw, want_est, _, _ = _oracle_sampled(nh, 4, fraction, seed * 3 + 2)
            assert np.array_equal(raw.cpu().numpy(), want_raw), fraction
            assert np.array_equal(est.cpu().numpy(), want_est), fraction


def test_work_queue_heavy_tailed(hm, queued):
    h = W.scaled_communication(0.004, 0)
    nh = core.normalise(h)
    want_raw, want_est, _, _ = _oracle_sampled(nh, 4, 0.2, 31)
    with _graph(hm, h, False) as g:
        est, raw = hm.count_sampled(g, 4, 0.2, 31, 0)
        # twice in a row: the queue counters are left clear
        est2, raw2 = hm.count_sampled(g, 4, 0.2, 31, 0)
    assert np.array_equal(raw.cpu().numpy(), want_raw)
    assert np.array_equal(raw2.cpu().numpy(), want_raw)
    assert np.array_equal(est2.cpu().numpy(), want_est)


def test_work_queue_census(hm, queued):
    h = W.scaled_communication(0.004, 0)
    exact = _golden("communication_scaled_0.004", 4)
    with _graph(hm, h, False) as g:
        st = g.stats()
        samples = {j: np.arange(st[f"n{j}"]) for j in range(2, 5)}
        est, raw = hm.count_sampled_indices(g, 4, samples)
        countmax = np.array([hm.hm_class_info(4, c)[2] for c in range(len(exact))])
    assert np.array_equal(raw.cpu().numpy(), exact * countmax)
    assert np.array_equal(est.cpu().numpy(), exact.astype(np.float32))


def test_chunk_scale_option_bounds(hm):
    for bad in (0, 1025):
        with pytest.raises(hm.HMError):
            hm.hm_set_option(hm.HM_OPT_SAMPLE_CHUNK_SCALE, bad)
    hm.hm_set_option(hm.HM_OPT_SAMPLE_CHUNK_SCALE, 1)


@pytest.fixture
def hub_rows(hm):
    """Dense adjacency rows for every node with at least 2 pairwise neighbours."""
    hm.hm_set_option(hm.HM_OPT_HUB_MIN_DEGREE, 2)
    try:
        yield
    finally:
        hm.hm_set_option(hm.HM_OPT_HUB_MIN_DEGREE, 256)


def test_hub_rows_heavy_tailed(hm, hub_rows, queued):
    h = W.scaled_communication(0.004, 0)
    nh = core.normalise(h)
    want_raw, want_est, _, _ = _oracle_sampled(nh, 4, 0.2, 31)
    with _graph(hm, h, False) as g:
        est, raw = hm.count_sampled(g, 4, 0.2, 31, 0)
    assert np.array_equal(raw.cpu().numpy(), want_raw)
    assert np.array_equal(est.cpu().numpy(), want_est)


def test_hub_rows_census(hm, hub_rows):
    h = W.scaled_communication(0.004, 0)
    exact = _golden("communication_scaled_0.004", 4)
    with _graph(hm, h, False) as g:
        st = g.stats()
        samples = {j: np.arange(st[f"n{j}"]) for j in range(2, 5)}
        est, raw = hm.count_sampled_indices(g, 4, samples)
        countmax = np.array([hm.hm_class_info(4, c)[2] for c in range(len(exact))])
    assert np.array_equal(raw.cpu().numpy(), exact * countmax)


def test_queue_buffers_outlive_the_call(hm, queued):
    """count_sampled returns before its kernels finish; the work queue it
    allocated is released in stream order, so a graph built and counted on
    another stream right after cannot be handed those blocks while the
    drain still reads them: the first call's raw counts stay exact."""
    import torch
    h = W.scaled_communication(0.004, 0)
    nh = core.normalise(h)
    want_raw, want_est, _, _ = _oracle_sampled(nh, 4, 0.2, 31)
    hb = W.random_small(4600, 60, 900, {2: 0.5, 3: 0.3, 4: 0.2})
    want_b = core.count_exact(hb, 4)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    with _graph(hm, h, False) as ga:
        with torch.cuda.stream(s1):
            hm.count_sampled(ga, 4, 0.2, 31, 0)      # builds the graph's cached indices
            s1.synchronize()
            est, raw = hm.count_sampled(ga, 4, 0.2, 31, 0)
        with torch.cuda.stream(s2):
            for _ in range(3):
                with _graph(hm, hb, False) as gb:
                    hm.count_sampled(gb, 4, 0.5, 7, 0)
                    got_b = hm.count_exact(gb, 4)
        torch.cuda.synchronize()
    assert np.array_equal(raw.cpu().numpy(), want_raw)
    assert np.array_equal(est.cpu().numpy(), want_est)
    assert np.array_equal(got_b.cpu().numpy(), want_b)
