"""Configuration-model null (Chodrow's pairwise reshuffles) and motif
profiles through the C ABI against the oracle.  Both sides draw from the
same published counter-based generator, so the copies must agree bit for
bit, and so must their exact counts; the profiles and their accuracy
measures agree to fp64 rounding."""
import numpy as np
import pytest

import workloads as W
from oracle import core, nulls, profiles

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hm():
    import torch
    import paper_2209_10241_amd as hm
    assert torch.cuda.is_available()
    return hm


@pytest.mark.parametrize("seed", range(6))
def test_config_copies_match_oracle(hm, seed):
    """Small hypergraphs, sizes up to 7, repeated input hyperedges, odd and
    even hyperedge counts: every copy identical to the oracle's chain."""
    h = W.random_small(9000 + seed, 20 + seed * 9, 61 + seed * 37, {1: 0.05, 2: 0.45, 3: 0.3, 4: 0.1, 7: 0.1},
                       allow_dups=bool(seed % 2))
    with hm.hm_graph_create(h.members, h.offsets, h.n_nodes) as g:
        for copy, sweeps in ((0, 1), (3, 5), (17, 2)):
            m, o = hm.hm_null_export_model(g, hm.HM_NULL_CONFIG, sweeps, 31 + seed, copy)
            wm, wo = profiles.config_model(h, sweeps, 31 + seed, copy)
            assert np.array_equal(o, wo)
            assert np.array_equal(m, wm), (seed, copy, sweeps)
            nulls.check_null_invariants(h, m, o)


def test_config_copies_heavy_tailed(hm):
    """Hyperedges of up to 50 nodes (communication recipe at 0.4%)."""
    h = W.scaled_communication(0.004, 0)
    with hm.hm_graph_create(h.members, h.offsets, h.n_nodes) as g:
        m, o = hm.hm_null_export_model(g, hm.HM_NULL_CONFIG, 3, 5, 1)
    wm, wo = profiles.config_model(h, 3, 5, 1)
    assert np.array_equal(o, wo) and np.array_equal(m, wm)
    nulls.check_null_invariants(h, m, o)


@pytest.mark.parametrize("k", [3, 4])
def test_config_counts_z_and_profile(hm, k):
    """count_nulls_model: the real counts, every copy's exact counts and the
    z-scores against the oracle; then the profile and its accuracy measures."""
    import torch
    h = W.random_small(9100 + k, 45, 300, {2: 0.5, 3: 0.3, 4: 0.15, 6: 0.05})
    R, sweeps, seed = 10, 4, 77
    with hm.hm_graph_create(h.members, h.offsets, h.n_nodes) as g:
        real, nl, z = hm.count_nulls_model(g, k, R, hm.HM_NULL_CONFIG, sweeps, seed)
        # a second call replays the captured pipeline with another seed
        real2, nl2, _ = hm.count_nulls_model(g, k, R, hm.HM_NULL_CONFIG, sweeps, seed + 1)
    want_real = core.count_exact(h, k)
    assert np.array_equal(real.cpu().numpy(), want_real)
    want = []
    for c in range(R):
        m, o = profiles.config_model(h, sweeps, seed, c)
        want.append(core.count_exact(W.Hypergraph(h.n_nodes, m, o), k))
    want = np.array(want)
    assert np.array_equal(nl.cpu().numpy(), want)
    m, o = profiles.config_model(h, sweeps, seed + 1, R - 1)
    assert np.array_equal(nl2.cpu().numpy()[R - 1], core.count_exact(W.Hypergraph(h.n_nodes, m, o), k))
    zz, want_z = z.cpu().numpy(), nulls.zscores(want_real, want)
    finite = np.isfinite(want_z)
    assert np.array_equal(np.isfinite(zz), finite)
    assert np.array_equal(np.sign(zz[~finite]), np.sign(want_z[~finite]))
    np.testing.assert_allclose(zz[finite], want_z[finite].astype(np.float32), rtol=2e-6, atol=1e-6)
    delta, sp = hm.hm_motif_profile(real.double(), nl.double())
    wd = profiles.relative_abundance(want_real, want)
    np.testing.assert_allclose(delta.cpu().numpy(), wd, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(sp.cpu().numpy(), profiles.significance_profile(wd), rtol=1e-12, atol=1e-15)
    # the profile from the second batch's nulls against the first
    d2, _ = hm.hm_motif_profile(real.double(), nl2.double())
    got = hm.hm_profile_quality(d2, delta)
    want_q = profiles.quality(profiles.relative_abundance(want_real, nl2.cpu().numpy()), wd)
    np.testing.assert_allclose(got, want_q, rtol=1e-10, atol=1e-13)
    del torch


def test_profile_measures_edge_cases(hm):
    """Constant profiles give rho = 0; a single class; eps = 0."""
    a = np.array([0.5, 0.5, 0.5])
    assert hm.hm_profile_quality(a, a)[0] == 0.0
    rho, mx, mae = hm.hm_profile_quality(np.array([0.2]), np.array([-0.1]))
    assert rho == 0.0 and abs(mx - 0.3) < 1e-15 and abs(mae - 0.3) < 1e-15
    real = np.array([3.0, 0.0, 1.0])
    nl = np.array([[1.0, 0.0, 1.0], [3.0, 0.0, 1.0]])
    d, s = hm.hm_motif_profile(real, nl, eps=0.0)
    np.testing.assert_allclose(d.cpu().numpy()[[0, 2]], [0.2, 0.0])
    assert np.isnan(d.cpu().numpy()[1])   # 0 / 0 with eps = 0, as the definition gives


def test_bad_model_arguments(hm):
    h = W.random_small(9200, 20, 50, {2: 0.6, 3: 0.4})
    with hm.hm_graph_create(h.members, h.offsets, h.n_nodes) as g:
        with pytest.raises(hm.HMError):
            hm.count_nulls_model(g, 4, 4, 7, 3, 1)
        with pytest.raises(hm.HMError):
            hm.count_nulls_model(g, 4, 4, hm.HM_NULL_CONFIG, 0, 1)
        with pytest.raises(hm.HMError):
            hm.hm_null_export_model(g, hm.HM_NULL_CONFIG, 5000, 1, 0)


def test_sampled_sizes_match_oracle(hm):
    """count_sampled_sizes: explicit draws per stratum, raw counts bit-exact."""
    from oracle import philox
    h = W.random_small(9300, 40, 300, {2: 0.5, 3: 0.3, 4: 0.2})
    nh = core.normalise(h)
    n = {j: nh.count(j) for j in (2, 3, 4)}
    for sizes in ({2: 7, 3: 0, 4: 13}, {2: 1, 3: 50, 4: 2}, {2: 0, 3: 0, 4: 5}):
        with hm.hm_graph_create(h.members, h.offsets, h.n_nodes) as g:
            est, raw = hm.count_sampled_sizes(g, 4, sizes, 123)
        samples = {j: philox.stratum_draws(123, j, n[j], sizes[j]) for j in sizes}
        want_raw = core.sampled_raw(nh, 4, samples)
        assert np.array_equal(raw.cpu().numpy(), want_raw), sizes
        want_est = core.scale_estimate(want_raw, 4, n, sizes).astype(np.float32)
        assert np.array_equal(est.cpu().numpy(), want_est), sizes


def test_stratum_search_matches_oracle(hm):
    """The appendix's grid search over S_3 / S_2 and S_4 / S_2: the mean
    correlation of every cell equals the oracle's (the same draws, the same
    float32 estimates; fp64 profiles and correlations)."""
    h = W.random_small(9400, 35, 260, {2: 0.55, 3: 0.3, 4: 0.15})
    k, R, S, reps, seed = 4, 6, 90, 3, 40
    with hm.hm_graph_create(h.members, h.offsets, h.n_nodes) as g:
        real, nl, _ = hm.count_nulls_model(g, k, R, hm.HM_NULL_CONFIG, 3, 2)
        delta, _ = hm.hm_motif_profile(real.double(), nl.double())
        r3, r4 = [0.5, 1.0, 3.0], [1.0, 2.0]
        got = hm.hm_stratum_search(g, k, S, r3, r4, reps, seed, nl.double(), delta)
        with pytest.raises(hm.HMError):
            hm.hm_stratum_search(g, k, 0, r3, r4, reps, seed, nl.double(), delta)
        with pytest.raises(hm.HMError):
            hm.hm_stratum_search(g, k, S, [-1.0], r4, reps, seed, nl.double(), delta)
    nulls_np = nl.cpu().numpy()
    prof = profiles.relative_abundance(real.cpu().numpy(), nulls_np)
    want = profiles.stratum_search(h, k, S, r3, r4, reps, seed, nulls_np, prof)
    np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-12)
    # order 3: one column
    with hm.hm_graph_create(h.members, h.offsets, h.n_nodes) as g:
        real3, nl3, _ = hm.count_nulls_model(g, 3, R, hm.HM_NULL_CONFIG, 3, 2)
        d3, _ = hm.hm_motif_profile(real3.double(), nl3.double())
        got3 = hm.hm_stratum_search(g, 3, 40, [0.5, 2.0], None, 2, seed, nl3.double(), d3)
    n3 = nl3.cpu().numpy()
    want3 = profiles.stratum_search(h, 3, 40, [0.5, 2.0], None, 2, seed, n3,
                                    profiles.relative_abundance(real3.cpu().numpy(), n3))
    np.testing.assert_allclose(got3, want3, rtol=1e-11, atol=1e-12)
