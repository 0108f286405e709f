"""Learned proposal through the C ABI against the oracle: MLP forward and
gradient (bf16 rounding points mirrored), per-hyperedge contributions, the
Hansen-Hurwitz estimate, training, and the estimator built on the trained
proposal (unbiased; its error compared with uniform Algorithm 4)."""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import core, mlp, stats
from oracle.classes import table

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


def _params(seed, scale=0.3):
    return np.random.default_rng(seed).normal(0, scale, mlp.N_PARAMS).astype(np.float32)


@pytest.mark.parametrize("n", [1, 16, 37, 300])
def test_mlp_forward_matches_oracle(hm, n):
    import torch
    rng = np.random.default_rng(n)
    x = rng.normal(size=(n, 16)).astype(np.float32)
    p = _params(n)
    got = hm.hm_mlp_forward(torch.from_numpy(p), torch.from_numpy(x)).cpu().numpy()
    want, _ = mlp.forward(p, x, mirror=True)
    np.testing.assert_allclose(got, want, rtol=2e-4, atol=2e-4)


@pytest.mark.parametrize("n", [16, 50, 257])
def test_mlp_gradient_matches_oracle(hm, n):
    import torch
    rng = np.random.default_rng(10 + n)
    x = rng.normal(size=(n, 16)).astype(np.float32)
    t = rng.normal(size=n).astype(np.float32)
    p = _params(10 + n)
    g, loss = hm.hm_mlp_grad(torch.from_numpy(p), torch.from_numpy(x), torch.from_numpy(t))
    g = g.cpu().numpy().astype(np.float64)
    want_loss, want = mlp.loss_and_grad(p, x, t, mirror=True)
    assert abs(loss - want_loss) <= 1e-4 * max(1.0, abs(want_loss))
    assert np.linalg.norm(g - want) <= 2e-3 * np.linalg.norm(want)
    close = np.isclose(g, want, rtol=5e-3, atol=5e-5 * np.abs(want).max())
    assert close.mean() > 0.995


@pytest.mark.parametrize("path", ["bits", "hash", "queued"])
def test_contributions_match_oracle(hm, path):
    """Per-hyperedge contributions (one sample row each); without bit rows, and
    with every long walk through the work queue."""
    h = W.random_small(6000, 30, 180, {2: 0.5, 3: 0.3, 4: 0.2})
    nh = core.normalise(h)
    t = table(4)
    hm.hm_set_option(hm.HM_OPT_BITSET_MAX_NODES, 8192 if path == "bits" else 0)
    hm.hm_set_option(hm.HM_OPT_SAMPLE_CHUNK_SCALE, 1024 if path == "queued" else 1)
    try:
        with hm.hm_graph_create(h.members, h.offsets, h.n_nodes) as g:
            y = hm.hm_contrib(g, 4).cpu().numpy()
    finally:
        hm.hm_set_option(hm.HM_OPT_BITSET_MAX_NODES, 8192)
        hm.hm_set_option(hm.HM_OPT_SAMPLE_CHUNK_SCALE, 1)
    want = []
    for j in (2, 3, 4):
        for i in range(nh.count(j)):
            raw = core.sampled_raw(nh, 4, {j: [i]})
            want.append(sum(raw[m] / t.countmax[m] for m in range(t.n_classes)))
    np.testing.assert_allclose(y, np.array(want), rtol=1e-12)


def test_contributions_sum_to_exact_totals(hm):
    """Census identity on the benchmark workload: per stratum j, the
    contributions sum to the exact total of the classes with maxcard j."""
    h = W.cfg1_facetoface_k4(0)
    exact = _golden("facetoface_N400_E30000", 4)
    t = table(4)
    with hm.hm_graph_create(h.members, h.offsets, h.n_nodes) as g:
        st = g.stats()
        y = hm.hm_contrib(g, 4).cpu().numpy()
    bounds = np.cumsum([0, st["n2"], st["n3"], st["n4"]])
    for j in (2, 3, 4):
        want = sum(int(exact[m]) for m in range(t.n_classes) if t.maxcard[m] == j)
        assert abs(y[bounds[j - 2]:bounds[j - 1]].sum() - want) <= 1e-9 * want


def test_weighted_estimate_matches_oracle(hm):
    h = W.random_small(6100, 40, 260, {2: 0.5, 3: 0.3, 4: 0.2})
    nh = core.normalise(h)
    t = table(4)
    rng = np.random.default_rng(4)
    samples = {j: rng.integers(0, nh.count(j), size=20) for j in (2, 3, 4)}
    probs = {j: rng.random(20) * 0.05 + 0.001 for j in (2, 3, 4)}
    with hm.hm_graph_create(h.members, h.offsets, h.n_nodes) as g:
        est, raw = hm.count_sampled_weighted_indices(g, 4, samples, probs)
    raw_ps, strata, ps = [], [], []
    for j in (2, 3, 4):
        for i, p in zip(samples[j], probs[j]):
            raw_ps.append(core.sampled_raw(nh, 4, {j: [int(i)]}))
            strata.append(j)
            ps.append(p)
    want = mlp.hansen_hurwitz(np.array(raw_ps), np.array(strata), np.array(ps), {2: 20, 3: 20, 4: 20},
                              t.maxcard, t.countmax)
    np.testing.assert_allclose(est.cpu().numpy(), want.astype(np.float32), rtol=1e-6)
    assert np.array_equal(raw.cpu().numpy(), core.sampled_raw(nh, 4, samples))


def test_weighted_uniform_is_algorithm4(hm):
    h = W.cfg1_facetoface_k4(0)
    with hm.hm_graph_create(h.members, h.offsets, h.n_nodes) as g:
        st = g.stats()
        rng = np.random.default_rng(5)
        samples = {j: rng.integers(0, st[f"n{j}"], size=60) for j in (2, 3, 4)}
        probs = {j: np.full(60, 1.0 / st[f"n{j}"]) for j in (2, 3, 4)}
        est_w, raw_w = hm.count_sampled_weighted_indices(g, 4, samples, probs)
        est_u, raw_u = hm.count_sampled_indices(g, 4, samples)
    assert np.array_equal(raw_w.cpu().numpy(), raw_u.cpu().numpy())
    np.testing.assert_allclose(est_w.cpu().numpy(), est_u.cpu().numpy(), rtol=1e-6)


def test_features_layout(hm):
    h = W.cfg1_facetoface_k4(0)
    with hm.hm_graph_create(h.members, h.offsets, h.n_nodes) as g:
        st = g.stats()
        x = hm.hm_features(g, 4).cpu().numpy()
    n2, n3, n4 = st["n2"], st["n3"], st["n4"]
    assert x.shape == (n2 + n3 + n4, 16)
    assert np.all(x[:n2, 0] == 1) and np.all(x[n2:n2 + n3, 1] == 1) and np.all(x[n2 + n3:, 2] == 1)
    assert np.all(x[:, 15] == 1) and np.all(np.isfinite(x))
    # standardised columns have mean ~0 within each stratum
    assert np.abs(x[:n2, 3:15].mean(axis=0)).max() < 1e-3


def test_training_reduces_loss(hm):
    h = W.scaled_communication(0.004, seed=0)
    with hm.hm_graph_create(h.members, h.offsets, h.n_nodes) as g:
        with hm.hm_model_train(g, 4, epochs=40, batch=512, lr=3e-3, seed=1) as m:
            loss = m.loss()
    assert len(loss) == 40
    assert loss[-1] < 0.7 * loss[0], loss


def test_learned_estimator_unbiased_and_compared(hm):
    """Train on a 5% hyperedge subsample, sample the full hypergraph with the
    proposal over 32 seeds: unbiased, and its error beside uniform sampling
    at the same fraction (printed)."""
    h = W.scaled_communication(0.004, seed=0)
    exact = _golden("communication_scaled_0.004", 4).astype(np.float64)
    h5 = W.subsample_edges(h, 0.05, seed=3)
    f = 0.05
    with hm.hm_graph_create(h.members, h.offsets, h.n_nodes) as g, \
            hm.hm_graph_create(h5.members, h5.offsets, h5.n_nodes) as g5:
        with hm.hm_model_train(g5, 4, epochs=60, batch=256, lr=3e-3, seed=2) as m:
            learned = np.array([hm.count_sampled_learned(g, m, 4, f, 500 + s)[0].cpu().numpy()
                                for s in range(32)], dtype=np.float64)
        uniform = np.array([hm.count_sampled(g, 4, f, 500 + s)[0].cpu().numpy() for s in range(32)],
                           dtype=np.float64)
    z = stats.bias_z(learned, exact)
    assert np.all(np.abs(z) < 4.5), np.abs(z).max()
    mre_l = stats.mean_relative_error(learned, exact)
    mre_u = stats.mean_relative_error(uniform, exact)
    print(f"mean relative error at {f:.0%}: learned {mre_l:.4f}, uniform {mre_u:.4f}")
    assert mre_l < 0.25
