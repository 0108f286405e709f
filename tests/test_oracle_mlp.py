"""Pins of the learned proposal's reference: finite differences for the
gradient, the bfloat16 rounding rule, and the Hansen-Hurwitz estimator
reducing to the correction of Algorithm 4 under uniform probabilities."""
import numpy as np
import pytest

import workloads as W
from oracle import core, mlp
from oracle.classes import table


def _params(seed):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.3, mlp.N_PARAMS)
    return p


def test_parameter_count():
    assert mlp.N_PARAMS == 16 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 5313


@pytest.mark.parametrize("seed", range(3))
def test_gradient_matches_finite_differences(seed):
    rng = np.random.default_rng(100 + seed)
    x = rng.normal(size=(24, 16))
    t = rng.normal(size=24)
    p = _params(seed)
    _, g = mlp.loss_and_grad(p, x, t)
    idx = rng.choice(mlp.N_PARAMS, size=40, replace=False).tolist() + [mlp.OFF_B3, mlp.OFF_W3, mlp.OFF_B1]
    fd = mlp.finite_difference(p, x, t, idx)
    np.testing.assert_allclose(g[idx], fd, rtol=1e-5, atol=1e-7)


def test_bf16_rounding_rule():
    v = np.array([1.0, 1.0 + 2**-8, 1.0 + 2**-7, 1.0 + 3 * 2**-8, -2.5, 0.0], dtype=np.float32)
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties go to the even mantissa (1.0);
    # 1 + 3*2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: ties to even (1 + 2^-6)
    want = np.array([1.0, 1.0, 1.0 + 2**-7, 1.0 + 2**-6, -2.5, 0.0], dtype=np.float32)
    assert np.array_equal(mlp.bf16(v), want)
    x = np.random.default_rng(0).normal(size=1000).astype(np.float32)
    r = mlp.bf16(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0**-8)
    assert np.all((r.view(np.uint32) & 0xFFFF) == 0)


def test_mirrored_gradient_is_close_to_exact():
    rng = np.random.default_rng(7)
    x = rng.normal(size=(64, 16))
    t = rng.normal(size=64)
    p = _params(7)
    _, g = mlp.loss_and_grad(p, x, t)
    _, gm = mlp.loss_and_grad(p, x, t, mirror=True)
    assert np.linalg.norm(gm - g) < 0.05 * np.linalg.norm(g)


def test_hansen_hurwitz_uniform_is_algorithm4():
    h = W.random_small(900, 18, 80, {2: 0.5, 3: 0.3, 4: 0.2})
    nh = core.normalise(h)
    k = 4
    t = table(k)
    rng = np.random.default_rng(1)
    n = {j: nh.count(j) for j in (2, 3, 4)}
    S = {j: 7 for j in n}
    draws = {j: rng.integers(0, n[j], size=S[j]) for j in n}
    raw_ps, strata, probs = [], [], []
    for j in (2, 3, 4):
        for i in draws[j]:
            raw_ps.append(core.sampled_raw(nh, k, {j: [int(i)]}))
            strata.append(j)
            probs.append(1.0 / n[j])
    est = mlp.hansen_hurwitz(np.array(raw_ps), np.array(strata), np.array(probs), S, t.maxcard, t.countmax)
    raw = core.sampled_raw(nh, k, draws)
    np.testing.assert_allclose(est, core.scale_estimate(raw, k, n, S), rtol=1e-12)


def test_hansen_hurwitz_is_unbiased_for_any_positive_proposal():
    """Exact expectation: sum over e of p_e * raw_e / (S p_e) * S = census."""
    h = W.random_small(901, 16, 70, {2: 0.5, 3: 0.3, 4: 0.2})
    nh = core.normalise(h)
    k = 4
    t = table(k)
    exact = core.count_exact(nh, k)
    rng = np.random.default_rng(2)
    expect = np.zeros(t.n_classes)
    for j in (2, 3, 4):
        nj = nh.count(j)
        p = rng.random(nj) + 0.1
        p /= p.sum()
        for i in range(nj):
            raw = core.sampled_raw(nh, k, {j: [i]})
            # one draw (S_j = 1) of e has probability p_i and contributes raw / p_i
            expect += p[i] * mlp.hansen_hurwitz(raw[None, :], np.array([j]), np.array([p[i]]), {j: 1},
                                                t.maxcard, t.countmax)
    np.testing.assert_allclose(expect, exact, rtol=1e-9)
