"""Pins of the learned proposal's reference: finite differences for the
gradient, the bfloat16 rounding rule, the rounding-error bound (it covers a
computation rounded at the kernels' points and catches planted mistakes),
and the Hansen-Hurwitz estimator reducing to the correction of Algorithm 4
under uniform probabilities."""
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


def _bf16(a):
    return mlp.bf16(np.asarray(a, dtype=np.float32))


def _rounded_network(p, x, t, plant=None):
    """A computation with the kernels' precision, in this test only: operands of
    the hidden-layer products rounded to bfloat16 (nearest even), everything
    else float32.  ``plant`` puts a plausible mistake into it."""
    W1, b1, W2, b2, w3, b3 = [np.asarray(a, dtype=np.float32) for a in mlp.unpack(p)]
    x = np.asarray(x, np.float32)
    t = np.asarray(t, np.float32)
    B = len(x)
    if plant == "transposed_W2":
        W2 = np.ascontiguousarray(W2.T)
    xb = _bf16(x)
    z1 = xb @ _bf16(W1).T + b1
    h1b = _bf16(np.maximum(z1, 0))
    z2 = h1b @ _bf16(W2).T + (0 if plant == "dropped_b2" else b2)
    h2 = np.maximum(z2, 0)
    out = h2 @ w3 + b3
    dout = np.float32(2) * (out - t) * np.float32(1 / B)
    if plant == "sign":
        dout = -dout
    g = np.zeros(mlp.N_PARAMS, np.float32)
    g[mlp.OFF_W3:mlp.OFF_B3] = dout @ h2
    g[mlp.OFF_B3] = dout.sum()
    dz2 = np.outer(dout, w3) * (z2 > 0)
    g[mlp.OFF_B2:mlp.OFF_W3] = dz2.sum(0)
    dz2b = _bf16(dz2)
    g[mlp.OFF_W2:mlp.OFF_B2] = (dz2b.T @ h1b).reshape(-1)
    dh1 = dz2b @ _bf16(W2)
    dz1 = dh1 * (z1 > 0) if plant != "no_relu_mask" else dh1
    g[mlp.OFF_B1:mlp.OFF_W2] = dz1.sum(0)
    g[mlp.OFF_W1:mlp.OFF_B1] = (_bf16(dz1).T @ xb).reshape(-1)
    return out, g, float(np.mean((out.astype(np.float64) - t) ** 2))


def _within(r, out, g, loss):
    return (np.all(np.abs(out - r["out"]) <= r["out_bound"])
            and np.linalg.norm(out - r["out"]) <= 2 * r["out_dev_norm"]
            and np.all(np.abs(g - r["grad"]) <= r["grad_bound"])
            and np.linalg.norm(g - r["grad"]) <= 2 * r["grad_dev_norm"]
            and abs(loss - r["loss"]) <= r["loss_bound"])


@pytest.mark.parametrize("seed", range(8))
def test_bound_covers_a_rounded_computation(seed):
    """The per-element bound (and twice the largest deviation norm of its
    runs) covers a computation rounded at the kernels' points."""
    rng = np.random.default_rng(300 + seed)
    B = [1, 16, 50, 257][seed % 4]
    p = rng.normal(0, 0.3, mlp.N_PARAMS)
    x = rng.normal(size=(B, 16))
    t = rng.normal(size=B)
    r = mlp.error_bounds(p, x, t, seed=seed)
    assert _within(r, *_rounded_network(p, x, t))


def test_bound_is_informative():
    """The bound is small beside the values where rounding is mild, and each
    planted mistake breaks it."""
    rng = np.random.default_rng(11)
    p = rng.normal(0, 0.3, mlp.N_PARAMS)
    x = rng.normal(size=(64, 16))
    t = rng.normal(size=64)
    r = mlp.error_bounds(p, x, t)
    assert np.median(r["out_bound"] / np.abs(r["out"])) < 0.1
    g, b = r["grad"], r["grad_bound"]
    for lo, hi in ((mlp.OFF_W2, mlp.OFF_B2), (mlp.OFF_B2, mlp.OFF_W3), (mlp.OFF_W3, mlp.OFF_B3)):
        nz = g[lo:hi] != 0
        assert np.median(b[lo:hi][nz] / np.abs(g[lo:hi][nz])) < 0.3
    for plant in ("transposed_W2", "dropped_b2", "sign", "no_relu_mask"):
        assert not _within(r, *_rounded_network(p, x, t, plant)), plant


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
