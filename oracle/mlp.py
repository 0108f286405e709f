"""Reference of the learned sampling proposal (oracle; test infrastructure only).

The proposal scores each hyperedge with a small MLP (16 features -> 64 -> 64
-> 1, ReLU) and draws hyperedges of stratum j with probability p_e; the
estimate stays unbiased with the Hansen-Hurwitz weights 1 / (S_j p_e), which
reduce to the correction factor of Algorithm 4 (Section 5) when p_e is
uniform.  This module gives:

  forward and backward in float64 (pinned by finite differences);
  a per-element bound on how far a computation may land from those exact
  values when the operands of its two hidden-layer products (forward: the
  inputs, W1, the first hidden activation, W2; backward: the two
  back-propagated pre-activation gradients and the operands they meet) are
  rounded to bfloat16 and every sum and product is formed in float32, in any
  summation order;
  the Hansen-Hurwitz estimate from per-sample raw class counts.

Parameter layout (flat, 5313 values): W1[64][16], b1[64], W2[64][64], b2[64],
w3[64], b3.  Loss: mean squared error over the batch.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H = 16, 64
OFF_W1 = 0
OFF_B1 = OFF_W1 + N_H * N_IN
OFF_W2 = OFF_B1 + N_H
OFF_B2 = OFF_W2 + N_H * N_H
OFF_W3 = OFF_B2 + N_H
OFF_B3 = OFF_W3 + N_H
N_PARAMS = OFF_B3 + 1


def bf16(x) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even), returned as float32."""
    u = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def unpack(p: np.ndarray):
    p = np.asarray(p, dtype=np.float64)
    return (p[OFF_W1:OFF_B1].reshape(N_H, N_IN), p[OFF_B1:OFF_W2], p[OFF_W2:OFF_B2].reshape(N_H, N_H),
            p[OFF_B2:OFF_W3], p[OFF_W3:OFF_B3], p[OFF_B3])


def forward(params, x):
    """Network output per row of x, float64."""
    W1, b1, W2, b2, w3, b3 = unpack(params)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    out = h2 @ w3 + b3
    return out, (x, z1, h1, z2, h2)


def loss_and_grad(params, x, t):
    """Mean squared error and its gradient with respect to the flat parameters."""
    W1, b1, W2, b2, w3, b3 = unpack(params)
    t = np.asarray(t, dtype=np.float64)
    B = len(t)
    out, (x, z1, h1, z2, h2) = forward(params, x)
    loss = float(np.mean((out - t) ** 2))
    dout = 2.0 * (out - t) / B
    g = np.zeros(N_PARAMS)
    g[OFF_W3:OFF_B3] = dout @ h2
    g[OFF_B3] = dout.sum()
    dz2 = np.outer(dout, w3) * (z2 > 0)
    g[OFF_B2:OFF_W3] = dz2.sum(axis=0)
    g[OFF_W2:OFF_B2] = (dz2.T @ h1).reshape(-1)
    dh1 = dz2 @ W2
    dz1 = dh1 * (z1 > 0)
    g[OFF_B1:OFF_W2] = dz1.sum(axis=0)
    g[OFF_W1:OFF_B1] = (dz1.T @ x).reshape(-1)
    return loss, g


# ------------------------------------------------------------ error bounds
# The kernels round to bfloat16 (8 significant bits, round to nearest: a
# relative error of at most U_BF16) the operands of their matrix products:
# forward the inputs x, W1, the first hidden activation h1 and W2; backward
# the two back-propagated pre-activation gradients dz2 and dz1, which meet h1,
# W2 and x.  Everything else is float32.
#
# The bound on |computed - exact| per output element has three parts:
#  1. bf16 rounding.  A worst-case sum of |error| over every rounded operand
#     grows by about n / sqrt(n) per layer of width n and is larger than the
#     values themselves after two layers, so it would test nothing.  Rounding
#     errors are instead modelled as independent, uniform on [-U_BF16, U_BF16]
#     relative to each operand (the probabilistic model of Higham and Mary,
#     SIAM J. Sci. Comput. 2019): the network is evaluated in float64 with
#     such perturbations R times, and the bound takes K_SIGMA standard
#     deviations of the deviation from the exact value.
#  2. ReLU switches.  A pre-activation within K_SWITCH standard deviations
#     of zero may take the other branch, which changes the back-propagated
#     gradient by its whole value: that value is added, through the absolute
#     values of what it meets, to every gradient it reaches.  (Past 4.5
#     deviations a switch has probability below 1e-5 under the model; the
#     runs of part 1 already switch the closer ones now and then.)
#  3. float32 arithmetic: Higham's gamma_n times the sum of absolute terms of
#     each product, n the length of the longest sum, doubled for the error
#     carried in from the layers before.
U_BF16 = 2.0 ** -8
U_F32 = 2.0 ** -23     # also covers truncating accumulation
K_SIGMA = 6.0
K_SWITCH = 4.5
N_RUNS = 64


def _gamma(n):
    nu = n * U_F32
    return nu / (1.0 - nu)


def _evaluate(params, x, t, rel):
    """Forward and backward with every rounded operand v replaced by v (1 + rel[name]);
    rel arrays carry a leading axis of runs.  Returns a dict of arrays over runs."""
    W1, b1, W2, b2, w3, b3 = unpack(params)
    x = np.asarray(x, dtype=np.float64)
    B = len(x)
    xb = x * (1 + rel["x"])
    W1b = W1 * (1 + rel["W1"])
    z1 = np.einsum("rbi,rji->rbj", xb, W1b) + b1
    h1 = np.maximum(z1, 0.0)
    h1b = h1 * (1 + rel["h1"])
    W2b = W2 * (1 + rel["W2"])
    z2 = np.einsum("rbk,rjk->rbj", h1b, W2b) + b2
    h2 = np.maximum(z2, 0.0)
    out = h2 @ w3 + b3
    res = dict(out=out, z1=z1, z2=z2)
    if t is None:
        return res
    t = np.asarray(t, dtype=np.float64)
    dout = 2.0 * (out - t) / B
    res["loss"] = np.mean((out - t) ** 2, axis=1)
    g = np.zeros((out.shape[0], N_PARAMS))
    g[:, OFF_W3:OFF_B3] = np.einsum("rb,rbj->rj", dout, h2)
    g[:, OFF_B3] = dout.sum(axis=1)
    dz2 = dout[:, :, None] * w3[None, None, :] * (z2 > 0)
    g[:, OFF_B2:OFF_W3] = dz2.sum(axis=1)
    dz2b = dz2 * (1 + rel["dz2"])
    g[:, OFF_W2:OFF_B2] = np.einsum("rbj,rbk->rjk", dz2b, h1b).reshape(len(out), -1)
    dh1 = np.einsum("rbj,rjk->rbk", dz2b, W2b)
    dz1 = dh1 * (z1 > 0)
    g[:, OFF_B1:OFF_W2] = dz1.sum(axis=1)
    dz1b = dz1 * (1 + rel["dz1"])
    g[:, OFF_W1:OFF_B1] = np.einsum("rbj,rbi->rji", dz1b, xb).reshape(len(out), -1)
    res.update(grad=g, dh1=dh1)
    return res


def _perturbations(B, runs, rng):
    shapes = dict(x=(B, N_IN), W1=(N_H, N_IN), h1=(B, N_H), W2=(N_H, N_H), dz2=(B, N_H), dz1=(B, N_H))
    if runs == 0:
        return {k: np.zeros((1,) + s) for k, s in shapes.items()}
    return {k: rng.uniform(-U_BF16, U_BF16, size=(runs,) + s) for k, s in shapes.items()}


def error_bounds(params, x, t=None, seed=0):
    """Exact forward (and, with targets t, the mean squared error and its
    gradient) with per-element bounds on the deviation of a computation
    rounded as described above.  Returns a dict: out, out_bound and, with t,
    loss, loss_bound, grad, grad_bound; also out_dev_norm and grad_dev_norm,
    the largest Euclidean norm of the whole deviation vector over the runs
    of part 1 (a check on the vector as a whole, which a wrong index or a
    dropped term exceeds many times over)."""
    W1, b1, W2, b2, w3, b3 = unpack(params)
    x = np.asarray(x, dtype=np.float64)
    B = len(x)
    tt = None if t is None else np.asarray(t, dtype=np.float64)
    ex = _evaluate(params, x, tt, _perturbations(B, 0, None))
    mc = _evaluate(params, x, tt, _perturbations(B, N_RUNS, np.random.default_rng(seed)))
    sd = {k: np.sqrt(np.mean((mc[k] - ex[k]) ** 2, axis=0)) for k in mc}
    e = {k: v[0] for k, v in ex.items()}
    z1, z2 = e["z1"], e["z2"]
    h1 = np.maximum(z1, 0.0)
    h2 = np.maximum(z2, 0.0)
    ax = np.abs(x)
    # float32: forward sums of 17, 65 and 66 terms
    f_z1 = _gamma(17) * (ax @ np.abs(W1).T + np.abs(b1))
    f_z2 = _gamma(65) * (h1 @ np.abs(W2).T + np.abs(b2)) + f_z1 @ np.abs(W2).T
    f_out = _gamma(66) * (h2 @ np.abs(w3) + abs(b3)) + f_z2 @ np.abs(w3)
    res = dict(out=e["out"], out_bound=K_SIGMA * sd["out"] + 2 * f_out,
               out_dev_norm=float(np.max(np.linalg.norm(mc["out"] - ex["out"], axis=1))))
    if tt is None:
        return res
    out = e["out"]
    dout = 2.0 * (out - tt) / B
    adout = np.abs(dout) + K_SIGMA * 2.0 / B * sd["out"]
    g = e["grad"]
    gb = K_SIGMA * sd["grad"]
    # ReLU switches: a pre-activation within K_SWITCH deviations of zero may
    # take the other branch on the device; h1 / h2 then move by at most |z|
    # plus its deviation, dz2 / dz1 by their whole value
    amb2 = np.abs(z2) <= K_SWITCH * sd["z2"] + f_z2
    amb1 = np.abs(z1) <= K_SWITCH * sd["z1"] + f_z1
    dh2 = np.where(amb2, np.abs(z2) + K_SIGMA * sd["z2"], 0.0)
    dh1v = np.where(amb1, np.abs(z1) + K_SIGMA * sd["z1"], 0.0)
    ddz2 = np.where(amb2, adout[:, None] * np.abs(w3)[None, :], 0.0)
    ddh1 = ddz2 @ np.abs(W2)
    adh1 = np.abs(e["dh1"]) + K_SIGMA * sd["dh1"]
    ddz1 = np.where(amb1, adh1 + ddh1, ddh1 * (z1 > 0))
    adz2 = np.abs(dout)[:, None] * np.abs(w3)[None, :] * (z2 > 0)
    sw = np.zeros(N_PARAMS)
    sw[OFF_W3:OFF_B3] = adout @ dh2
    sw[OFF_B2:OFF_W3] = ddz2.sum(axis=0)
    sw[OFF_W2:OFF_B2] = (ddz2.T @ (h1 + dh1v) + adz2.T @ dh1v).reshape(-1)
    sw[OFF_B1:OFF_W2] = ddz1.sum(axis=0)
    sw[OFF_W1:OFF_B1] = (ddz1.T @ ax).reshape(-1)
    adz1 = np.abs(e["dh1"]) * (z1 > 0)
    # float32 of the backward sums (B rows, 64 hidden units)
    n = B + 70
    f = np.zeros(N_PARAMS)
    f[OFF_B3] = np.sum(np.abs(dout))
    f[OFF_W3:OFF_B3] = np.abs(dout) @ h2
    f[OFF_B2:OFF_W3] = adz2.sum(axis=0)
    f[OFF_W2:OFF_B2] = (adz2.T @ h1).reshape(-1)
    f[OFF_B1:OFF_W2] = adz1.sum(axis=0)
    f[OFF_W1:OFF_B1] = (adz1.T @ ax).reshape(-1)
    f *= 4 * _gamma(n)
    res.update(loss=float(e["loss"]), loss_bound=float(K_SIGMA * sd["loss"] + 4 * _gamma(n) * np.mean((np.abs(out - tt) + 1) ** 2)),
               grad=g, grad_bound=gb + sw + f,
               grad_dev_norm=float(np.max(np.linalg.norm(mc["grad"] - ex["grad"], axis=1))))
    return res


def finite_difference(params, x, t, idx, h=1e-6):
    p = np.asarray(params, dtype=np.float64).copy()
    out = []
    for i in idx:
        p[i] += h
        lp, _ = loss_and_grad(p, x, t)
        p[i] -= 2 * h
        lm, _ = loss_and_grad(p, x, t)
        p[i] += h
        out.append((lp - lm) / (2 * h))
    return np.array(out)


def hansen_hurwitz(raw_per_sample: np.ndarray, stratum_of_sample: np.ndarray, p_of_sample: np.ndarray,
                   S_by_size: dict, maxcard, countmax) -> np.ndarray:
    """est_m = sum over draws s of stratum maxcard(m) of raw[s, m] / (S_j p_s countmax_m), float64."""
    raw = np.asarray(raw_per_sample, dtype=np.float64)
    n_classes = raw.shape[1] if raw.ndim == 2 else len(maxcard)
    est = np.zeros(n_classes)
    for m in range(n_classes):
        j = maxcard[m]
        sel = stratum_of_sample == j
        if S_by_size.get(j, 0) == 0 or not sel.any():
            continue
        est[m] = float(np.sum(raw[sel, m] / (float(S_by_size[j]) * p_of_sample[sel]))) / countmax[m]
    return est
