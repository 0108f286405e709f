"""Reference of the learned sampling proposal (oracle; test infrastructure only).

The proposal scores each hyperedge with a small MLP (16 features -> 64 -> 64
-> 1, ReLU) and draws hyperedges of stratum j with probability p_e; the
estimate stays unbiased with the Hansen-Hurwitz weights 1 / (S_j p_e), which
reduce to the correction factor of Algorithm 4 (Section 5) when p_e is
uniform.  This module gives:

  forward/backward in float64, exact (pinned by finite differences) or with
  the rounding points of the device kernels mirrored: inputs, weights of the
  two hidden layers, the first hidden activation and the two backpropagated
  pre-activation gradients are rounded to bfloat16 (round to nearest even);
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


def _r(x, mirror):
    return bf16(np.asarray(x, dtype=np.float32)).astype(np.float64) if mirror else np.asarray(x, dtype=np.float64)


def forward(params, x, mirror=False):
    W1, b1, W2, b2, w3, b3 = unpack(params)
    xb = _r(x, mirror)
    W1b, W2b = _r(W1, mirror), _r(W2, mirror)
    z1 = xb @ W1b.T + b1
    h1 = np.maximum(z1, 0.0)
    h1b = _r(h1, mirror)
    z2 = h1b @ W2b.T + b2
    h2 = np.maximum(z2, 0.0)
    out = h2 @ w3 + b3
    return out, (xb, W1b, W2b, z1, h1b, z2, h2)


def loss_and_grad(params, x, t, mirror=False):
    """Mean squared error and its gradient with respect to the flat parameters."""
    W1, b1, W2, b2, w3, b3 = unpack(params)
    t = np.asarray(t, dtype=np.float64)
    B = len(t)
    out, (xb, W1b, W2b, z1, h1b, z2, h2) = forward(params, x, mirror)
    loss = float(np.mean((out - t) ** 2))
    dout = 2.0 * (out - t) / B
    g = np.zeros(N_PARAMS)
    g[OFF_W3:OFF_B3] = dout @ h2
    g[OFF_B3] = dout.sum()
    dz2 = np.outer(dout, w3) * (z2 > 0)
    g[OFF_B2:OFF_W3] = dz2.sum(axis=0)
    dz2b = _r(dz2, mirror)
    g[OFF_W2:OFF_B2] = (dz2b.T @ h1b).reshape(-1)
    dh1 = dz2b @ W2b
    dz1 = dh1 * (z1 > 0)
    g[OFF_B1:OFF_W2] = dz1.sum(axis=0)
    dz1b = _r(dz1, mirror)
    g[OFF_W1:OFF_B1] = (dz1b.T @ xb).reshape(-1)
    return loss, g


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
