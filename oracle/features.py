"""Reference of the learned proposal's per-hyperedge features (oracle; test
infrastructure only).

The learned proposal is an addition to the paper's Algorithm 4 (Section 5):
it needs, for every hyperedge e of size j = 2..k, a vector of 16 local
features from which a small network predicts e's motif contribution.  The
features are plain functions of the normalised hypergraph (Section 3: a set
of hyperedges; sizes above k lie in no k-node set, but every hyperedge of
size 2..4 is counted in the node degrees below, whatever k).  Per member v
of e (s = |e| members):

    d2(v)  pairwise degree: 2-node hyperedges holding v (neighbours in G2)
    d3(v)  3-node hyperedges holding v
    d4(v)  4-node hyperedges holding v

and the columns, in float64:

     0..2  one-hot of s = 2, 3, 4
        3  log(1 + mean d2)         4  log(1 + max d2)     5  log(1 + min d2)
        6  log(1 + mean d3)         7  log(1 + max d3)
        8  log(1 + mean d4)         9  log(1 + max d4)
       10  fraction of the C(s, 2) member pairs that are 2-node hyperedges
       11  log(1 + sum C(d2, 2)) / 2       (pairwise wedges at the members)
       12  log(1 + sum d2 d3) / 2
       13  log(1 + sum over member pairs of d2(a) d2(b)) / 2
       14  log(1 + sum C(d2, 3)) / 3       (pairwise 3-stars at the members)
       15  1

Columns 3..14 are then standardised within each stratum: (x - mean) / sd
with the population standard deviation, and 0 for a column whose variance is
below 1e-12 (constant within the stratum).  Rows follow stratum order: the
size-2 hyperedges, then size 3, then (k = 4) size 4, each in first-occurrence
order.
"""
from __future__ import annotations

import math

import numpy as np

from .core import Normalised, normalise

N_FEATURES = 16
STANDARDISED = range(3, 15)


def node_degrees(nh: Normalised):
    """(d2, d3, d4): per node, the number of 2-, 3- and 4-node hyperedges holding it."""
    out = []
    for j in (2, 3, 4):
        d = np.zeros(nh.n_nodes, dtype=np.int64)
        e = nh.edges(j)
        if len(e):
            np.add.at(d, e.reshape(-1), 1)
        out.append(d)
    return tuple(out)


def raw_features(h, k: int) -> np.ndarray:
    """Unstandardised features, one row per hyperedge of size 2..k, float64."""
    nh = h if isinstance(h, Normalised) else normalise(h)
    d2, d3, d4 = node_degrees(nh)
    pairs = {tuple(p) for p in nh.edges(2).tolist()}
    rows = []
    for s in range(2, k + 1):
        for e in nh.edges(s).tolist():
            a2 = [int(d2[v]) for v in e]
            a3 = [int(d3[v]) for v in e]
            a4 = [int(d4[v]) for v in e]
            member_pairs = [(e[x], e[y]) for x in range(s) for y in range(x + 1, s)]
            joined = sum((p in pairs) for p in member_pairs)
            pd = sum(d2[a] * d2[b] for a, b in member_pairs)
            f = [float(s == 2), float(s == 3), float(s == 4),
                 math.log1p(sum(a2) / s), math.log1p(max(a2)), math.log1p(min(a2)),
                 math.log1p(sum(a3) / s), math.log1p(max(a3)),
                 math.log1p(sum(a4) / s), math.log1p(max(a4)),
                 joined / len(member_pairs),
                 0.5 * math.log1p(sum(math.comb(x, 2) for x in a2)),
                 0.5 * math.log1p(sum(x * y for x, y in zip(a2, a3))),
                 0.5 * math.log1p(float(pd)),
                 math.log1p(sum(math.comb(x, 3) for x in a2)) / 3.0,
                 1.0]
            rows.append(f)
    return np.array(rows, dtype=np.float64).reshape(-1, N_FEATURES)


def strata_bounds(h, k: int) -> list:
    nh = h if isinstance(h, Normalised) else normalise(h)
    b = [0]
    for s in range(2, k + 1):
        b.append(b[-1] + nh.count(s))
    return b


def standardise(X: np.ndarray, bounds: list):
    """Standardise columns 3..14 per stratum; returns (Z, mean, inv_sd) with
    mean and inv_sd of shape (n_strata, 16)."""
    Z = X.copy()
    ns = len(bounds) - 1
    mean = np.zeros((ns, N_FEATURES))
    inv_sd = np.zeros((ns, N_FEATURES))
    for s in range(ns):
        blk = X[bounds[s]:bounds[s + 1]]
        if len(blk) == 0:
            continue
        for f in STANDARDISED:
            m = blk[:, f].mean()
            var = ((blk[:, f] - m) ** 2).mean()
            mean[s, f] = m
            inv_sd[s, f] = 1.0 / math.sqrt(var) if var > 1e-12 else 0.0
            Z[bounds[s]:bounds[s + 1], f] = (blk[:, f] - m) * inv_sd[s, f]
    return Z, mean, inv_sd


def features(h, k: int) -> np.ndarray:
    """Standardised features (float64), the rows of every hyperedge of size 2..k."""
    X = raw_features(h, k)
    return standardise(X, strata_bounds(h, k))[0]
