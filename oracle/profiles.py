"""Motif profiles against a configuration-model null, and the accuracy
measures of sampled profiles (oracle; test infrastructure only).

Section 6.3 scores sampled estimates on motif *profiles*: observed
frequencies compared with those of hypergraphs drawn from a configuration
model that keeps every node's degree and every hyperedge's size, ten draws,
and then Pearson's correlation, the largest and the mean absolute error
between the estimated and the exact profile.  The profile's formula is not
printed in the paper (it follows the cited higher-order motif work, which
takes the relative abundance of Milo et al., Science 2004):

    delta_m = (x_m - mu_m) / (x_m + mu_m + eps),   eps = 4,

x_m the count in the observed hypergraph, mu_m its mean over the null
draws; the significance profile is delta / ||delta||_2.  This reading is
parity unpinned against the paper: its values are checked here only against
their definition (hand-worked examples and properties).

The stratum-budget search of the appendix (Fig. 6) splits S draws as
S_2 : S_3 : S_4 = 1 : r3 : r4 and, over a grid of (r3, r4), keeps the mean
Pearson correlation between estimated and exact profiles; it is composed of
the pinned parts (Algorithm 4's estimator, the profile, rho) and the size
rule, which is pinned by hand-worked values.

The configuration model is sampled by Markov chain Monte Carlo with the
pairwise reshuffle move of Chodrow (J. Complex Networks 2020): for two
hyperedges e and f, the nodes they share stay in both, and the nodes in
exactly one of them are dealt out again uniformly at random, keeping both
sizes.  The move is symmetric, so the chain keeps the uniform distribution
over hypergraphs with the given degree and size sequences (in which no
hyperedge repeats a node).  One round reshuffles disjoint pairs at once:

  round r   key_i = word 0 of Philox(counter (i, r, 0, 0)) for hyperedge i;
            order the hyperedges by (key, i) into pi; pair t is
            (pi[2t], pi[2t + 1]); an odd last hyperedge waits
  pair t    e, f their current members (ascending); I = e & f;
            D = (e - f ascending) followed by (f - e ascending); a = |e - f|;
            for q = 0 .. a - 1: w = word (q mod 4) of
            Philox(counter (t, r, 1 + q div 4, 0)), j = q + hi64(w (|D| - q)),
            swap D[q] and D[j]; then e = sort(I + D[:a]), f = sort(I + D[a:])

with the key (seed, (5 << 32) | copy), over the unique hyperedges of size
>= 2 in first-occurrence order.  A copy may hold a node set twice; counting
collapses such repeats (Section 3).
"""
from __future__ import annotations

import math

import numpy as np

from . import philox
from .core import Normalised, normalise, sampled_raw, scale_estimate

DOMAIN_CONFIG = 5
EPS = 4.0


def config_model(h, sweeps: int, seed: int, copy: int):
    """One draw: (members uint32, offsets uint64), hyperedges in the input's order."""
    nh = h if isinstance(h, Normalised) else normalise(h)
    edges = [list(e) for e in nh.order]
    E = len(edges)
    k0, k1 = philox.stream_key(seed, DOMAIN_CONFIG, copy)
    idx = np.arange(E, dtype=np.uint64)
    for r in range(sweeps):
        keys = philox.philox_vec(idx, np.uint64(r), 0, 0, k0, k1)[0]
        pi = np.lexsort((np.arange(E), keys))
        for t in range(E // 2):
            ie, jf = int(pi[2 * t]), int(pi[2 * t + 1])
            e, f = edges[ie], edges[jf]
            fs, es = set(f), set(e)
            inter = [v for v in e if v in fs]
            D = [v for v in e if v not in fs] + [v for v in f if v not in es]
            a = len(e) - len(inter)
            words = []
            for q in range(a):
                if q % 4 == 0:
                    words = philox.philox4x64_10((t, r, 1 + q // 4, 0), (k0, k1))
                w = words[q % 4]
                j = q + ((w * (len(D) - q)) >> 64)
                D[q], D[j] = D[j], D[q]
            edges[ie] = sorted(inter + D[:a])
            edges[jf] = sorted(inter + D[a:])
    sizes = np.array([len(e) for e in edges], dtype=np.int64)
    offsets = np.zeros(E + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum(sizes)
    members = np.array([v for e in edges for v in e], dtype=np.uint32)
    return members, offsets


def relative_abundance(real, nulls, eps: float = EPS) -> np.ndarray:
    """delta_m = (x_m - mu_m) / (x_m + mu_m + eps), mu the mean over the null rows, float64."""
    x = np.asarray(real, dtype=np.float64)
    mu = np.asarray(nulls, dtype=np.float64).mean(axis=0)
    return (x - mu) / (x + mu + eps)


def significance_profile(delta) -> np.ndarray:
    """delta / ||delta||_2 (all zeros when delta is)."""
    d = np.asarray(delta, dtype=np.float64)
    n = math.sqrt(float(np.sum(d * d)))
    return d / n if n > 0 else np.zeros_like(d)


def quality(est_profile, exact_profile):
    """(rho, MaxAE, MAE): Pearson's correlation, largest and mean absolute error (Section 6.3)."""
    a = np.asarray(est_profile, dtype=np.float64)
    b = np.asarray(exact_profile, dtype=np.float64)
    da, db = a - a.mean(), b - b.mean()
    den = math.sqrt(float(np.sum(da * da)) * float(np.sum(db * db)))
    rho = float(np.sum(da * db)) / den if den > 0 else 0.0
    err = np.abs(a - b)
    return rho, float(err.max()), float(err.mean())


def _round_half_up(x: float) -> int:
    return int(math.floor(x + 0.5))


def stratum_sizes(S: int, r3: float, r4: float, k: int = 4) -> dict:
    """S_2 : S_3 : S_4 = 1 : r3 : r4 with S_2 + S_3 + S_4 = S (appendix, Fig. 6):
    S_2 = round(S / (1 + r3 + r4)), S_3 = min(S - S_2, round(r3 S_2)), S_4 the rest
    (k = 3: S_3 = S - S_2), halves rounded up."""
    s2 = _round_half_up(S / (1.0 + r3 + (r4 if k == 4 else 0.0)))
    if k == 3:
        return {2: s2, 3: S - s2}
    s3 = min(S - s2, _round_half_up(r3 * s2))
    return {2: s2, 3: s3, 4: S - s2 - s3}


def stratum_search(h, k: int, S: int, ratio3, ratio4, reps: int, seed: int, nulls, exact_profile,
                   eps: float = EPS) -> np.ndarray:
    """The appendix's exhaustive search: for every (r3, r4) cell the mean over
    `reps` estimates (seeds seed, seed + 1, ...) of Pearson's rho between the
    estimated profile and exact_profile.  Estimates follow Algorithm 4 with the
    cell's stratum sizes (rounded to float32 as the library returns them)."""
    nh = h if isinstance(h, Normalised) else normalise(h)
    n = {j: nh.count(j) for j in range(2, k + 1)}
    r4s = list(ratio4) if k == 4 else [0.0]
    out = np.zeros((len(ratio3), len(r4s)))
    for i, r3 in enumerate(ratio3):
        for j, r4 in enumerate(r4s):
            sizes = stratum_sizes(S, r3, r4, k)
            sizes = {s: (v if n[s] > 0 else 0) for s, v in sizes.items()}
            acc = 0.0
            for r in range(reps):
                samples = {s: philox.stratum_draws(seed + r, s, n[s], sizes[s]) for s in sizes}
                raw = sampled_raw(nh, k, samples)
                est = scale_estimate(raw, k, n, sizes).astype(np.float32).astype(np.float64)
                acc += quality(relative_abundance(est, nulls, eps), exact_profile)[0]
            out[i, j] = acc / reps
    return out

