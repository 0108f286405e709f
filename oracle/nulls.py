"""Null hypergraphs by stub matching, and motif over/under-expression
(oracle; test infrastructure only).

Section 1 and Section 3 describe the pipeline: count motifs in the observed
hypergraph, count them again in randomised hypergraphs drawn from a null
model that keeps node degrees and hyperedge sizes, and score each motif's
over- or under-expression; Section 6.3 draws such randomisations from a
configuration model.  The null model implemented here is stub matching that
keeps every node's degree and every hyperedge's size exactly:

  stubs   every unique hyperedge of size >= 2, in first-occurrence order,
          contributes its members (ascending); node v appears deg(v) times
  round 0 the stubs are put in the order of their random keys
          (Philox word 0 of counter (t, 0, 0, 0)) and cut into hyperedges of the
          original sizes, in the original order
  repair  while some hyperedge repeats a node (round r = 1, 2, ...): take the
          offending hyperedges B (ascending), give the q-th of them a partner
          hyperedge hi64(word0(counter (q, r, 1, 0)) * E), pool the current
          members of B and the partners (ascending hyperedge order, stored
          member order), reorder the pool by the keys word0(counter (t, r, 0, 0))
          and deal it back in the same hyperedge order
  give up after 64 repair rounds

Keys use the null-model stream of copy c: key = (seed, (2 << 32) | c).  Ties
between equal keys keep position order.  A copy may hold the same node set
twice; the set semantics of Section 3 collapse such repeats when it is
counted.
"""
from __future__ import annotations

import numpy as np

from . import philox
from .core import Normalised, normalise

MAX_REPAIR_ROUNDS = 64


def _keys(k0, k1, t, r, lane):
    return philox.philox_vec(t, np.uint64(r), np.uint64(lane), 0, k0, k1)[0]


def stub_matching(h, seed: int, copy: int):
    """One null copy: (members uint32, offsets uint64) with the input's size sequence."""
    nh = h if isinstance(h, Normalised) else normalise(h)
    sizes = np.array([len(e) for e in nh.order], dtype=np.int64)
    offsets = np.zeros(len(sizes) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    stubs = np.array([v for e in nh.order for v in e], dtype=np.int64)
    n_edges = len(sizes)
    k0, k1 = philox.stream_key(seed, philox.DOMAIN_NULL, copy)
    t = np.arange(len(stubs), dtype=np.uint64)
    keys = _keys(k0, k1, t, 0, 0)
    members = stubs[np.lexsort((np.arange(len(stubs)), keys))]
    for r in range(1, MAX_REPAIR_ROUNDS + 1):
        bad = [i for i in range(n_edges)
               if len(set(members[offsets[i]:offsets[i + 1]].tolist())) != sizes[i]]
        if not bad:
            return members.astype(np.uint32), offsets.astype(np.uint64)
        q = np.arange(len(bad), dtype=np.uint64)
        partners = philox.bounded(_keys(k0, k1, q, r, 1), n_edges).astype(np.int64)
        chosen = sorted(set(bad) | set(partners.tolist()))
        pool = np.concatenate([members[offsets[i]:offsets[i + 1]] for i in chosen])
        pk = _keys(k0, k1, np.arange(len(pool), dtype=np.uint64), r, 0)
        pool = pool[np.lexsort((np.arange(len(pool)), pk))]
        pos = 0
        for i in chosen:
            members[offsets[i]:offsets[i + 1]] = pool[pos:pos + sizes[i]]
            pos += sizes[i]
    raise RuntimeError("stub matching: repeated nodes remain after the repair rounds")


def degree_sequence(members, offsets, n_nodes: int) -> np.ndarray:
    sizes = np.diff(np.asarray(offsets, dtype=np.int64))
    keep = np.repeat(sizes >= 2, sizes)
    return np.bincount(np.asarray(members, dtype=np.int64)[keep], minlength=n_nodes)


def check_null_invariants(h, members, offsets) -> None:
    """The copy keeps the size sequence and every node degree, and repeats no node."""
    nh = h if isinstance(h, Normalised) else normalise(h)
    sizes = np.array([len(e) for e in nh.order], dtype=np.int64)
    got_sizes = np.diff(np.asarray(offsets, dtype=np.int64))
    if not np.array_equal(sizes, got_sizes):
        raise AssertionError("size sequence changed")
    ref_off = np.zeros(len(sizes) + 1, dtype=np.int64)
    ref_off[1:] = np.cumsum(sizes)
    ref_members = np.array([v for e in nh.order for v in e], dtype=np.int64)
    if not np.array_equal(degree_sequence(ref_members, ref_off, nh.n_nodes),
                          degree_sequence(members, offsets, nh.n_nodes)):
        raise AssertionError("degree sequence changed")
    m = np.asarray(members, dtype=np.int64)
    off = np.asarray(offsets, dtype=np.int64)
    for i in range(len(sizes)):
        e = m[off[i]:off[i + 1]]
        if len(np.unique(e)) != len(e):
            raise AssertionError(f"hyperedge {i} repeats a node")


def zscores(real: np.ndarray, nulls: np.ndarray) -> np.ndarray:
    """z_m = (x_m - mean_m) / sd_m over the null copies (sd with n-1), float64.

    A class with sd = 0 scores 0 when x equals the mean, else +/-inf.
    """
    x = np.asarray(real, dtype=np.float64)
    y = np.asarray(nulls, dtype=np.float64)
    n = y.shape[0]
    mu = y.sum(axis=0) / n
    var = ((y - mu) ** 2).sum(axis=0) / (n - 1)
    sd = np.sqrt(var)
    z = np.zeros_like(x)
    nz = sd > 0
    z[nz] = (x[nz] - mu[nz]) / sd[nz]
    z[~nz & (x > mu)] = np.inf
    z[~nz & (x < mu)] = -np.inf
    return z
