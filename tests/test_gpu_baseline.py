"""The projection baseline (Algorithm 1) through the C ABI on the GPU against
the oracle: counts bit-exact, and the candidates ESU enumerates (and those it
discards) equal to the oracle's."""
import json
import os
from math import comb

import numpy as np
import pytest

import workloads as W
from oracle import core

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def hm():
    import torch
    import paper_2209_10241_amd as hm
    assert torch.cuda.is_available()
    return hm


def _gpu(hm, h, k):
    with hm.hm_graph_create(h.members, h.offsets, h.n_nodes) as g:
        counts, stats = hm.count_baseline(g, k)
        return counts.cpu().numpy(), [int(x) for x in stats.cpu().numpy()]


def _golden(name, k):
    with open(os.path.join(ROOT, "tests", "golden", "workload_counts.json")) as f:
        for c in json.load(f)["cases"]:
            if c["workload"] == name and c["k"] == k:
                return np.array(c["counts"], dtype=np.int64)
    raise KeyError(name)


# node counts spanning one to ten 32-bit words per row (ragged last word)
# and the largest graph kept as bit rows (8192 nodes, 256 words), hyperedges
# of size 1 to 7 with repeats
CASES = [(0, 20, 60), (1, 33, 90), (2, 64, 150), (3, 97, 220), (4, 150, 260), (5, 300, 400), (6, 8192, 6000)]


@pytest.mark.parametrize("k", [3, 4])
@pytest.mark.parametrize("seed,n,e", CASES)
def test_random_matches_oracle(hm, seed, n, e, k):
    h = W.random_small(700 + seed, n, e, {1: 0.05, 2: 0.45, 3: 0.25, 4: 0.12, 5: 0.06, 7: 0.07}, allow_dups=True)
    print(f"baseline k={k} seed={seed} n={n} e={e}", flush=True)
    want, cand, disc = core.count_baseline(h, k)
    got, stats = _gpu(hm, h, k)
    assert np.array_equal(got, want)
    assert stats == [cand, disc]


@pytest.mark.parametrize("k", [3, 4])
def test_degenerate_inputs(hm, k):
    cases = [
        W.from_lists([[0, 1, 2, 3, 4]], n_nodes=5),          # one hyperedge above the order: all discarded
        W.from_lists([[0, 1]], n_nodes=3),                    # too few nodes for a motif
        W.from_lists([[0], [1], [2]], n_nodes=3),             # singletons only
        W.from_lists([[0, 1], [1, 2], [2, 3], [0, 3]], n_nodes=40),
        W.from_lists([[0, 1, 2, 3], [1, 2, 3], [2, 3]], n_nodes=4),
    ]
    for h in cases:
        want, cand, disc = core.count_baseline(h, k)
        got, stats = _gpu(hm, h, k)
        assert np.array_equal(got, want)
        assert stats == [cand, disc]


def test_repeated_calls_agree(hm):
    h = W.random_small(9, 90, 200, {2: 0.5, 3: 0.3, 4: 0.15, 6: 0.05})
    with hm.hm_graph_create(h.members, h.offsets, h.n_nodes) as g:
        first = [x.cpu().numpy().copy() for x in hm.count_baseline(g, 4)]
        exact = hm.count_exact(g, 4).cpu().numpy()
        again = [x.cpu().numpy() for x in hm.count_baseline(g, 4)]
        third = [x.cpu().numpy() for x in hm.count_baseline(g, 3)]
    assert np.array_equal(first[0], again[0]) and np.array_equal(first[1], again[1])
    assert np.array_equal(first[0], exact)
    want3, cand3, disc3 = core.count_baseline(h, 3)
    assert np.array_equal(third[0], want3) and list(third[1]) == [cand3, disc3]


def test_face_to_face_order3_matches_golden(hm):
    h = W.cfg0_facetoface_k3(0)
    got, (cand, disc) = _gpu(hm, h, 3)
    assert np.array_equal(got, _golden("facetoface_N200_E2000", 3))
    assert cand - disc == int(got.sum())


def test_face_to_face_order4_matches_golden(hm):
    # the benchmark's workload at full size: the counts are the oracle's
    # (stored), the candidates bounded by the 4-node sets
    h = W.cfg1_facetoface_k4(0)
    got, (cand, disc) = _gpu(hm, h, 4)
    assert np.array_equal(got, _golden("facetoface_N400_E30000", 4))
    assert cand - disc == int(got.sum())
    assert int(got.sum()) < cand <= comb(h.n_nodes, 4)


def test_without_bit_rows_is_refused(hm):
    h = W.random_small(3, 60, 100, {2: 0.6, 3: 0.4})
    hm.hm_set_option(hm.HM_OPT_BITSET_MAX_NODES, 32)
    try:
        with hm.hm_graph_create(h.members, h.offsets, h.n_nodes) as g:
            with pytest.raises(hm.HMError):
                hm.count_baseline(g, 4)
            with pytest.raises(hm.HMError):
                hm.count_baseline(g, 5)
    finally:
        hm.hm_set_option(hm.HM_OPT_BITSET_MAX_NODES, 8192)
