"""count_exact_noalloc (the entry point for callers that cannot allocate
device memory) through the C ABI against count_exact: bit-exact int64 on two
calls in a row, the second on a smaller graph, at both orders; and the
refusal of a graph without bit rows."""
import ctypes
import json
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def hm():
    import torch
    import paper_2209_10241_amd as hm
    assert torch.cuda.is_available()
    return hm


def _noalloc(hm, g, k):
    import torch
    out = torch.full((hm.hm_num_classes(k),), -1, dtype=torch.int64, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = hm.lib().count_exact_noalloc(g.handle, k, ctypes.c_void_p(out.data_ptr()), st)
    assert rc == 0, hm.lib().hm_last_error().decode()
    return out.cpu().numpy()


def _golden(name, k):
    with open(os.path.join(ROOT, "tests", "golden", "workload_counts.json")) as f:
        for c in json.load(f)["cases"]:
            if c["workload"] == name and c["k"] == k:
                return np.array(c["counts"], dtype=np.int64)
    raise KeyError(name)


@pytest.mark.parametrize("k", [3, 4])
def test_noalloc_matches_count_exact_twice(hm, k):
    big = W.cfg1_facetoface_k4(0)                                      # 400 nodes, 30,000 hyperedges
    small = W.random_small(8800 + k, 60, 500, {2: 0.5, 3: 0.3, 4: 0.2}, allow_dups=True)
    with hm.hm_graph_create(big.members, big.offsets, big.n_nodes) as gb, \
            hm.hm_graph_create(small.members, small.offsets, small.n_nodes) as gs:
        first = _noalloc(hm, gb, k)
        second = _noalloc(hm, gs, k)
        want_first = hm.count_exact(gb, k).cpu().numpy()
        want_second = hm.count_exact(gs, k).cpu().numpy()
    assert np.array_equal(first, want_first)
    assert np.array_equal(second, want_second)
    if k == 4:
        assert np.array_equal(first, _golden("facetoface_N400_E30000", 4))


def test_noalloc_refuses_graphs_without_bit_rows(hm):
    h = W.random_small(8900, 40, 200, {2: 0.6, 3: 0.4})
    hm.hm_set_option(hm.HM_OPT_BITSET_MAX_NODES, 0)
    try:
        with hm.hm_graph_create(h.members, h.offsets, h.n_nodes) as g:
            import torch
            out = torch.zeros(171, dtype=torch.int64, device="cuda")
            rc = hm.lib().count_exact_noalloc(g.handle, 4, ctypes.c_void_p(out.data_ptr()), None)
            assert rc == hm.binding.HM_EUNSUPPORTED
            assert b"bit rows" in hm.lib().hm_last_error()
            assert int(out.abs().sum()) == 0
    finally:
        hm.hm_set_option(hm.HM_OPT_BITSET_MAX_NODES, 8192)
