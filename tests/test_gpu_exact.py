"""Exact counts through the C ABI on the GPU against the oracle (bit-exact int64)."""
import json
import os

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


def _gpu_counts(hm, h, k, bit_rows=True):
    """Counts through the C ABI; bit_rows=False forces the hash-probe kernels."""
    hm.hm_set_option(hm.HM_OPT_BITSET_MAX_NODES, 8192 if bit_rows else 0)
    try:
        with hm.hm_graph_create(h.members, h.offsets, h.n_nodes) as g:
            return hm.count_exact(g, k).cpu().numpy()
    finally:
        hm.hm_set_option(hm.HM_OPT_BITSET_MAX_NODES, 8192)


def _golden(name, k):
    with open(os.path.join(ROOT, "tests", "golden", "workload_counts.json")) as f:
        for c in json.load(f)["cases"]:
            if c["workload"] == name and c["k"] == k:
                return np.array(c["counts"], dtype=np.int64)
    raise KeyError(name)


def test_ingest_strata_match_oracle(hm):
    h = W.random_small(3, 30, 300, {1: 0.05, 2: 0.5, 3: 0.3, 4: 0.1, 5: 0.05}, allow_dups=True)
    nh = core.normalise(h)
    with hm.hm_graph_create(h.members, h.offsets, h.n_nodes) as g:
        st = g.stats()
        assert (st["n2"], st["n3"], st["n4"]) == (nh.count(2), nh.count(3), nh.count(4))
        assert st["singletons"] == nh.n_dropped_singletons and st["duplicates"] == nh.n_duplicates
        for j in (2, 3, 4):
            assert np.array_equal(g.export(j).astype(np.int64), nh.edges(j))


@pytest.mark.parametrize("bit_rows", [True, False], ids=["bits", "hash"])
@pytest.mark.parametrize("seed", range(40))
def test_random_small_matches_oracle(hm, seed, bit_rows):
    mixes = [{2: 0.6, 3: 0.3, 4: 0.1}, {1: 0.05, 2: 0.45, 3: 0.3, 4: 0.15, 5: 0.05}, {2: 0.2, 3: 0.5, 4: 0.3},
             {2: 1.0}, {3: 0.5, 4: 0.5}]
    n = 12 + (seed * 7) % 60
    h = W.random_small(1000 + seed, n, 20 + (seed * 37) % 400, mixes[seed % len(mixes)], allow_dups=bool(seed % 3))
    for k in (3, 4):
        assert np.array_equal(_gpu_counts(hm, h, k, bit_rows), core.count_exact(h, k)), (seed, k)


def test_hand_examples(hm, golden_dir):
    with open(os.path.join(golden_dir, "hand_examples.json")) as f:
        examples = json.load(f)["examples"]
    for ex in examples:
        h = W.from_lists(ex["edges"], ex["n_nodes"])
        for k in (3, 4):
            for bit_rows in (True, False):
                assert np.array_equal(_gpu_counts(hm, h, k, bit_rows), core.count_exact(h, k)), ex["name"]


@pytest.mark.parametrize("bit_rows", [True, False], ids=["bits", "hash"])
def test_facetoface_order3_workload(hm, bit_rows):
    h = W.cfg0_facetoface_k3(0)
    assert np.array_equal(_gpu_counts(hm, h, 3, bit_rows), _golden("facetoface_N200_E2000", 3))


@pytest.mark.parametrize("bit_rows", [True, False], ids=["bits", "hash"])
def test_facetoface_order4_workload(hm, bit_rows):
    """The benchmark's workload: N=400, 30,000 hyperedges, k=4."""
    h = W.cfg1_facetoface_k4(0)
    assert np.array_equal(_gpu_counts(hm, h, 4, bit_rows), _golden("facetoface_N400_E30000", 4))


@pytest.mark.parametrize("bit_rows", [True, False], ids=["bits", "hash"])
def test_communication_scaled_workload(hm, bit_rows):
    """Heavy-tailed degrees (communication recipe at 0.4% of its size), stored oracle counts."""
    h = W.scaled_communication(0.004, 0)
    assert np.array_equal(_gpu_counts(hm, h, 4, bit_rows), _golden("communication_scaled_0.004", 4))


def _heavy_goldens():
    with open(os.path.join(ROOT, "tests", "golden", "workload_counts.json")) as f:
        names = [c["workload"] for c in json.load(f)["cases"]]
    out = []
    for name in names:
        for family, maker in (("communication", W.scaled_communication), ("coauthorship", W.scaled_coauthorship)):
            prefix = f"{family}_scaled_"
            if name.startswith(prefix) and name != "communication_scaled_0.004":
                out.append((name, maker, float(name[len(prefix):])))
    return out


@pytest.mark.parametrize("bit_rows", [True, False], ids=["bits", "hash"])
@pytest.mark.parametrize("name,maker,scale", _heavy_goldens(), ids=[c[0] for c in _heavy_goldens()])
def test_heavy_tailed_scaled_goldens(hm, name, maker, scale, bit_rows):
    """The heavy-tailed recipes at the largest fractions of their size whose
    oracle counts are stored (Algorithm 3 on every host core): both GPU paths
    bit-exact.  Graphs with more nodes than bit rows hold have one path."""
    h = maker(scale, 0)
    if bit_rows and h.n_nodes > 8192:
        pytest.skip(f"{h.n_nodes} nodes: more than adjacency bit rows hold, the hash path is the only one")
    assert np.array_equal(_gpu_counts(hm, h, 4, bit_rows), _golden(name, 4))


@pytest.fixture(scope="module")
def full_size():
    """The co-authorship (10^6 nodes, 2x10^6 draws) and communication (5x10^4
    nodes, 5x10^6 draws) workloads at full size, generated once."""
    out = {}
    for name, maker in (("coauthorship", W.cfg3_coauthorship), ("communication", W.cfg4_communication)):
        print(f"generating {name}", flush=True)
        out[name] = maker(0)
    return out


@pytest.mark.parametrize("name", ["coauthorship", "communication"])
def test_full_size_relabelling_and_census(hm, full_size, name):
    """At full size, where the oracle cannot run: (1) the exact counts do not
    change under a fixed node relabelling (Section 3: a motif is an
    isomorphism class), and (2) a census through the sampler - every
    hyperedge of size 2..4 drawn exactly once (Algorithm 4 with S_j = |E_j|)
    - gives raw counts countmax_m * n_m for every class and estimates equal to
    the exact counts.  The sampler enumerates each hyperedge's neighbourhood;
    the exact count uses graph identities and ownership rules: two
    independent routes to the same int64 vector."""
    h = full_size[name]
    with hm.hm_graph_create(h.members, h.offsets, h.n_nodes) as g:
        exact = hm.count_exact(g, 4).cpu().numpy()
        st = g.stats()
        samples = {j: np.arange(st[f"n{j}"]) for j in range(2, 5)}
        print(f"{name}: census of {sum(len(v) for v in samples.values())} hyperedges", flush=True)
        est, raw = hm.count_sampled_indices(g, 4, samples)
    countmax = np.array([hm.hm_class_info(4, c)[2] for c in range(len(exact))], dtype=np.int64)
    assert exact.sum() > 10**12
    assert np.array_equal(raw.cpu().numpy(), exact * countmax)
    assert np.array_equal(est.cpu().numpy(), exact.astype(np.float32))
    perm = np.random.default_rng(11).permutation(h.n_nodes)
    hp = W.Hypergraph(h.n_nodes, perm[h.members.astype(np.int64)].astype(np.uint32), h.offsets.copy())
    print(f"{name}: relabelled count", flush=True)
    assert np.array_equal(_gpu_counts(hm, hp, 4), exact)


@pytest.mark.parametrize("scale", [0.02, 0.05])
def test_sparse_path_agrees_with_bit_rows(hm, scale):
    """Larger heavy-tailed graphs: the counting formulas without bit rows and the
    bit-row enumeration are independent routes to the same int64 counts."""
    h = W.scaled_communication(scale, 1)
    for k in (3, 4):
        a = _gpu_counts(hm, h, k, True)
        b = _gpu_counts(hm, h, k, False)
        assert np.array_equal(a, b), (scale, k)
        assert a.sum() > 0


@pytest.mark.parametrize("bit_rows", [True, False], ids=["bits", "hash"])
def test_repeated_calls_on_one_graph(hm, bit_rows):
    """The counting scratch is left clear after every call: orders alternate on
    one graph and every call matches the oracle."""
    h = W.random_small(77, 50, 600, {2: 0.5, 3: 0.3, 4: 0.2}, allow_dups=True)
    want = {k: core.count_exact(h, k) for k in (3, 4)}
    hm.hm_set_option(hm.HM_OPT_BITSET_MAX_NODES, 8192 if bit_rows else 0)
    try:
        with hm.hm_graph_create(h.members, h.offsets, h.n_nodes) as g:
            for k in (4, 4, 3, 4, 3, 3, 4):
                assert np.array_equal(hm.count_exact(g, k).cpu().numpy(), want[k]), k
    finally:
        hm.hm_set_option(hm.HM_OPT_BITSET_MAX_NODES, 8192)


def test_facetoface_order4_relabelled(hm):
    h = W.cfg1_facetoface_k4(0)
    perm = np.random.default_rng(5).permutation(h.n_nodes)
    hp = W.Hypergraph(h.n_nodes, perm[h.members.astype(np.int64)].astype(np.uint32), h.offsets.copy())
    assert np.array_equal(_gpu_counts(hm, hp, 4), _golden("facetoface_N400_E30000", 4))


@pytest.mark.parametrize("n_ids", [200_000, 1 << 22], ids=["ids_2e5", "ids_4M"])
@pytest.mark.parametrize("seed", range(3))
def test_large_node_ids(hm, seed, n_ids):
    """More nodes than the adjacency bit rows allow: pairs are probed in the hash set.
    At 2^22 ids three node ids no longer pack into 63 bits, so the 4-node
    hyperedges holding a 3-node one are found through the incidence lists
    instead of the 3-subset index."""
    base = W.random_small(2000 + seed, 60, 500, {2: 0.6, 3: 0.3, 4: 0.1})
    rng = np.random.default_rng(seed)
    ids = np.sort(rng.choice(n_ids, size=60, replace=False))
    h = W.Hypergraph(n_ids, ids[base.members.astype(np.int64)].astype(np.uint32), base.offsets.copy())
    for k in (3, 4):
        assert np.array_equal(_gpu_counts(hm, h, k), core.count_exact(h, k)), (seed, k)


def test_device_resident_input(hm):
    import torch
    h = W.random_small(77, 50, 400, {2: 0.5, 3: 0.3, 4: 0.2})
    m = torch.from_numpy(h.members.astype(np.int32)).cuda()
    o = torch.from_numpy(h.offsets.astype(np.int64)).cuda()
    with hm.hm_graph_create(m, o, h.n_nodes) as g:
        for k in (3, 4):
            assert np.array_equal(hm.count_exact(g, k).cpu().numpy(), core.count_exact(h, k))


def test_degenerate_inputs(hm):
    empty = W.Hypergraph(5, np.zeros(0, np.uint32), np.zeros(1, np.uint64))
    singles = W.from_lists([[0], [3], [4]], 5)
    big_only = W.from_lists([[0, 1, 2, 3, 4]], 5)
    for h in (empty, singles, big_only):
        for k in (3, 4):
            assert _gpu_counts(hm, h, k).sum() == 0


@pytest.mark.parametrize("edges,n", [([[0, 1], [2, 2]], 3), ([[0, 7]], 3)])
def test_invalid_inputs(hm, edges, n):
    h = W.from_lists(edges, n)
    with pytest.raises(hm.HMError) as e:
        hm.hm_graph_create(h.members, h.offsets, n)
    assert e.value.code == -1


def test_empty_hyperedge_is_rejected(hm):
    with pytest.raises(hm.HMError):
        hm.hm_graph_create(np.array([0, 1], np.uint32), np.array([0, 2, 2], np.uint64), 3)


@pytest.mark.parametrize("where", ["host", "device"])
@pytest.mark.parametrize("offsets", [[1, 3, 5], [0, 3, 2], [0, 2, 7]], ids=["start", "decrease", "beyond"])
def test_bad_offsets_are_rejected(hm, where, offsets):
    """Offsets must start at 0, not decrease and stay within the members."""
    import torch
    m = np.array([0, 1, 2, 3, 4], np.uint32)
    o = np.array(offsets, np.uint64)
    if where == "device":
        m = torch.from_numpy(m.astype(np.int32)).cuda()
        o = torch.from_numpy(o.astype(np.int64)).cuda()
    with pytest.raises(hm.HMError) as e:
        hm.hm_graph_create(m, o, 6)
    assert e.value.code == -1


def test_members_beyond_the_last_offset_are_ignored(hm):
    """Trailing entries of members that no hyperedge reaches do not count."""
    import torch
    h = W.random_small(78, 30, 200, {2: 0.5, 3: 0.3, 4: 0.2})
    tail = np.array([29, 29, 29], np.uint32)
    for dev in (False, True):
        m = np.concatenate([h.members.astype(np.uint32), tail])
        o = h.offsets.astype(np.uint64)
        if dev:
            m = torch.from_numpy(m.astype(np.int32)).cuda()
            o = torch.from_numpy(o.astype(np.int64)).cuda()
        with hm.hm_graph_create(m, o, h.n_nodes) as g:
            assert np.array_equal(hm.count_exact(g, 4).cpu().numpy(), core.count_exact(h, 4))


def test_many_graphs_created_and_destroyed_in_stream_order(hm):
    """Graphs destroyed without a device-wide wait: memory released in stream
    order is not reused before the work that reads it has run."""
    import torch
    hs = [W.random_small(90 + i, 40, 300, {2: 0.5, 3: 0.3, 4: 0.2}) for i in range(6)]
    want = [core.count_exact(h, 4) for h in hs]
    outs = []
    for _ in range(3):
        for h in hs:
            m = torch.from_numpy(h.members.astype(np.int32)).cuda()
            o = torch.from_numpy(h.offsets.astype(np.int64)).cuda()
            g = hm.hm_graph_create(m, o, h.n_nodes)
            outs.append(hm.count_exact(g, 4))
            g.close()
    torch.cuda.synchronize()
    for i, c in enumerate(outs):
        assert np.array_equal(c.cpu().numpy(), want[i % len(hs)]), i


@pytest.fixture(params=["one_pass", "two_pass"])
def build_mode(hm, request):
    """Graphs built in one pass (buffers sized by bounds) or in two (sized
    exactly after the counting pass)."""
    hm.hm_set_option(hm.HM_OPT_ONE_PASS_MAX_EDGES, (1 << 20) if request.param == "one_pass" else 0)
    yield request.param
    hm.hm_set_option(hm.HM_OPT_ONE_PASS_MAX_EDGES, 1 << 20)


@pytest.mark.parametrize("seed", range(6))
def test_build_modes_match_oracle(hm, build_mode, seed):
    h = W.random_small(500 + seed, 20 + 9 * seed, 100 + 90 * seed, {1: 0.05, 2: 0.5, 3: 0.3, 4: 0.1, 5: 0.05},
                       allow_dups=True)
    nh = core.normalise(h)
    with hm.hm_graph_create(h.members, h.offsets, h.n_nodes) as g:
        st = g.stats()
        assert (st["n2"], st["n3"], st["n4"]) == (nh.count(2), nh.count(3), nh.count(4))
        for j in (2, 3, 4):
            assert np.array_equal(g.export(j).astype(np.int64), nh.edges(j))
        for k in (3, 4):
            assert np.array_equal(hm.count_exact(g, k).cpu().numpy(), core.count_exact(h, k)), k
        est, _ = hm.count_sampled(g, 4, 0.5, 3)
        assert np.isfinite(est.cpu().numpy()).all()


@pytest.mark.parametrize("edges,n", [([[0, 1], [2, 2]], 3), ([[0, 7]], 3), ([[0, 1], [1, 2, 9]], 4)])
def test_build_modes_reject_invalid_input(hm, build_mode, edges, n):
    h = W.from_lists(edges, n)
    with pytest.raises(hm.HMError) as e:
        hm.hm_graph_create(h.members, h.offsets, n)
    assert e.value.code == -1
    # the library is still usable afterwards
    ok = W.random_small(7, 12, 40, {2: 0.6, 3: 0.4})
    with hm.hm_graph_create(ok.members, ok.offsets, ok.n_nodes) as g:
        assert np.array_equal(hm.count_exact(g, 4).cpu().numpy(), core.count_exact(ok, 4))


def test_one_pass_option_bounds(hm):
    with pytest.raises(hm.HMError):
        hm.hm_set_option(hm.HM_OPT_ONE_PASS_MAX_EDGES, (1 << 20) + 1)
    with pytest.raises(hm.HMError):
        hm.hm_set_option(hm.HM_OPT_ONE_PASS_MAX_EDGES, -1)
    assert hm.hm_get_option(hm.HM_OPT_ONE_PASS_MAX_EDGES) == 1 << 20


def test_wide_bit_rows(hm):
    """More than 64 words per bit row (N > 2048): the word loop of the pairs-only kernel."""
    base = W.random_small(3000, 80, 900, {2: 0.6, 3: 0.3, 4: 0.1})
    ids = np.sort(np.random.default_rng(9).choice(8000, size=80, replace=False))
    h = W.Hypergraph(8000, ids[base.members.astype(np.int64)].astype(np.uint32), base.offsets.copy())
    for k in (3, 4):
        assert np.array_equal(_gpu_counts(hm, h, k), core.count_exact(h, k)), k


def test_bit_row_option_bounds(hm):
    with pytest.raises(hm.HMError):
        hm.hm_set_option(hm.HM_OPT_BITSET_MAX_NODES, 8193)
    with pytest.raises(hm.HMError):
        hm.hm_set_option(99, 0)


def _hub_hypergraph(seed=11, n=150):
    """Hubs 0 and 1 with more than 64 pairwise neighbours each, the pair {0, 1}
    in 99 3-node hyperedges and {0, 2} in 38, and the 3-node hyperedge
    {0, 1, 2} inside 88 4-node hyperedges, over random background hyperedges:
    the exact step without bit rows meets lists both short enough to hold in
    LDS and too long to."""
    rng = np.random.default_rng(seed)
    E = set()

    def add(t):
        E.add(tuple(sorted(int(x) for x in t)))

    def count(k):
        return sum(1 for e in E if len(e) == k)

    for y in range(2, 91):
        add((0, y))
        add((1, y))
    while count(2) < 700:
        add(rng.choice(n, 2, replace=False))
    for y in range(2, 101):
        add((0, 1, y))
    for y in range(3, 41):
        add((0, 2, y))
    target = count(3) + 300
    while count(3) < target:
        add(rng.choice(n, 3, replace=False))
    for y in range(3, 91):
        add((0, 1, 2, y))
    target = count(4) + 200
    while count(4) < target:
        add(rng.choice(n, 4, replace=False))
    return W.from_lists([list(e) for e in sorted(E)], n)


@pytest.mark.parametrize("bit_rows", [True, False], ids=["bits", "hash"])
def test_hub_lists_match_oracle(hm, bit_rows):
    h = _hub_hypergraph()
    for k in (3, 4):
        assert np.array_equal(_gpu_counts(hm, h, k, bit_rows), core.count_exact(h, k)), k


@pytest.fixture
def hub_rows(hm):
    """Dense adjacency rows for every node with at least 2 pairwise
    neighbours, so that the bit-free kernels read rows instead of probing."""
    hm.hm_set_option(hm.HM_OPT_HUB_MIN_DEGREE, 2)
    try:
        yield
    finally:
        hm.hm_set_option(hm.HM_OPT_HUB_MIN_DEGREE, 256)


def test_hub_rows_match_oracle(hm, hub_rows):
    h = _hub_hypergraph()
    assert np.array_equal(_gpu_counts(hm, h, 4, bit_rows=False), core.count_exact(h, 4))
    h = W.scaled_communication(0.004, 0)
    assert np.array_equal(_gpu_counts(hm, h, 4, bit_rows=False), _golden("communication_scaled_0.004", 4))
    for seed in range(6):
        h = W.random_small(7100 + seed, 30 + 9 * seed, 200 + 60 * seed, {2: 0.5, 3: 0.35, 4: 0.15})
        assert np.array_equal(_gpu_counts(hm, h, 4, bit_rows=False), core.count_exact(h, 4)), seed


def test_hub_option_bounds(hm):
    with pytest.raises(hm.HMError):
        hm.hm_set_option(hm.HM_OPT_HUB_MIN_DEGREE, -1)
    with pytest.raises(hm.HMError):
        hm.hm_set_option(hm.HM_OPT_HUB_MIN_DEGREE, 1 << 32)
    assert hm.hm_get_option(hm.HM_OPT_HUB_MIN_DEGREE) == 256


def test_concurrent_threads_own_streams(hm):
    """Graphs built and counted from several host threads at once, each on its
    own stream, as the benchmark's throughput measurement runs them: every
    count equals the stored oracle counts, and an invalid input on one thread
    fails there alone with its own message."""
    import threading
    import torch
    dev = torch.device("cuda:0")
    h = W.cfg1_facetoface_k4(0)
    want = _golden("facetoface_N400_E30000", 4)
    members = torch.from_numpy(h.members.astype(np.int32)).to(dev)
    offsets = torch.from_numpy(h.offsets.astype(np.int64)).to(dev)
    bad = members.clone()
    bad[5] = h.n_nodes   # a node id out of range
    n_threads, per = 3, 12
    results, errors = {}, []

    def worker(t):
        try:
            torch.cuda.set_device(dev)
            st = torch.cuda.Stream()
            out = []
            for i in range(per):
                if t == 2 and i % 4 == 1:
                    with pytest.raises(hm.HMError, match="node id"):
                        hm.hm_graph_create(bad, offsets, h.n_nodes, stream=st)
                    continue
                with hm.hm_graph_create(members, offsets, h.n_nodes, stream=st) as g:
                    c = hm.count_exact(g, 4, stream=st)
                st.synchronize()
                out.append(c.cpu().numpy())
            results[t] = out
        except BaseException as e:
            errors.append(e)

    th = [threading.Thread(target=worker, args=(t,)) for t in range(n_threads)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    assert not errors, errors[0]
    assert sorted(results) == list(range(n_threads))
    for t, out in results.items():
        assert len(out) == (per - 3 if t == 2 else per)
        for c in out:
            assert np.array_equal(c, want), t


@pytest.mark.parametrize("bit_rows", [True, False], ids=["bits", "hash"])
@pytest.mark.parametrize("tag_bits", [0, 1, -1, 32])
def test_duplicate_search_paths(hm, tag_bits, bit_rows):
    """The build's duplicate search.  With 0 tag bits every probe meets the
    first entry on its way, with 1 about half the meetings are of different
    hyperedges: the build finds them one launch later and repeats the search
    exactly.  -1 takes the exact search from the start, 32 is the default.
    Strata, singleton and duplicate counts and the order-4 counts equal the
    oracle's either way."""
    hm.hm_set_option(hm.HM_OPT_DEDUP_TAG_BITS, tag_bits)
    hm.hm_set_option(hm.HM_OPT_BITSET_MAX_NODES, 8192 if bit_rows else 0)
    try:
        for seed in range(6):
            h = W.random_small(500 + seed, 40, 100 + 60 * seed, {1: 0.05, 2: 0.45, 3: 0.3, 4: 0.15, 5: 0.05},
                               allow_dups=True)
            nh = core.normalise(h)
            with hm.hm_graph_create(h.members, h.offsets, h.n_nodes) as g:
                st = g.stats()
                assert (st["n2"], st["n3"], st["n4"]) == (nh.count(2), nh.count(3), nh.count(4)), seed
                assert st["singletons"] == nh.n_dropped_singletons and st["duplicates"] == nh.n_duplicates, seed
                for j in (2, 3, 4):
                    assert np.array_equal(g.export(j).astype(np.int64), nh.edges(j)), (seed, j)
                assert np.array_equal(hm.count_exact(g, 4).cpu().numpy(), core.count_exact(h, 4)), seed
    finally:
        hm.hm_set_option(hm.HM_OPT_DEDUP_TAG_BITS, 32)
        hm.hm_set_option(hm.HM_OPT_BITSET_MAX_NODES, 8192)


def test_invalid_input_then_valid_same_size(hm):
    """A build that fails validation leaves its duplicate-search table
    unreturned to the all-ones state; the next build of the same size must
    not take it for a clean one.  Alternating invalid and valid builds of one
    size keeps giving the oracle's counts."""
    h = W.random_small(77, 50, 400, {2: 0.5, 3: 0.3, 4: 0.2}, allow_dups=True)
    want = core.count_exact(h, 4)
    bad = h.members.copy()
    bad[3] = h.n_nodes
    for _ in range(4):
        with pytest.raises(hm.HMError, match="node id"):
            hm.hm_graph_create(bad, h.offsets, h.n_nodes)
        with hm.hm_graph_create(h.members, h.offsets, h.n_nodes) as g:
            assert np.array_equal(hm.count_exact(g, 4).cpu().numpy(), want)


def _device_graphs(hs):
    import torch
    dev = torch.device("cuda:0")
    return [(torch.from_numpy(h.members.astype(np.int32)).to(dev), torch.from_numpy(h.offsets.astype(np.int64)).to(dev),
             h.n_nodes) for h in hs]


@pytest.mark.parametrize("workers", [1, 3, 8])
def test_count_exact_many_matches_oracle(hm, workers):
    """Many hypergraphs in one call, shared among worker threads with a
    stream each: every row equals the oracle's counts of its hypergraph
    (different sizes, repeated hyperedges and singletons)."""
    hs = [W.random_small(900 + s, 10 + 9 * s, 40 + 50 * s, {1: 0.05, 2: 0.45, 3: 0.3, 4: 0.15, 5: 0.05},
                         allow_dups=True) for s in range(12)]
    # and the degenerate cases: no hyperedge, singletons only, one pair
    hs += [W.Hypergraph(7, np.zeros(0, np.uint32), np.zeros(1, np.uint64)),
           W.Hypergraph(5, np.array([0, 3, 4], np.uint32), np.array([0, 1, 2, 3], np.uint64)),
           W.Hypergraph(4, np.array([1, 2], np.uint32), np.array([0, 2], np.uint64))]
    graphs = _device_graphs(hs)
    for k in (3, 4):
        got = hm.count_exact_many(graphs, k, workers=workers).cpu().numpy()
        assert got.shape == (len(hs), hm.hm_num_classes(k))
        for g, h in enumerate(hs):
            assert np.array_equal(got[g], core.count_exact(h, k)), (k, g)


def test_count_exact_many_benchmark_workload(hm):
    """The benchmark's workload 24 times over in one call, three workers:
    every row equals the stored oracle counts."""
    h = W.cfg1_facetoface_k4(0)
    got = hm.count_exact_many(_device_graphs([h]) * 24, 4, workers=3).cpu().numpy()
    want = _golden("facetoface_N400_E30000", 4)
    for g in range(24):
        assert np.array_equal(got[g], want), g


@pytest.mark.parametrize("workers", [1, 3])
def test_count_exact_many_reports_the_failing_graph(hm, workers):
    """An invalid hypergraph among valid ones: the call fails with the
    hypergraph's index and its validation message, and the next call on valid
    input counts as before."""
    good = W.random_small(31, 30, 200, {2: 0.5, 3: 0.3, 4: 0.2}, allow_dups=True)
    bad_members = good.members.copy()
    bad_members[7] = good.n_nodes
    bad = W.Hypergraph(good.n_nodes, bad_members, good.offsets)
    graphs = _device_graphs([good, good, good, bad, good, good])
    with pytest.raises(hm.HMError, match="hypergraph 3: .*node id"):
        hm.count_exact_many(graphs, 4, workers=workers)
    got = hm.count_exact_many(_device_graphs([good] * 4), 4, workers=workers).cpu().numpy()
    for g in range(4):
        assert np.array_equal(got[g], core.count_exact(good, 4))


def test_count_exact_many_host_memory(hm):
    """count_exact_many with the hypergraphs in host memory (HM_MEM_HOST),
    called through the C ABI: each worker copies its graphs' arrays to the
    device on its own stream; every row equals the oracle's counts."""
    import ctypes
    import torch
    hs = [W.random_small(700 + s, 15 + 7 * s, 60 + 40 * s, {2: 0.5, 3: 0.3, 4: 0.2}, allow_dups=True)
          for s in range(9)]
    n = len(hs)
    C = hm.hm_num_classes(4)
    out = torch.empty((n, C), dtype=torch.int64, device="cuda")
    mp, op = (ctypes.c_void_p * n)(), (ctypes.c_void_p * n)()
    ne, nm, nn = (ctypes.c_uint64 * n)(), (ctypes.c_uint64 * n)(), (ctypes.c_uint32 * n)()
    for g, h in enumerate(hs):
        mp[g], op[g] = h.members.ctypes.data, h.offsets.ctypes.data
        ne[g], nm[g], nn[g] = h.n_edges, len(h.members), h.n_nodes
    st = torch.cuda.current_stream()
    rc = hm.lib().count_exact_many(n, mp, op, ne, nm, nn, hm.binding.HM_MEM_HOST, 4, ctypes.c_void_p(out.data_ptr()),
                                   4, ctypes.c_void_p(st.cuda_stream))
    assert rc == 0, hm.lib().hm_last_error().decode()
    got = out.cpu().numpy()
    for g, h in enumerate(hs):
        assert np.array_equal(got[g], core.count_exact(h, 4)), g


def test_count_exact_many_repeats_the_duplicate_search(hm):
    """With no tag bits every build's one-launch duplicate search meets
    different hyperedges and is repeated exactly, here inside the worker
    threads of count_exact_many: the rows still equal the oracle's counts."""
    hs = [W.random_small(610 + s, 25 + 5 * s, 150 + 40 * s, {1: 0.05, 2: 0.5, 3: 0.3, 4: 0.15}, allow_dups=True)
          for s in range(6)]
    hm.hm_set_option(hm.HM_OPT_DEDUP_TAG_BITS, 0)
    try:
        got = hm.count_exact_many(_device_graphs(hs), 4, workers=3).cpu().numpy()
    finally:
        hm.hm_set_option(hm.HM_OPT_DEDUP_TAG_BITS, 32)
    for g, h in enumerate(hs):
        assert np.array_equal(got[g], core.count_exact(h, 4)), g
