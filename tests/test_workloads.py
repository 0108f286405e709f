"""The seeded generators are deterministic and give the stated shapes."""
import numpy as np

import workloads as W


def test_facetoface_k3_shape():
    h = W.cfg0_facetoface_k3(0)
    assert h.n_nodes == 200 and h.n_edges == 2000
    assert set(np.unique(h.sizes())) <= {2, 3, 4}
    assert int(h.members.max()) < 200
    h2 = W.cfg0_facetoface_k3(0)
    assert np.array_equal(h.members, h2.members) and np.array_equal(h.offsets, h2.offsets)


def test_facetoface_k4_shape():
    h = W.cfg1_facetoface_k4(0)
    assert h.n_nodes == 400 and h.n_edges == 30000
    assert set(np.unique(h.sizes())) == {2, 3, 4, 5}
    # members are distinct within each hyperedge and hyperedges are unique
    edges = [tuple(sorted(e)) for e in h.edges()]
    assert all(len(set(e)) == len(e) for e in edges)
    assert len(set(edges)) == len(edges)
    # community structure: most members share the hyperedge's majority block
    blocks = [np.bincount(np.array(e) // 40).max() / len(e) for e in edges]
    assert np.mean(blocks) > 0.85


def test_scaled_heavy_tailed_shape():
    h = W.scaled_coauthorship(0.01, seed=0)
    assert h.n_nodes == 10000
    s = h.sizes()
    assert s.min() >= 2 and s.max() <= 25
    deg = np.bincount(h.members.astype(np.int64), minlength=h.n_nodes)
    assert deg.max() > 20 * max(1.0, deg.mean())       # heavy tail


def test_subsample_keeps_id_space():
    h = W.cfg1_facetoface_k4(0)
    s = W.subsample_edges(h, 0.05, seed=1)
    assert s.n_nodes == h.n_nodes
    assert 0.03 * h.n_edges < s.n_edges < 0.07 * h.n_edges
