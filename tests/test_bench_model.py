"""The benchmark's count of the positions the 3-node-hyperedge step without
bit rows walks (k_sp_b4 and k_sp_b4_runs), against a loop that follows the
kernels' rules one hyperedge and one index entry at a time."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def _hub_strata(seed, n, m2, m3, m4):
    rng = np.random.default_rng(seed)

    def draw(k, m, p):
        s = set()
        while len(s) < m:
            if rng.random() < p:
                base = [0, 1] if k >= 3 else [0]
                rest = rng.choice(np.arange(2, n), k - len(base), replace=False).tolist()
                s.add(tuple(sorted(base + rest)))
            else:
                s.add(tuple(sorted(rng.choice(n, k, replace=False).tolist())))
        return np.array(sorted(s), dtype=np.uint32)

    return draw(2, m2, 0.5), draw(3, m3, 0.5), draw(4, m4, 0.3)


def _loop_positions(e2, e3, e4, n):
    adj = [set() for _ in range(n)]
    for x, y in e2.tolist():
        adj[x].add(y)
        adj[y].add(x)
    E3 = [tuple(t) for t in e3.tolist()]
    E4 = [set(f) for f in e4.tolist()]
    run = {}
    for t in E3:
        for i in range(3):
            for j in range(i + 1, 3):
                run.setdefault((t[i], t[j]), []).append(t[3 - i - j])

    def L(x, y):
        return len(run.get((min(x, y), max(x, y)), []))

    b4 = runs = active = 0
    for e in E3:
        hold = sum(1 for f in E4 if set(e) <= f)
        b4 += min(len(adj[v]) for v in e) + hold
        for i, j in ((0, 1), (0, 2), (1, 2)):
            p0, p1, t = e[i], e[j], e[3 - i - j]
            n_run = L(p0, p1)
            if n_run < 2:
                continue
            active += 1
            listed = len(adj[t]) + L(p0, t) + L(p1, t) + hold
            runs += n_run - 1 if n_run - 1 <= listed else listed
    return b4, runs, active


@pytest.mark.parametrize("seed,n,sizes", [(5, 60, (200, 400, 200)), (7, 120, (900, 700, 500)), (9, 16, (40, 150, 80))])
def test_b4_positions_match_loop(seed, n, sizes):
    e2, e3, e4 = _hub_strata(seed, n, *sizes)
    m = bench._b4_positions(e2, e3, e4, n)
    assert (m["positions_b4"], m["positions_runs"], m["entries_active"]) == _loop_positions(e2, e3, e4, n)
    assert m["hyperedges"] == len(e3) and m["entries"] == 3 * len(e3)


def test_b4_positions_empty():
    e = np.zeros((0, 3), np.uint32)
    assert bench._b4_positions(np.zeros((0, 2), np.uint32), e, np.zeros((0, 4), np.uint32), 10)["positions_b4"] == 0
