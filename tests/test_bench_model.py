"""The benchmark's count of memory transactions of the 3-node-hyperedge
fill-in step (the live lookup-bandwidth figure) against a per-hyperedge loop
that follows the same rules one entry at a time."""
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


def _loop_model(e2, e3, e4, n, hub_min_degree):
    run_max, q_max, adj_max = bench.SHORT_RUN, bench.SHORT_Q, bench.SHORT_ADJ
    adj = [set() for _ in range(n)]
    for x, y in e2.tolist():
        adj[x].add(y)
        adj[y].add(x)
    # dense rows: degree at least hub_min_degree, highest first (ties by id), within the budget
    cand = sorted((v for v in range(n) if hub_min_degree and len(adj[v]) >= hub_min_degree),
                  key=lambda v: (-len(adj[v]), v))
    hubs = set(cand[: bench.HUB_ROW_BYTES // (4 * ((n + 31) // 32))])

    def pair_cost(x):
        """(probes, streamed bytes) of one pair test against member x"""
        if len(adj[x]) <= adj_max:
            return 0, 0
        return (0, 4) if x in hubs else (1, 0)

    E3 = [tuple(t) for t in e3.tolist()]
    E4 = [tuple(f) for f in e4.tolist()]
    inc4 = [[f for f in E4 if v in f] for v in range(n)]
    run = {}
    for t in E3:
        for i in range(3):
            for j in range(i + 1, 3):
                run.setdefault((t[i], t[j]), []).append([u for u in t if u not in (t[i], t[j])][0])
    probes = stream = 0
    for a, b, c in E3:
        pab, pac, pbc = (int(len(run[p]) > run_max) for p in ((a, b), (a, c), (b, c)))
        (pa, sa), (pb, sb), (pc, sc) = (pair_cost(x) for x in (a, b, c))
        fa, fb, fc = len(inc4[a]), len(inc4[b]), len(inc4[c])
        l3 = fa if (fa <= fb and fa <= fc) else (fb if fb <= fc else fc)
        hold = sum(1 for f in E4 if {a, b, c} <= set(f))
        qp = 0 if (l3 <= 64 and hold <= q_max) else 1
        da, db, dc = len(adj[a]), len(adj[b]), len(adj[c])
        dmin = min(da, db, dc)
        # the shortest row walked against the other two members
        others = (b, c) if (da <= db and da <= dc) else ((a, c) if db <= dc else (a, b))
        probes += 7
        for x in others:
            if x in hubs:
                stream += 4 * dmin
            else:
                probes += dmin
        stream += 4 * dmin + 60 + 20 * l3 + (20 * l3 if l3 <= 64 else 0)
        stream += sum(4 * len(adj[x]) for x in (a, b, c) if len(adj[x]) <= adj_max)
        for (x, y), m, slot in (((a, b), c, 0), ((a, c), b, 1), ((b, c), a, 2)):
            L = len(run[(x, y)])
            stream += 5 * L + (4 * L if L <= run_max else 0)
            pm, sm = ((pc, sc), (pb, sb), (pa, sa))[slot]
            for w in run[(x, y)]:
                if w == m:
                    continue
                stream += sm
                if w > m:
                    probes += (pac + pbc, pab + pbc, pab + pac)[slot] + qp + pm
                else:
                    probes += (0, pab, pab + pac)[slot] + pm
        probes += hold * (pab + pac + pbc + pa + pb + pc)
        stream += hold * (sa + sb + sc)
    return probes, stream


@pytest.mark.parametrize("hub_min_degree", [0, 20, 70])
@pytest.mark.parametrize("seed,n,sizes", [(5, 60, (200, 400, 200)), (7, 120, (900, 700, 500)), (9, 16, (40, 150, 80))])
def test_b4_lookup_model_matches_loop(seed, n, sizes, hub_min_degree):
    e2, e3, e4 = _hub_strata(seed, n, *sizes)
    m = bench._b4_lookup_model(e2, e3, e4, n, hub_min_degree)
    probes, stream = _loop_model(e2, e3, e4, n, hub_min_degree)
    assert (m["probes"], m["stream_bytes"]) == (probes, stream)
