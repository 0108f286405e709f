"""Deterministic hypergraph generators (numpy PCG64, fixed seeds).

Recipes (sizes, distributions and structure) follow the workload shapes the
paper measures on (Section 6.1, Table 1): face-to-face proximity networks
(few hundred nodes, mostly pairs, strong community structure), co-authorship
networks (about a million nodes, heavy-tailed activity, papers of 2..25
authors) and e-mail networks (heavy-tailed activity, large recipient lists).

Members of a hyperedge are drawn without replacement by redrawing duplicates
from the same distribution until the hyperedge has distinct nodes.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Hypergraph", "from_lists", "random_small", "cfg0_facetoface_k3",
    "cfg1_facetoface_k4", "cfg3_coauthorship", "cfg4_communication",
    "scaled_coauthorship", "scaled_communication", "subsample_edges", "WORKLOADS",
]


@dataclass
class Hypergraph:
    """A hyperedge list in CSR form: hyperedge i is ``members[offsets[i]:offsets[i+1]]``."""

    n_nodes: int
    members: np.ndarray          # uint32[nnz]
    offsets: np.ndarray          # uint64[E+1]
    name: str = ""
    meta: dict = field(default_factory=dict)

    def __post_init__(self):
        self.members = np.ascontiguousarray(self.members, dtype=np.uint32)
        self.offsets = np.ascontiguousarray(self.offsets, dtype=np.uint64)

    @property
    def n_edges(self) -> int:
        return len(self.offsets) - 1

    def sizes(self) -> np.ndarray:
        return np.diff(self.offsets.astype(np.int64))

    def edges(self):
        off = self.offsets.astype(np.int64)
        m = self.members
        return [m[off[i]:off[i + 1]].tolist() for i in range(len(off) - 1)]


def from_lists(edges, n_nodes: int | None = None, name: str = "") -> Hypergraph:
    edges = [list(map(int, e)) for e in edges]
    sizes = np.array([len(e) for e in edges], dtype=np.int64)
    offsets = np.zeros(len(edges) + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum(sizes)
    members = np.array([v for e in edges for v in e], dtype=np.uint32)
    if n_nodes is None:
        n_nodes = int(members.max()) + 1 if len(members) else 0
    return Hypergraph(n_nodes, members, offsets, name=name)


def _redraw_duplicates(rng, members, seg, redraw):
    """Redraw, in place, every member that repeats an earlier member of its hyperedge.

    Each pass looks only at positions of hyperedges that still held a repeat.
    """
    active = np.arange(len(members))
    for _ in range(10_000):
        order = active[np.lexsort((members[active], seg[active]))]
        ms, ss = members[order], seg[order]
        dup = (ms[1:] == ms[:-1]) & (ss[1:] == ss[:-1])
        if not dup.any():
            return members
        pos = order[1:][dup]
        members[pos] = redraw(rng, pos)
        bad = np.unique(seg[pos])
        active = active[np.isin(seg[active], bad)]
    raise RuntimeError("duplicate redraw did not converge")


def _cdf_sampler(weights):
    cdf = np.cumsum(weights, dtype=np.float64)
    cdf /= cdf[-1]
    n = len(weights)

    def draw(rng, count):
        u = rng.random(count)
        return np.minimum(np.searchsorted(cdf, u, side="right"), n - 1).astype(np.int64)
    return draw


def _draw_edges(rng, sizes, draw_at):
    """Draw members for hyperedges of the given sizes; draw_at(rng, positions, seg) -> nodes."""
    sizes = np.asarray(sizes, dtype=np.int64)
    seg = np.repeat(np.arange(len(sizes)), sizes)
    pos = np.arange(len(seg))
    members = draw_at(rng, pos, seg)
    members = _redraw_duplicates(rng, members, seg, lambda r, p: draw_at(r, p, seg[p]))
    offsets = np.zeros(len(sizes) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    return members, offsets


def _until_unique(rng, target, batch, draw_batch):
    """Draw hyperedges in batches, keep first occurrences, stop at ``target`` unique ones."""
    seen = set()
    out = []
    while len(out) < target:
        members, offsets = draw_batch(rng, batch)
        for i in range(len(offsets) - 1):
            e = members[offsets[i]:offsets[i + 1]]
            key = tuple(sorted(e.tolist()))
            if key in seen:
                continue
            seen.add(key)
            out.append(e.tolist())
            if len(out) == target:
                break
    return out


def _dedup_after(members, offsets):
    """Drop repeated hyperedges (as node sets), keeping first occurrences in draw order."""
    sizes = np.diff(offsets)
    keep = np.zeros(len(sizes), dtype=bool)
    for s in np.unique(sizes):
        idx = np.nonzero(sizes == s)[0]
        rows = members[offsets[idx][:, None] + np.arange(s)[None, :]]
        rows = np.sort(rows, axis=1)
        _, first = np.unique(rows, axis=0, return_index=True)
        keep[idx[first]] = True
    kept = np.nonzero(keep)[0]
    new_sizes = sizes[kept]
    new_off = np.zeros(len(kept) + 1, dtype=np.int64)
    new_off[1:] = np.cumsum(new_sizes)
    seg = np.repeat(kept, new_sizes)
    within = np.arange(len(seg)) - np.repeat(new_off[:-1], new_sizes)
    gather = offsets[seg] + within
    return members[gather], new_off


def random_small(seed: int, n_nodes: int, n_edges: int, size_probs: dict, allow_dups: bool = False,
                 name: str = "") -> Hypergraph:
    """Tiny random hypergraph with uniformly drawn members.

    ``size_probs`` maps hyperedge size (may include 1 or sizes above the motif
    order) to probability.  With ``allow_dups`` repeated hyperedges are kept in
    the list (ingest must collapse them).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes_v = np.array(sorted(size_probs), dtype=np.int64)
    p = np.array([size_probs[s] for s in sizes_v], dtype=np.float64)
    p /= p.sum()
    sizes = rng.choice(sizes_v, size=n_edges, p=p)
    sizes = np.minimum(sizes, n_nodes)
    members, offsets = _draw_edges(rng, sizes, lambda r, pos, seg: r.integers(0, n_nodes, len(pos)))
    if not allow_dups:
        members, offsets = _dedup_after(members, offsets)
    return Hypergraph(n_nodes, members.astype(np.uint32), offsets.astype(np.uint64),
                      name=name or f"random_small(seed={seed},N={n_nodes},E={n_edges})")


def cfg0_facetoface_k3(seed: int = 0) -> Hypergraph:
    """CPU-sized order-3 workload: N=200, 2,000 unique hyperedges, sizes 2/3/4 w.p. .70/.25/.05,
    node r (1-based rank) drawn with weight r^-0.8."""
    n, target = 200, 2000
    rng = np.random.Generator(np.random.PCG64(seed))
    draw_node = _cdf_sampler(np.arange(1, n + 1, dtype=np.float64) ** -0.8)

    def batch(r, count):
        sizes = r.choice(np.array([2, 3, 4]), size=count, p=[0.70, 0.25, 0.05])
        return _draw_edges(r, sizes, lambda rr, pos, seg: draw_node(rr, len(pos)))
    edges = _until_unique(rng, target, 512, batch)
    h = from_lists(edges, n, name="facetoface_N200_E2000")
    h.meta.update(seed=seed, recipe="cfg0")
    return h


def cfg1_facetoface_k4(seed: int = 0) -> Hypergraph:
    """Order-4 face-to-face workload: N=400 in 10 communities of 40 (community(v)=v//40),
    30,000 unique hyperedges, size s in 2..5 with P(s) ~ 0.4^(s-2); each hyperedge picks a
    community uniformly and each member comes from it w.p. 0.9, else uniformly from all nodes."""
    n, target, ncomm, csize = 400, 30000, 10, 40
    rng = np.random.Generator(np.random.PCG64(seed))
    svals = np.arange(2, 6)
    sp = 0.4 ** (svals - 2)
    sp /= sp.sum()

    def batch(r, count):
        sizes = r.choice(svals, size=count, p=sp)
        comm = r.integers(0, ncomm, count)

        def draw_at(rr, pos, seg):
            inside = rr.random(len(pos)) < 0.9
            local = rr.integers(0, csize, len(pos)) + comm[seg] * csize
            anywhere = rr.integers(0, n, len(pos))
            return np.where(inside, local, anywhere)
        return _draw_edges(r, sizes, draw_at)
    edges = _until_unique(rng, target, 4096, batch)
    h = from_lists(edges, n, name="facetoface_N400_E30000")
    h.meta.update(seed=seed, recipe="cfg1")
    return h


def _heavy_tailed(seed, n, n_draws, alpha, smax, size_exp, name, dedup=True):
    rng = np.random.Generator(np.random.PCG64(seed))
    u = 1.0 - rng.random(n)                      # in (0, 1]
    weights = u ** (-1.0 / alpha)                # Pareto(alpha) by inverse CDF (scale cancels)
    draw_node = _cdf_sampler(weights)
    svals = np.arange(2, smax + 1)
    sp = svals.astype(np.float64) ** (-size_exp)
    sp /= sp.sum()
    sizes = rng.choice(svals, size=n_draws, p=sp)
    members, offsets = _draw_edges(rng, sizes, lambda r, pos, seg: draw_node(r, len(pos)))
    if dedup:
        members, offsets = _dedup_after(members, offsets)
    h = Hypergraph(n, members.astype(np.uint32), offsets.astype(np.uint64), name=name)
    h.meta.update(seed=seed, draws=n_draws, alpha=alpha)
    return h


def cfg3_coauthorship(seed: int = 0, dedup: bool = True) -> Hypergraph:
    """Co-authorship-shaped: N=1,000,000, 2,000,000 draws (deduplicated after drawing),
    size s in 2..25 with P(s) ~ s^-2.5, node weights ~ Pareto(alpha=1.2)."""
    return _heavy_tailed(seed, 1_000_000, 2_000_000, 1.2, 25, 2.5, "coauthorship_N1e6_E2e6", dedup)


def cfg4_communication(seed: int = 0, dedup: bool = True) -> Hypergraph:
    """Communication-shaped: N=50,000, 5,000,000 draws (deduplicated after drawing),
    size s in 2..50 with P(s) ~ s^-2, node weights ~ Pareto(alpha=1.0)."""
    return _heavy_tailed(seed, 50_000, 5_000_000, 1.0, 50, 2.0, "communication_N5e4_E5e6", dedup)


def scaled_coauthorship(scale: float, seed: int = 0) -> Hypergraph:
    """The co-authorship recipe with N and the number of draws multiplied by ``scale``."""
    n = max(50, int(1_000_000 * scale))
    d = max(50, int(2_000_000 * scale))
    return _heavy_tailed(seed, n, d, 1.2, 25, 2.5, f"coauthorship_scaled_{scale:g}")


def scaled_communication(scale: float, seed: int = 0) -> Hypergraph:
    """The communication recipe with N and the number of draws multiplied by ``scale``."""
    n = max(50, int(50_000 * scale))
    d = max(50, int(5_000_000 * scale))
    return _heavy_tailed(seed, n, d, 1.0, 50, 2.0, f"communication_scaled_{scale:g}")


def subsample_edges(h: Hypergraph, p: float, seed: int) -> Hypergraph:
    """Keep each hyperedge independently with probability p (same node id space)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    keep = np.nonzero(rng.random(h.n_edges) < p)[0]
    off = h.offsets.astype(np.int64)
    sizes = off[keep + 1] - off[keep]
    new_off = np.zeros(len(keep) + 1, dtype=np.int64)
    new_off[1:] = np.cumsum(sizes)
    seg = np.repeat(keep, sizes)
    within = np.arange(len(seg)) - np.repeat(new_off[:-1], sizes)
    members = h.members[off[seg] + within]
    out = Hypergraph(h.n_nodes, members, new_off.astype(np.uint64), name=f"{h.name}_sub{p:g}")
    out.meta.update(parent=h.name, p=p, seed=seed)
    return out


WORKLOADS = {
    "facetoface_N200_E2000": cfg0_facetoface_k3,
    "facetoface_N400_E30000": cfg1_facetoface_k4,
    "coauthorship_N1e6_E2e6": cfg3_coauthorship,
    "communication_N5e4_E5e6": cfg4_communication,
}
