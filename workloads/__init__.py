"""Seeded synthetic hypergraph generators.

These generators are the only code shared between the product path and the
oracle.  They draw hyperedge lists and nothing else: no motif arithmetic lives
here.  Each generator returns a :class:`Hypergraph` in the boundary's layout
(``members`` uint32, ``offsets`` uint64 with ``offsets[0] == 0``), with members
of a hyperedge in draw order (unsorted), so that ingest's normalisation is
exercised.

The workloads stand in for the paper's datasets (Section 6.1, Table 1), which
are not available: face-to-face-shaped (dense, few nodes, many small
hyperedges, community structure), co-authorship-shaped (a million nodes,
heavy-tailed node weights, heavy-tailed sizes) and communication-shaped
(fewer nodes, very heavy-tailed weights, large hyperedges).
"""
from .synth import (  # noqa: F401
    Hypergraph,
    from_lists,
    random_small,
    cfg0_facetoface_k3,
    cfg1_facetoface_k4,
    cfg3_coauthorship,
    cfg4_communication,
    scaled_coauthorship,
    scaled_communication,
    subsample_edges,
    WORKLOADS,
)
