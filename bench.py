#!/usr/bin/env python3
"""Order-4 motif count time per hypergraph on the face-to-face workload
(N=400 nodes in 10 communities, 30,000 unique hyperedges of sizes 2..5, k=4).

One step = build the device hypergraph from the raw hyperedge list already
resident in HBM (validate, sort, collapse repeats, hash sets, adjacency) and
count every order-4 motif exactly.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "order-4 motif count time per hypergraph; sampled speedup at ≤2% mean rel err"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_exact_k4_facetoface_N400_E30000.md")
# sources the exact counting kernels are compiled from: HBM traffic measured with
# hardware counters is only reported while these are unchanged
EXACT_SOURCES = ("exact.hip", "hm_items.h", "hm_b4.h", "hm_device.h", "hm_internal.h")
HBM_PEAK_GBS = 8000.0
# integer VALU issue rate: 256 CUs x 64 lanes per cycle x 2.4 GHz
# worker threads (one stream each) of the count_exact_many call that the
# headline measurement makes: 3 gave 36 us per hypergraph, 7 or 8 about 31.5,
# 10 to 16 no better
PIPELINE = 8
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12


def _unit_counts(e2: np.ndarray, e3: np.ndarray, n_nodes: int, words: int) -> dict:
    """Work units of each counting kernel, from the exported strata."""
    n = n_nodes
    rows = [[] for _ in range(n)]
    for a, b in e2.tolist():
        rows[a].append(b)
        rows[b].append(a)
    rows = [np.array(sorted(r), dtype=np.int64) for r in rows]
    deg2 = np.array([len(r) for r in rows], dtype=np.int64)
    deg3 = np.bincount(e3.reshape(-1).astype(np.int64), minlength=n) if len(e3) else np.zeros(n, np.int64)
    # pairs-only shapes: (pair {r<x}) x (y in N(r) above x, and y in N(x) above r) x words
    ys = 0
    for r, x in e2.tolist():
        ys += len(rows[r]) - np.searchsorted(rows[r], x, side="right")
        ys += len(rows[x]) - np.searchsorted(rows[x], r, side="right")
    # 3-node generators: every pairwise neighbour of a, b, c and every incident 3-node
    # hyperedge of a and b
    cand = 0
    if len(e3):
        t = e3.astype(np.int64)
        cand = int(deg2[t[:, 0]].sum() + deg2[t[:, 1]].sum() + deg2[t[:, 2]].sum()
                   + deg3[t[:, 0]].sum() + deg3[t[:, 1]].sum())
    # case (c) by graph identities: per pair of G2 its W common-neighbour words
    # and, per common neighbour above the pair, W words of edges among them;
    # per node pair u < w its W codegree words
    above = 0
    for r, x in e2.tolist():
        i = np.searchsorted(rows[r], x, side="right")
        above += len(np.intersect1d(rows[r][i:], rows[x], assume_unique=True))
    return {"c4_word_tasks": int(ys) * words, "b4_word_tasks": int(len(e3)) * words, "b4_candidates": cand,
            "id_edge_word_tasks": int(len(e2)) * words, "id_k4_word_tasks": int(above) * words,
            "id_c4_pair_word_tasks": n * (n - 1) // 2 * words}


def _b4_positions(e2: np.ndarray, e3: np.ndarray, e4: np.ndarray, n_nodes: int) -> dict:
    """Work of the 3-node-hyperedge step without bit rows, counted from the
    strata as its two kernels walk it.  k_sp_b4, per 3-node hyperedge
    e = {a<b<c}: the shortest pairwise row among a, b, c (each entry tested
    against the other two members) and the 4-node hyperedges holding e.
    k_sp_b4_runs, per entry of the pair index (a pair P of e with the third
    node t) whose run holds L >= 2 entries: the other L - 1 entries of the
    run when L - 1 <= d(t) + L(P0, t) + L(P1, t) + (4-node hyperedges holding
    e), else those lists.  Each position is a few lookups (a third node, a
    membership test against a list in LDS, a dense-row word or a hash probe)."""
    n = np.int64(n_nodes)
    if len(e3) == 0:
        return {"positions_b4": 0, "positions_runs": 0, "hyperedges": 0, "entries": 0, "entries_active": 0}
    deg2 = np.bincount(e2.reshape(-1).astype(np.int64), minlength=n_nodes) if len(e2) else np.zeros(n_nodes, np.int64)
    t = e3.astype(np.int64)
    a, b, c = t[:, 0], t[:, 1], t[:, 2]
    dmin = np.minimum(np.minimum(deg2[a], deg2[b]), deg2[c])
    if len(e4):
        q = e4.astype(np.int64)
        sub = np.concatenate([(q[:, i] * n + q[:, j]) * n + q[:, k]
                              for i, j, k in ((0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3))])
        su, sc = np.unique(sub, return_counts=True)
        k3 = (a * n + b) * n + c
        pos = np.minimum(np.searchsorted(su, k3), len(su) - 1)
        holding = np.where(su[pos] == k3, sc[pos], 0)
    else:
        holding = np.zeros(len(t), np.int64)
    pk = np.concatenate([a * n + b, a * n + c, b * n + c])
    uk, cnt = np.unique(pk, return_counts=True)

    def run_len(x, y):
        k = np.minimum(x, y) * n + np.maximum(x, y)
        i = np.minimum(np.searchsorted(uk, k), len(uk) - 1)
        return np.where(uk[i] == k, cnt[i], 0)

    runs = 0
    active = 0
    for p0, p1, th in ((a, b, c), (a, c, b), (b, c, a)):
        L = run_len(p0, p1)
        listed = deg2[th] + run_len(p0, th) + run_len(p1, th) + holding
        on = L >= 2
        active += int(on.sum())
        runs += int(np.where(on, np.where(L - 1 <= listed, L - 1, listed), 0).sum())
    return {"positions_b4": int((dmin + holding).sum()), "positions_runs": runs, "hyperedges": int(len(t)),
            "entries": 3 * int(len(t)), "entries_active": active}


def exact_source_digest() -> str:
    import hashlib
    d = hashlib.sha256()
    for name in EXACT_SOURCES:
        with open(os.path.join(ROOT, "paper_2209_10241_amd", "csrc", name), "rb") as f:
            d.update(f.read())
    return d.hexdigest()[:16]


def measured_traffic() -> dict:
    """Per-launch HBM bytes (FETCH_SIZE + WRITE_SIZE, copy-calibrated) by kernel, if still current."""
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return {}
    digest = next((l.split("`")[1] for l in lines if l.startswith("source digest:")), None)
    if digest != exact_source_digest():
        return {}
    out = {}
    for l in lines:
        cols = [c.strip() for c in l.strip().strip("|").split("|")]
        if len(cols) == 6 and cols[0].startswith("k_") and cols[5].replace(".", "").isdigit():
            out[cols[0].split("<")[0]] = float(cols[5])
    return out


VALU_FILE = os.path.join(ROOT, "profiles", "valu_issue_k_exact4_bits_facetoface_N400_E30000.md")


def measured_valu_issue():
    """Fraction of the chip's VALU issue rate k_exact4_bits used (SQ_INSTS_VALU over
    its trace duration, from the committed counter profile), if still current."""
    try:
        lines = open(VALU_FILE).read().splitlines()
    except OSError:
        return None
    digest = next((l.split("`")[1] for l in lines if l.startswith("source digest:")), None)
    frac = next((l.split("`")[1] for l in lines if l.startswith("VALU issue fraction:")), None)
    if digest != exact_source_digest() or frac is None:
        return None
    return float(frac)


LOOKUP_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_lookup_k_sp_b4_heavy_tailed.md")
LOOKUP_SOURCES = ("sparse.hip", "hm_sparse.h", "hm_device.h", "hm_internal.h", "prims.hip")


def lookup_source_digest() -> str:
    import hashlib
    d = hashlib.sha256()
    for name in LOOKUP_SOURCES:
        with open(os.path.join(ROOT, "paper_2209_10241_amd", "csrc", name), "rb") as f:
            d.update(f.read())
    return d.hexdigest()[:16]


def measured_lookup_traffic() -> dict:
    """HBM bytes per count of k_sp_b4 plus k_sp_b4_runs (FETCH_SIZE + WRITE_SIZE,
    copy-calibrated) by workload, if the profile is still current."""
    try:
        lines = open(LOOKUP_TRAFFIC_FILE).read().splitlines()
    except OSError:
        return {}
    digest = next((l.split("`")[1] for l in lines if l.startswith("source digest:")), None)
    if digest != lookup_source_digest():
        return {}
    out = {}
    for l in lines:
        cols = [c.strip() for c in l.strip().strip("|").split("|")]
        if len(cols) == 4 and cols[0] in ("coauthorship_N1e6_E2e6", "communication_N5e4_E5e6") \
                and cols[3].replace(".", "").isdigit():
            out[cols[0]] = float(cols[3])
    return out


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def _mre(runs, exact) -> float:
    r = np.asarray(runs, dtype=np.float64)
    return float(np.mean(np.abs(r - exact).sum(axis=1) / exact.sum()))


def large_workloads(hm, W, torch, seeds: int = 32, exact_only: bool = False) -> dict:
    """Exact order-4 counts and sampled estimates (uniform, and the learned
    proposal trained on a 5% hyperedge subsample) on the heavy-tailed
    workloads; with exact_only, the exact counts and their lookup figures."""
    out = {}
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, reps):
        ev0.record(stream)
        res = [fn(i) for i in range(reps)]
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / reps, res

    for name, maker in (("coauthorship_N1e6_E2e6", W.cfg3_coauthorship), ("communication_N5e4_E5e6", W.cfg4_communication)):
        h = maker(0)
        dev = torch.device("cuda:0")
        members = torch.from_numpy(h.members.astype(np.int32)).to(dev)
        offsets = torch.from_numpy(h.offsets.astype(np.int64)).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = hm.hm_graph_create(members, offsets, h.n_nodes, stream=stream)
        torch.cuda.synchronize()
        ingest_ms = (time.perf_counter() - t0) * 1e3
        st = g.stats()
        hm.count_exact(g, 4, stream=stream)
        exact_ms, res = timed(lambda i: hm.count_exact(g, 4, stream=stream), 3)
        exact = res[-1].cpu().numpy().astype(np.float64)
        # the fill-in step of 3-node neighbourhoods, timed live with HIP events
        # on the counting stream; effective lookup bandwidth at 64 B per probe
        hm.hm_profile_reset()
        hm.hm_profile_enable(True)
        for _ in range(3):
            hm.count_exact(g, 4, stream=stream)
        torch.cuda.synchronize()
        prof = hm.hm_profile_read()
        hm.hm_profile_enable(False)
        kernels = {k: {"launches": n, "avg_ms": ms / max(n, 1)} for k, (n, ms) in prof.items()}
        model = _b4_positions(g.export(2), g.export(3), g.export(4), h.n_nodes)
        lookup = None
        if "k_sp_b4" in kernels and "k_sp_b4_runs" in kernels:
            ms = kernels["k_sp_b4"]["avg_ms"] + kernels["k_sp_b4_runs"]["avg_ms"]
            lookup = {"kernels": ["k_sp_b4", "k_sp_b4_runs"], "ms": ms,
                      "positions_per_s": (model["positions_b4"] + model["positions_runs"]) / (ms / 1e3), **model}
            # HBM bytes of the two kernels from the committed counter runs
            # (FETCH_SIZE + WRITE_SIZE per launch), while the sources match
            meas = measured_lookup_traffic().get(name)
            if meas:
                gbs = meas / (ms / 1e3) / 1e9
                lookup.update({"bound": "latency", "traffic": meas, "achieved": gbs, "peak": HBM_PEAK_GBS,
                               "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS})
            else:
                lookup.update({"bound": "latency", "traffic": None, "achieved": None, "peak": HBM_PEAK_GBS,
                               "unit": "GB/s", "frac": None})
        if exact_only:
            out[name] = {"n_nodes": h.n_nodes, "unique_by_size": [st["n2"], st["n3"], st["n4"], st["n5plus"]],
                         "connected_4_sets": int(exact.sum()), "ingest_ms": ingest_ms, "exact_ms": exact_ms,
                         "exact_kernels": kernels, "lookup_roofline": lookup}
            g.close()
            del members, offsets
            torch.cuda.empty_cache()
            continue
        h5 = W.subsample_edges(h, 0.05, seed=3)
        g5 = hm.hm_graph_create(h5.members, h5.offsets, h5.n_nodes, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        model = hm.hm_model_train(g5, 4, epochs=30, batch=4096, lr=3e-3, seed=2)
        torch.cuda.synchronize()
        train_ms = (time.perf_counter() - t0) * 1e3
        t0 = time.perf_counter()
        hm.count_sampled(g, 4, 0.01, 7, stream=stream)
        torch.cuda.synchronize()
        first_uniform_ms = (time.perf_counter() - t0) * 1e3
        t0 = time.perf_counter()
        hm.count_sampled_learned(g, model, 4, 0.01, 7, stream=stream)
        torch.cuda.synchronize()
        first_learned_ms = (time.perf_counter() - t0) * 1e3
        rows = {}
        for f in (0.0007, 0.001, 0.0015, 0.0025, 0.005, 0.01, 0.02, 0.05, 0.1):
            ms_u, ru = timed(lambda i: hm.count_sampled(g, 4, f, 1000 + i, stream=stream)[0], seeds)
            ms_l, rl = timed(lambda i: hm.count_sampled_learned(g, model, 4, f, 1000 + i, stream=stream)[0], seeds)
            rows[f"{f:g}"] = {
                "uniform": {"ms": ms_u, "mre": _mre(torch.stack(ru).cpu().numpy(), exact), "speedup_vs_exact": exact_ms / ms_u},
                "learned": {"ms": ms_l, "mre": _mre(torch.stack(rl).cpu().numpy(), exact), "speedup_vs_exact": exact_ms / ms_l},
            }

        def best(kind):
            ok = [(v[kind]["ms"], k) for k, v in rows.items() if v[kind]["mre"] <= 0.02]
            if not ok:
                return None
            ms, k = min(ok)
            return {"fraction": float(k), "ms": ms, "mre": rows[k][kind]["mre"], "speedup_vs_exact": exact_ms / ms}

        fastest = {"uniform": best("uniform"), "learned": best("learned")}
        amortised = None
        if fastest["learned"]:
            lm = fastest["learned"]["ms"]
            # training once, then n estimates: (train + n * learned) against n exact counts
            amortised = {"training_ms": train_ms, "learned_ms_per_estimate": lm,
                         "speedup_vs_exact_incl_training_1_estimate": exact_ms / (train_ms + lm),
                         "speedup_vs_exact_incl_training_100_estimates": 100 * exact_ms / (train_ms + 100 * lm),
                         "estimates_to_amortise_training": (train_ms / (exact_ms - lm)) if exact_ms > lm else None}
            if fastest["uniform"]:
                um = fastest["uniform"]["ms"]
                amortised["estimates_before_learned_beats_uniform"] = (train_ms / (um - lm)) if um > lm else None
        out[name] = {
            "n_nodes": h.n_nodes, "unique_by_size": [st["n2"], st["n3"], st["n4"], st["n5plus"]],
            "connected_4_sets": int(exact.sum()), "ingest_ms": ingest_ms, "exact_ms": exact_ms,
            "learned_incl_training": amortised,
            "first_call_ms": {"uniform_1pct_incl_index_build": first_uniform_ms,
                              "learned_1pct_incl_proposal": first_learned_ms},
            "learned_training_ms": train_ms, "training_set": "5% hyperedge subsample",
            "exact_kernels": kernels, "lookup_roofline": lookup,
            "sampled": rows, "fastest_at_2pct_mre": fastest,
            "seeds": seeds,
        }
        model.close()
        g5.close()
        g.close()
        del members, offsets
        torch.cuda.empty_cache()
    return out


def order5_leg(hm, W, stream):
    """Order 5 (Section 6.4 samples at order 5) on the communication recipe
    at 0.004 of its size (N=200, hyperedges of sizes 2..5: a pair sample
    enumerates about 10^6 candidate sets, the dense face-to-face graph 10^7):
    the exact counts from the census (every hyperedge of size 2..5 drawn once,
    whose estimate is the exact count of every class), then sampled estimates
    at 1, 5 and 10% of every stratum over 16 seeds, with the mean relative
    error of the order-4 rows."""
    h5 = W.scaled_communication(0.004)
    g5 = hm.hm_graph_create(h5.members, h5.offsets, h5.n_nodes, stream=stream)
    sizes5 = hm.hm_order5_sizes(g5, stream=stream)
    everyone = {j: np.arange(sizes5[j]) for j in (2, 3, 4, 5)}
    hm.count_sampled5(g5, 0.01, 999, stream=stream)   # untimed: first-call set-up
    t0 = time.perf_counter()
    c_can, _, c_est = hm.count_sampled5_indices(g5, everyone, stream=stream)
    census_ms = (time.perf_counter() - t0) * 1e3
    exact5 = dict(zip(c_can.tolist(), c_est.astype(np.float64).tolist()))
    total5 = sum(exact5.values())
    rows5 = {}
    for f in (0.01, 0.05, 0.10):
        outs = []
        t0 = time.perf_counter()
        for seed in range(16):
            can, _, est = hm.count_sampled5(g5, f, 2000 + seed, stream=stream)
            outs.append(dict(zip(can.tolist(), est.astype(np.float64).tolist())))
        ms5 = (time.perf_counter() - t0) * 1e3 / 16
        errs = []
        for got in outs:
            keys = set(exact5) | set(got)
            errs.append(sum(abs(got.get(c, 0.0) - exact5.get(c, 0.0)) for c in keys) / total5)
        rows5[f"{f:g}"] = {"ms": ms5, "mre": float(np.mean(errs)), "speedup_vs_census": census_ms / ms5}
    g5.close()
    order5 = {"workload": "communication_scaled_0.004_N200", "classes": len(exact5),
              "connected_5_sets": total5, "census_ms": census_ms, "hyperedges_by_size": sizes5,
              "sampled": rows5, "timing": "host clock per call, results copied back"}
    return order5


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--exact-only", action="store_true", help="skip the sampled and null-model measurements")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the co-authorship and communication workloads (exact, uniform and learned sampling)")
    ap.add_argument("--lookup-only", action="store_true",
                    help="only the exact counts of the co-authorship and communication workloads and their "
                         "lookup-bandwidth figures (one JSON line)")
    ap.add_argument("--learned-only", action="store_true",
                    help="only train the learned proposal on the communication workload's 5%% subsample and draw "
                         "8 learned estimates at 0.15%% (for a kernel trace of the learned path)")
    ap.add_argument("--order5-only", action="store_true",
                    help="only the order-5 leg (census and sampled estimates), for profiling")
    ap.add_argument("--nulls-only", action="store_true",
                    help="only the 64-copy stub-matching null batch of the face-to-face workload: the first call "
                         "(tuning and capture) and 5 replays (for a kernel trace of the null pipeline)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 256 MiB device to device (a kernel of known traffic for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the counting path runs on a single MI355X "
              "(sharding across GPUs is designed but not built)", file=sys.stderr)
        return 2

    import torch
    import paper_2209_10241_amd as hm
    import workloads as W

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.learned_only:
        h = W.cfg4_communication(0)
        stream = torch.cuda.current_stream()
        g = hm.hm_graph_create(h.members, h.offsets, h.n_nodes, stream=stream)
        h5 = W.subsample_edges(h, 0.05, seed=3)
        g5 = hm.hm_graph_create(h5.members, h5.offsets, h5.n_nodes, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        model = hm.hm_model_train(g5, 4, epochs=30, batch=4096, lr=3e-3, seed=2)
        torch.cuda.synchronize()
        train_ms = (time.perf_counter() - t0) * 1e3
        hm.count_sampled_learned(g, model, 4, 0.0015, 7, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(8):
            hm.count_sampled_learned(g, model, 4, 0.0015, 100 + i, stream=stream)
        torch.cuda.synchronize()
        print(json.dumps({"learned_only": {"training_ms": train_ms,
                                           "ms_per_estimate": (time.perf_counter() - t0) * 1e3 / 8}}))
        return 0
    if args.lookup_only:
        print(json.dumps({"large_workloads": large_workloads(hm, W, torch, exact_only=True)}))
        return 0
    if args.order5_only:
        print(json.dumps({"order5": order5_leg(hm, W, torch.cuda.current_stream())}))
        return 0
    if args.nulls_only:
        h = W.cfg1_facetoface_k4(0)
        stream = torch.cuda.current_stream()
        g = hm.hm_graph_create(h.members, h.offsets, h.n_nodes, stream=stream)
        t0 = time.perf_counter()
        hm.count_nulls(g, 4, 64, 1, stream=stream)
        first_ms = (time.perf_counter() - t0) * 1e3
        t0 = time.perf_counter()
        for i in range(5):
            hm.count_nulls(g, 4, 64, 2 + i, stream=stream)
        print(json.dumps({"nulls_only": {"copies": 64, "first_call_ms": first_ms,
                                         "ms_per_batch": (time.perf_counter() - t0) * 1e3 / 5,
                                         "tile_sizes": hm.hm_null_tile_sizes(g)}}))
        g.close()
        return 0
    h = W.cfg1_facetoface_k4(0)
    members = torch.from_numpy(h.members.astype(np.int32)).to(dev)
    offsets = torch.from_numpy(h.offsets.astype(np.int64)).to(dev)
    counts = torch.empty(hm.hm_num_classes(4), dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()

    def step(st=stream, out=counts):
        g = hm.hm_graph_create(members, offsets, h.n_nodes, stream=st)
        hm.count_exact(g, 4, out=out, stream=st)
        g.close()

    # one hypergraph after another on one stream: the latency of a build and
    # its count
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    sequential_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    total = int(counts.sum().item())

    # whole-job throughput: the K hypergraphs in one call of count_exact_many,
    # whose PIPELINE worker threads build and count them on streams of their
    # own.  A build ends with the host waiting for its validation report, so
    # one hypergraph after another leaves the GPU idle during that wait and
    # while the next launches are issued; with several workers one
    # hypergraph's build runs on the CUs beside another's count.
    many_out = torch.empty((max(args.steps, args.warmup, PIPELINE), counts.numel()), dtype=torch.int64, device=dev)
    hm.count_exact_many([(members, offsets, h.n_nodes)] * max(args.warmup, PIPELINE), 4, workers=PIPELINE,
                        out=many_out, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hm.count_exact_many([(members, offsets, h.n_nodes)] * args.steps, 4, workers=PIPELINE, out=many_out,
                        stream=stream)
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / args.steps
    if not bool((many_out[:args.steps] == counts.unsqueeze(0)).all()):
        raise RuntimeError("a pipelined count differs from the sequential one")

    # counting alone on a resident graph, and per-kernel event timing
    g = hm.hm_graph_create(members, offsets, h.n_nodes, stream=stream)
    for _ in range(3):
        hm.count_exact(g, 4, out=counts, stream=stream)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(args.steps):
        hm.count_exact(g, 4, out=counts, stream=stream)
    stop.record(stream)
    torch.cuda.synchronize()
    count_ms = start.elapsed_time(stop) / args.steps
    hm.hm_profile_reset()
    hm.hm_profile_enable(True)
    for _ in range(args.steps):
        hm.count_exact(g, 4, out=counts, stream=stream)
    torch.cuda.synchronize()
    prof = hm.hm_profile_read()
    hm.hm_profile_enable(False)
    stats = g.stats()
    e2, e3 = g.export(2), g.export(3)
    exact = counts.cpu().numpy().astype(np.float64)

    # the projection baseline (Algorithm 1, Section 4.1) on the same resident
    # graph: the comparison of Table 2 (its projection rebuilt by every call)
    base_counts, base_stats = hm.count_baseline(g, 4, stream=stream)   # untimed: allocates the bit rows
    torch.cuda.synchronize()
    base_reps = 3
    start.record(stream)
    for _ in range(base_reps):
        hm.count_baseline(g, 4, out=base_counts, stats=base_stats, stream=stream)
    stop.record(stream)
    torch.cuda.synchronize()
    base_ms = start.elapsed_time(stop) / base_reps
    bs = base_stats.cpu().numpy()
    baseline = {"ms": base_ms, "candidates": int(bs[0]), "discarded": int(bs[1]),
                "matches_exact": bool(np.array_equal(base_counts.cpu().numpy(), counts.cpu().numpy())),
                "exact_speedup_over_baseline": base_ms / count_ms}
    print(f"baseline (Algorithm 1): {base_ms:.2f} ms per count, {int(bs[0])} candidates", file=sys.stderr, flush=True)
    # order 3 (Algorithm 2 against the baseline) on the smaller face-to-face
    # workload (N=200, 2,000 hyperedges)
    h3 = W.cfg0_facetoface_k3(0)
    with hm.hm_graph_create(h3.members, h3.offsets, h3.n_nodes, stream=stream) as g3:
        c3 = hm.count_exact(g3, 3, stream=stream)
        b3, s3 = hm.count_baseline(g3, 3, stream=stream)
        torch.cuda.synchronize()
        start.record(stream)
        for _ in range(args.steps):
            hm.count_exact(g3, 3, out=c3, stream=stream)
        stop.record(stream)
        torch.cuda.synchronize()
        exact3_ms = start.elapsed_time(stop) / args.steps
        start.record(stream)
        for _ in range(args.steps):
            hm.count_baseline(g3, 3, out=b3, stats=s3, stream=stream)
        stop.record(stream)
        torch.cuda.synchronize()
        base3_ms = start.elapsed_time(stop) / args.steps
        bs3 = s3.cpu().numpy()
        baseline["order3_facetoface_N200_E2000"] = {
            "ms": base3_ms, "exact_ms": exact3_ms, "candidates": int(bs3[0]), "discarded": int(bs3[1]),
            "matches_exact": bool(np.array_equal(b3.cpu().numpy(), c3.cpu().numpy())),
            "exact_speedup_over_baseline": base3_ms / exact3_ms}

    # sampled counting (Algorithm 4): time per call and mean relative error
    # over 32 seeds at 1% to 10% of every stratum
    sampled = {}
    for f in (() if args.exact_only else (0.01, 0.02, 0.03, 0.05, 0.10)):
        hm.count_sampled(g, 4, f, 999, stream=stream)   # untimed: first-call set-up
        torch.cuda.synchronize()
        runs = []
        start.record(stream)
        for seed in range(32):
            est, _ = hm.count_sampled(g, 4, f, 1000 + seed, stream=stream)
            runs.append(est)
        stop.record(stream)
        torch.cuda.synchronize()
        ms = start.elapsed_time(stop) / 32
        r = torch.stack(runs).double().cpu().numpy()
        mre = float(np.mean(np.abs(r - exact).sum(axis=1) / exact.sum()))
        sampled[f"{f:g}"] = {"ms": ms, "mre": mre, "speedup_vs_exact_count": count_ms / ms}
    ok = [k for k, v in sampled.items() if v["mre"] <= 0.02]
    best = min(ok, key=lambda k: float(k)) if ok else None

    order5 = None if args.exact_only else order5_leg(hm, W, stream)

    # Section 6.3 and Table 3: motif profiles against 10 configuration-model
    # draws (counted exactly), and the accuracy of profiles whose observed
    # counts are sampled (rho, MaxAE, MAE, mean over 10 repetitions); then the
    # appendix's stratum-budget search (Fig. 6) at 1% of the hyperedges
    profile_acc = None
    if not args.exact_only:
        sweeps = 10
        t0 = time.perf_counter()
        real_c, null_c, _ = hm.count_nulls_model(g, 4, 10, hm.HM_NULL_CONFIG, sweeps, 1, stream=stream)
        torch.cuda.synchronize()
        null_ms = (time.perf_counter() - t0) * 1e3
        t0 = time.perf_counter()
        hm.count_nulls_model(g, 4, 10, hm.HM_NULL_CONFIG, sweeps, 2, stream=stream)
        torch.cuda.synchronize()
        null_ms_replay = (time.perf_counter() - t0) * 1e3
        nd = null_c.double()
        exact_prof, _ = hm.hm_motif_profile(real_c.double(), nd)
        acc = {}
        for f in (0.01, 0.02, 0.05, 0.10):
            qs = []
            for rep in range(10):
                est, _ = hm.count_sampled(g, 4, f, 5000 + rep, stream=stream)
                d, _ = hm.hm_motif_profile(est.double(), nd)
                qs.append(hm.hm_profile_quality(d, exact_prof))
            q = np.array(qs)
            acc[f"{f:g}"] = {"rho": float(q[:, 0].mean()), "max_ae": float(q[:, 1].mean()),
                             "mae": float(q[:, 2].mean())}
        S = int(0.01 * (stats["n2"] + stats["n3"] + stats["n4"]))
        r3, r4 = [1.0, 2.0, 3.0, 4.0, 5.0], [1.0, 2.0, 3.0, 4.0]
        t0 = time.perf_counter()
        rho = hm.hm_stratum_search(g, 4, S, r3, r4, 10, 7000, nd, exact_prof, stream=stream)
        search_ms = (time.perf_counter() - t0) * 1e3
        bi, bj = np.unravel_index(int(np.argmax(rho)), rho.shape)
        profile_acc = {"null": "configuration model, 10 draws, 10 reshuffle sweeps",
                       "null_first_call_ms": null_ms, "null_ms_per_batch": null_ms_replay,
                       "sampled_profile_accuracy": acc,
                       "stratum_search": {"S": S, "ratio3": r3, "ratio4": r4, "reps": 10, "ms": search_ms,
                                          "mean_rho": rho.tolist(),
                                          "best": {"S3_over_S2": r3[bi], "S4_over_S2": r4[bj],
                                                   "rho": float(rho[bi, bj])},
                                          "paper_split_1_3_2_rho": float(rho[2, 1])}}

    # batched null model: 64 stub-matched copies counted at k = 4 in one graph launch
    nulls = None
    if not args.exact_only:
        t0 = time.perf_counter()
        hm.count_nulls(g, 4, 64, 1, stream=stream)
        first_ms = (time.perf_counter() - t0) * 1e3
        reps = 5
        t0 = time.perf_counter()
        for i in range(reps):
            hm.count_nulls(g, 4, 64, 2 + i, stream=stream)
        null_ms = (time.perf_counter() - t0) * 1e3 / reps
        nulls = {"copies": 64, "ms_per_batch": null_ms, "ms_per_copy": null_ms / 64,
                 "first_call_ms_incl_tuning_and_capture": first_ms, "tile_sizes": hm.hm_null_tile_sizes(g)}
    g.close()
    words = (h.n_nodes + 31) // 32
    units = _unit_counts(e2, e3, h.n_nodes, words)
    kernels = {k: {"launches": n, "avg_ms": ms / max(n, 1)} for k, (n, ms) in prof.items()}

    # roofline of the dominant kernel
    traffic = measured_traffic()
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"])
    avg_s = kernels[dom]["avg_ms"] / 1e3
    if dom == "k_exact4_bits":
        # the fused counting launch; its work is integer logic on adjacency words
        # held in LDS.  Case (c) by graph identities: per (pair, word) an AND, a
        # mask, a popcount and an add (4); per (pair, common neighbour, word) of
        # the 4-clique count the same 4; per (node pair, word) of the codegrees
        # an AND, a popcount and an add (3).  Case (b): per (3-node hyperedge,
        # word) 7 popcounts and about 21 further operations (28)
        ops = (units["id_edge_word_tasks"] * 4 + units["id_k4_word_tasks"] * 4
               + units["id_c4_pair_word_tasks"] * 3 + units["b4_word_tasks"] * 28)
        # beside the op model: the share of the VALU issue rate the launch used
        # (hardware counters), which shows what the op model leaves out
        roof = {"bound": "alu", "achieved": ops / avg_s / 1e12, "peak": ALU_PEAK_TOPS, "unit": "Tops/s",
                "frac": ops / avg_s / 1e12 / ALU_PEAK_TOPS, "traffic": traffic.get(dom),
                "valu_issue_frac": measured_valu_issue()}
    else:
        raise RuntimeError(f"unexpected dominant kernel {dom}")
    roof["kernel"] = dom

    large = None if (args.no_large or args.exact_only) else large_workloads(hm, W, torch)

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import core
        gpu_counts = counts.cpu().numpy()
        # the oracle's Algorithm 3 with its steps spread over every host thread
        # it is given (OMP_NUM_THREADS, else all cores), and on one thread
        threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
        t0 = time.perf_counter()
        ref, used = core.count_exact_threads(h, 4, threads)
        cpu_s = time.perf_counter() - t0
        t0 = time.perf_counter()
        ref1 = core.count_exact(h, 4)
        cpu1_s = time.perf_counter() - t0
        cpu = {"value": cpu_s * 1e3, "unit": "ms/hypergraph", "cores": used, "kind": "oracle",
               "sample": "one full count of the same hypergraph (Algorithm 3 in C, OpenMP over each step)",
               "single_thread": {"value": cpu1_s * 1e3, "unit": "ms/hypergraph", "cores": 1,
                                 "matches_gpu": bool(np.array_equal(ref1, gpu_counts))},
               "host_cpu": _cpu_model(), "host_cores": os.cpu_count(),
               "matches_gpu": bool(np.array_equal(ref, gpu_counts))}

    out = {
        "metric": METRIC,
        "value": ms_per_step,
        "unit": "ms/hypergraph",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "facetoface_N400_E30000", "k": 4, "seed": 0, "n_nodes": h.n_nodes,
                   "unique_by_size": [stats["n2"], stats["n3"], stats["n4"], stats["n5plus"]],
                   "connected_4_sets": total},
        "pipeline": {"workers": PIPELINE, "streams": PIPELINE,
                     "what": "the K hypergraphs in one count_exact_many call: worker threads of the library, "
                             "one stream each"},
        "sequential_ms_per_hypergraph": sequential_ms,
        "count_only_ms": count_ms,
        "baseline_algorithm1": baseline,
        "ingest_ms": sequential_ms - count_ms,
        "sampled": sampled,
        "sampled_speedup_at_2pct": ({"fraction": float(best), "speedup": sampled[best]["speedup_vs_exact_count"]}
                                    if best else None),
        "nulls": nulls,
        "order5": order5,
        "profiles": profile_acc,
        "large_workloads": large,
        "kernels": kernels,
        "units": units,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
