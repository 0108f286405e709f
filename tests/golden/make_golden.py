"""Write the stored expected counts under tests/golden/ by running the oracle.

Only ``oracle/`` and the seeded generators in ``workloads`` are called.
Run from the repository root:

    python tests/golden/make_golden.py            # every case
    python tests/golden/make_golden.py --heavy    # only the scaled heavy-tailed
                                                  # cases, merged into the file

The scaled heavy-tailed cases (the co-authorship and communication recipes
at a fraction of their nodes and draws) use the oracle's Algorithm 3 spread
over every host core; the smaller ones the single-thread routine.
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import core, nulls  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "workload_counts.json")


HEAVY = [("communication", W.scaled_communication, 0.01), ("communication", W.scaled_communication, 0.02),
         ("coauthorship", W.scaled_coauthorship, 0.004), ("communication", W.scaled_communication, 0.05),
         ("coauthorship", W.scaled_coauthorship, 0.01), ("coauthorship", W.scaled_coauthorship, 0.02)]


def heavy(only=None):
    """Scaled heavy-tailed cases, merged into the stored file one by one."""
    with open(OUT) as f:
        out = json.load(f)
    for family, fn, scale in HEAVY:
        name = f"{family}_scaled_{scale:g}"
        if only and name not in only:
            continue
        h = fn(scale, seed=0)
        t0 = time.time()
        c, threads = core.count_exact_threads(h, 4)
        case = {"workload": name, "seed": 0, "k": 4, "counts": c.tolist(),
                "oracle": "count_exact_threads", "threads": threads, "oracle_seconds": round(time.time() - t0, 1)}
        out["cases"] = [x for x in out["cases"] if not (x["workload"] == name and x["k"] == 4)] + [case]
        with open(OUT, "w") as f:
            json.dump(out, f, indent=1)
        print(name, int(c.sum()), f"{time.time() - t0:.1f}s on {threads} threads", flush=True)


def main():
    out = {"generator": "workloads.synth, numpy PCG64", "oracle": "oracle.core.count_exact (Algorithms 2 and 3)",
           "cases": []}
    for name, fn, k in [("facetoface_N200_E2000", W.cfg0_facetoface_k3, 3),
                        ("facetoface_N400_E30000", W.cfg1_facetoface_k4, 4)]:
        h = fn(0)
        t0 = time.time()
        c = core.count_exact(h, k)
        out["cases"].append({"workload": name, "seed": 0, "k": k, "counts": c.tolist(),
                             "oracle_seconds": round(time.time() - t0, 2)})
        print(name, k, int(c.sum()), f"{time.time() - t0:.1f}s", flush=True)
    h = W.scaled_communication(0.004, seed=0)
    t0 = time.time()
    c = core.count_exact(h, 4)
    out["cases"].append({"workload": "communication_scaled_0.004", "seed": 0, "k": 4, "counts": c.tolist(),
                         "oracle_seconds": round(time.time() - t0, 2)})
    print("communication_scaled_0.004", int(c.sum()), flush=True)
    # null copies of the order-4 workload (stub matching, seed 1): a few copies
    h = W.cfg1_facetoface_k4(0)
    for copy in (0, 1, 63):
        m, o = nulls.stub_matching(h, seed=1, copy=copy)
        c = core.count_exact(W.Hypergraph(h.n_nodes, m, o), 4)
        out["cases"].append({"workload": "facetoface_N400_E30000/null", "seed": 0, "null_seed": 1,
                             "copy": copy, "k": 4, "counts": c.tolist()})
        print("null copy", copy, int(c.sum()), flush=True)
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    if "--heavy" in sys.argv:
        heavy([a for a in sys.argv[1:] if not a.startswith("--")])
    else:
        main()
        heavy()
