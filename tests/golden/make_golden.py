"""Write the oracle's results for the full-size workloads (stored expected values).

Only the CPU oracle (oracle/) and the seeded generator (graphgen) are used: no value here
comes from the GPU path.  Each golden file holds, for one (workload, seed, queue size,
threshold), the iteration count, the cc-free score history as exact hex floats, the
number of memberships and a SHA-256 of the membership arrays (offsets int64 + community
ids int32, little-endian, exactly as lf_get_memberships returns them), plus the node
statistics' hashes.

    python tests/golden/make_golden.py social 4096      # ~ several minutes on 8 cores
    python tests/golden/make_golden.py -j6 dense 16384  # -jN: oracle thread count
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import graphgen  # noqa: E402
import oracle  # noqa: E402


def sha(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def make(name, q, seed=0, threshold=0.01, max_iters=50, nthreads=None):
    nthreads = nthreads or min(8, os.cpu_count() or 1)
    t0 = time.time()
    g = graphgen.named_config(name, seed=seed)
    o = oracle.Oracle().load_graph(g.n, g.src, g.dst).init_communities(nthreads)
    tri, ccl, order = o.node_stats()
    sc = o.scores()
    t1 = time.time()
    info = o.run_iterations(q, threshold, max_iters, mode=oracle.MODE_FAST, nthreads=nthreads)
    off, ids = o.memberships()
    out = {
        "workload": name, "seed": seed, "queue": q, "threshold": threshold, "max_iters": max_iters,
        "nodes": o.n, "edges": o.nedges, "triangles": sc["triangles"], "cc": sc["cc"].hex(),
        "tri_sha256": sha(tri), "ccl_sha256": sha(ccl), "order_sha256": sha(order),
        "iterations": info["iterations"], "converged": info["converged"],
        "wtilde_hist": [float(w).hex() for w in info["wtilde_hist"]],
        "joins": info["joins"].tolist(), "leaves": info["leaves"].tolist(),
        "communities": info["communities"].tolist(),
        "memberships": int(ids.size), "memberships_sha256": sha(off.astype("<i8"), ids.astype("<i4")),
        "oracle_seconds": {"init": round(t1 - t0, 1), "iterations": round(time.time() - t1, 1)},
        "made_by": "tests/golden/make_golden.py (CPU oracle, fast mode, %d threads)" % nthreads,
    }
    path = os.path.join(HERE, "%s_q%d_seed%d.json" % (name, q, seed))
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path, "iterations", out["iterations"], "in %.0fs" % (time.time() - t0))
    return out


if __name__ == "__main__":
    args = sys.argv[1:]
    nthreads = None
    if args and args[0].startswith("-j"):
        nthreads = int(args.pop(0)[2:])
    name = args[0] if args else "social"
    qs = [int(a) for a in args[1:]] or [4096]
    for q in qs:
        make(name, q, nthreads=nthreads)
