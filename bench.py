"""Benchmark of the LazyFox hot path on one MI355X.

One step = the whole hot path on one synthetic graph, from its raw edge list in pinned
host memory to the memberships in host memory: graph build (upload, dedup, CSR),
triangles / local CC / node order, greedy initial clustering, LazyFox iterations until the
stopping rule (threshold 0.01), memberships copied back.  Metric: node evaluations per
second over the whole step (n x iterations / step time); the end-to-end seconds are
ms_per_step.  Every timed step's memberships are hashed and checked against the oracle's
stored result for the same graph, queue size and threshold when one exists.

Prints one JSON line with, besides the contract fields, the roofline of the dominant
kernel (algorithmic bytes per launch / average launch duration, measured with HIP events
on the library's stream around every k-th launch of that kernel inside the timed steps),
byte-model rooflines of every kernel class above 5 % of the step (evaluation, apply,
triangles), the queue-size sweep, the dense workload, the serving comparison and the CPU
oracle timed on the same graph (build and initialisation windows, and a stated prefix of
queues of the first iteration at all host cores and at one thread).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, published
WORKLOADS = {
    # name: (graphgen config, default queue size, description)
    "social": ("social", 4096, "social-shaped planted-overlap power-law graph, 4,000,000 nodes, "
                               "~35M edges (exp 2.3, max degree 15,000, 1-4 memberships, mixing 0.4)"),
    "copurchase": ("copurchase", 256, "co-purchase-shaped graph, 335,000 nodes, ~926k edges"),
    "tiny_sbm": ("tiny_sbm", 64, "2,000-node overlapping SBM"),
    "dense": ("dense", 16384, "dense heavy-tail planted-overlap graph, 3,000,000 nodes, ~117M edges "
                              "(exp 2.1, max degree 33,000, 1-5 memberships, mixing 0.5)"),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="social", choices=sorted(WORKLOADS))
    ap.add_argument("--queue", type=int, default=0, help="queue size (default per workload)")
    ap.add_argument("--threshold", type=float, default=0.01)
    ap.add_argument("--max-iters", type=int, default=50)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-queues", type=int, default=0,
                    help="queues of the first iteration the oracle runs at all host cores (default: as many as "
                         "fill about 10 s)")
    ap.add_argument("--cpu-queues-1t", type=int, default=0,
                    help="queues the oracle runs at one thread (default: as many as fill about 10 s)")
    ap.add_argument("--event-stride", type=int, default=16,
                    help="HIP events bracket every k-th launch of the dominant kernel in the timed steps")
    ap.add_argument("--no-dense", action="store_true", help="skip the dense-workload run")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="also run a device copy of this many MiB (for HBM counter scaling)")
    ap.add_argument("--sweep", default="1024,2048,8192,16384,32768,65536",
                    help="comma-separated queue sizes run after the timed steps (end-to-end time, F1, "
                         "per-kernel bandwidth); empty to skip")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip tuning the path thresholds and launch shapes on the workload (untimed)")
    ap.add_argument("--options", default="",
                    help="fixed options instead of tuning, e.g. wave_table=128,med_table=512,grp_table=2048,"
                         "hub_blocks=1024,refresh_blocks=1024")
    ap.add_argument("--serving-jobs", type=int, default=10000,
                    help="jobs of the serving comparison (0 = skip it)")
    ap.add_argument("--serving-rate", type=float, default=200.0, help="Poisson arrival rate (jobs/s)")
    ap.add_argument("--serving-max-batch", type=int, default=256)
    ap.add_argument("--serving-budget-gib", type=float, default=64.0)
    ap.add_argument("--serving-no-graph", action="store_true", help="issue batch steps launch by launch")
    ap.add_argument("--serving-plain-jobs", type=int, default=500,
                    help="jobs of the trace (a prefix, in arrival order) also run one at a time (-1: all)")
    return ap.parse_args()


# Algorithmic bytes per unit of evaluation work (the per-unit bytes of the method's data,
# independent of how the kernels lay it out): per decided node 16 (its record) + 24 (the
# decision) + 8 per own membership; per neighbour 4 (column index) + 4 + 16 (its record);
# per neighbour membership visited 8; per candidate scored 44 (size 4, internal edges 8,
# score 8, one exact sum 24).
B_NODE, B_OWN, B_NEIGHBOUR, B_VISIT, B_CAND = 40.0, 8.0, 24.0, 8.0, 44.0
# Apply (bulk apply of Algorithm 2), bytes per unit of the apply work counters:
#   k_apply: every queued node 24 (decision 12, order entry 4, join position 4, line
#   placement 4); every moved node 52 (record 16, slot word 4, count 4, two sizes 8,
#   two touched flags 8, member-list entry 4, two member-list ranges 8) + 8 per own
#   membership scanned; every in-count unit of a moved node 24 (its record); every
#   neighbour in those units 36 (column 4, line header 16, order position 4, its decision
#   when queued ~12) + 8 per membership of it scanned; every touched community 24 to plan
#   (member-list range 16, part record 8) + 40 per part written.
#   k_refresh: every part 40 read + 16 (size, list length, overflow flag); every member
#   re-summed 20 (list entry 4, line header 16) + 8 per membership of it scanned; every
#   touched community 64 rewritten (its record).
A_QNODE, A_MOVE, A_OWN, A_UNIT, A_NEIGH, A_SLOT, A_PART, A_PLAN, A_REC, A_MEMBER, A_PSTAT = (
    24.0, 52.0, 8.0, 24.0, 36.0, 8.0, 40.0, 24.0, 64.0, 20.0, 16.0)


def path_bytes(w, with_candidates=True):
    b = (B_NODE * w["nodes"] + B_OWN * w.get("own", 0) + B_NEIGHBOUR * w["neighbours"]
         + B_VISIT * w["visits"])
    return b + (B_CAND * w["candidates"] if with_candidates else 0.0)


def apply_bytes(kernel, work):
    """Algorithmic bytes one pass moves through an apply kernel (work = the profile)."""
    a = work["apply"]
    if kernel == "k_apply":
        return (A_QNODE * work["node_evals"] + A_MOVE * a["moves"] + A_OWN * a["own_slots"]
                + A_UNIT * a["in_units"] + A_NEIGH * a["in_neighbours"] + A_SLOT * a["in_slots"]
                + A_PLAN * a["touched"] + A_PART * a["parts"])
    if kernel == "k_refresh":
        return ((A_PART + A_PSTAT) * a["parts"] + A_MEMBER * a["members"] + A_SLOT * a["member_slots"]
                + A_REC * a["touched"])
    return None


def kernel_bytes(kernel, work):
    """Algorithmic bytes one pass moves through `kernel` (None if no model for it).  A single
    graph's medium-path nodes are evaluated by k_eval, and so is the small path's work on
    the benchmark workload (its queues, >= 1024 small-path nodes, all give them k_eval
    blocks); k_eval_big holds the workgroup path and the table path's visits."""
    paths = work["paths"]
    if kernel == "k_eval":
        return path_bytes(paths["small"]) + path_bytes(paths["medium"])
    if kernel == "k_eval_big":
        return path_bytes(paths["group"]) + path_bytes(paths["table"], False)
    if kernel == "k_big_final":
        return B_CAND * paths["table"]["candidates"]
    return apply_bytes(kernel, work)


EVAL_KERNELS = ("k_eval", "k_eval_big", "k_big_final", "k_big_tie")
APPLY_KERNELS = ("k_apply", "k_refresh")


def eval_rates(timing, work):
    """Node evaluations, candidate scores and neighbour-membership visits per second of
    evaluation-kernel time (HIP-event times of the timing pass, counts of the counter pass)."""
    sec = sum(timing["ms"].get(k, 0.0) for k in EVAL_KERNELS) * 1e-3
    if sec <= 0.0:
        return None
    paths = work["paths"].values()
    return {"node_evals_per_s": timing["node_evals"] / sec,
            "candidate_evals_per_s": sum(p["candidates"] for p in paths) / sec,
            "membership_visits_per_s": sum(p["visits"] for p in paths) / sec}


def kernel_rooflines(timing, work):
    """Achieved algorithmic GB/s of each queue kernel with a byte model (HIP-event times of
    a profiled pass, bytes of a counter pass), of the evaluation kernels together and of
    the apply kernels together."""
    out = {}
    groups = {"evaluation": [0.0, 0.0], "apply": [0.0, 0.0]}
    for k in EVAL_KERNELS[:3] + APPLY_KERNELS:
        b = kernel_bytes(k, work)
        ms = timing["ms"].get(k, 0.0)
        if b is None or ms <= 0.0:
            continue
        gbs = b / (ms * 1e-3) / 1e9
        out[k] = {"GB_s": gbs, "frac": gbs / HBM_PEAK_GBS, "launches": timing["launches"][k], "ms": ms,
                  "bytes_per_pass": b}
        grp = groups["evaluation" if k in EVAL_KERNELS else "apply"]
        grp[0] += b
        grp[1] += ms
    groups["evaluation"][1] += timing["ms"].get("k_big_tie", 0.0)
    for name, (b, ms) in groups.items():
        if ms > 0.0:
            gbs = b / (ms * 1e-3) / 1e9
            out[name] = {"GB_s": gbs, "frac": gbs / HBM_PEAK_GBS, "ms": ms}
    return out


def triangle_roofline(h, timing_ms):
    """Byte models of the triangle phase (orientation by (degree, id), counting) over its
    measured time: B_min = 8(n+1) + 8|E| + 8n (the CSR once, the counts out) and the probe
    model B_probe = 8(n+1) + 4|E| (out-lists as the hash side) + 4 P (P = sum over
    oriented edges u->v of |N+(v)|, the probe side) + 8|E| (credits) + 8n."""
    import numpy as np
    rp, col = h.csr()
    n = rp.size - 1
    deg = np.diff(rp)
    row = np.repeat(np.arange(n, dtype=np.int64), deg)
    du, dv = deg[row], deg[col]
    later = (dv > du) | ((dv == du) & (col > row))          # v after u in (degree, id) order
    outd = np.bincount(row[later], minlength=n).astype(np.int64)
    ind = deg - outd
    E = int(col.size // 2)
    P = int(np.dot(ind, outd))
    b_min = 8.0 * (n + 1) + 8.0 * E + 8.0 * n
    b_probe = 8.0 * (n + 1) + 4.0 * E + 4.0 * P + 8.0 * E + 8.0 * n
    sec = timing_ms * 1e-3
    if sec <= 0:
        return None
    return {"ms": timing_ms, "probes": P, "B_min": b_min, "B_probe": b_probe,
            "GB_s_probe": b_probe / sec / 1e9, "frac_probe": b_probe / sec / 1e9 / HBM_PEAK_GBS,
            "GB_s_min": b_min / sec / 1e9, "frac_min": b_min / sec / 1e9 / HBM_PEAK_GBS,
            "what": "whole triangle phase (out-degrees, oriented lists, k_tri_wave / k_tri_group) by HIP events"}


# the translation unit of the evaluation and apply kernels and every header it includes
KERNEL_SOURCES = ("iterate.hip", "method.h", "exact.h", "lf_internal.h")


def kernel_sources_sha():
    """Hash of the sources the queue kernels are built from (their translation unit and
    its headers, the public header included)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2210_03211_amd", "csrc")
    for f in KERNEL_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    with open(os.path.join(ROOT, "include", "lazyfox.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()


def active_options(h):
    return ",".join("%s=%d" % (k, h.lf_get_option(k)) for k in TRAFFIC_OPTIONS)


TRAFFIC_OPTIONS = ("wave_table", "med_table", "grp_table", "hub_blocks", "refresh_blocks")


def stored_traffic(kernel, workload, options=None):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE per dispatch, scaled by the same counters on a copy of known
    size), or None if there is none, the kernel sources changed since it was taken, or it
    was taken with other launch options (they decide which paths share a launch)."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.txt" % (kernel, workload))
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_sources_sha256") != kernel_sources_sha():
        return None
    if options is not None and kv.get("options") != options:
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_peak_gbs(torch, nbytes=1 << 30, reps=5, device="cuda"):
    """Achievable memory rate of a plain device copy: bytes read plus bytes written per
    second, best of `reps` copies of `nbytes` (events on torch's current stream, where the
    copy runs; the host clock on a CPU device)."""
    a = torch.empty(nbytes, dtype=torch.uint8, device=device)
    b = torch.empty_like(a)
    a.fill_(1)
    b.copy_(a)                       # first touch
    best = None
    for _ in range(reps):
        if device == "cuda":
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            b.copy_(a)
            e1.record()
            e1.synchronize()
            sec = e0.elapsed_time(e1) * 1e-3
        else:
            t = time.perf_counter()
            b.copy_(a)
            sec = time.perf_counter() - t
        if sec > 0 and (best is None or sec < best):
            best = sec
    return 2.0 * nbytes / best / 1e9 if best else None


def host_info():
    """nproc, the CPUs this process may use, and the CPU model of the host."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "allowed_cpus": allowed, "cpu_model": model,
            "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline(args, g, q, gpu_iterations, golden):
    """The CPU oracle on the benchmark graph itself (same generator output, queue size and
    threshold): graph build and initialisation windows at all usable host cores (at most
    16, the host share of one GPU), then the first k queues of iteration 1 at one thread
    and again, from the same initial state (warm start from the saved initial cover), at
    all cores.  k is sized from a short pilot so that the one-thread window takes about
    10 s.  value = node evaluations per second of the all-core window."""
    import numpy as np
    import oracle
    hi = host_info()
    threads = max(1, min(16, hi["allowed_cpus"] or 1))
    t0 = time.perf_counter()
    o = oracle.Oracle().load_graph(g.n, g.src, g.dst)
    t_build = time.perf_counter() - t0
    t0 = time.perf_counter()
    o.init_communities(threads)
    t_init = time.perf_counter() - t0
    off0, ids0 = o.memberships()
    K0 = int(o.L.lfo_num_communities_created(o.h))
    n = o.n
    nq = (n + q - 1) // q

    def restore():
        o.init_from_memberships(off0, ids0, K0, threads)

    t0 = time.perf_counter()
    o.run_queue_prefix(q, 2, nthreads=1)
    pilot = (time.perf_counter() - t0) / 2
    k1 = args.cpu_queues_1t or int(max(2, min(nq, 10.0 / max(pilot, 1e-3))))
    k = args.cpu_queues or k1
    restore()
    t0 = time.perf_counter()
    done1 = o.run_queue_prefix(q, k1, nthreads=1)
    t_1 = time.perf_counter() - t0
    off1, ids1 = o.memberships()
    restore()
    t0 = time.perf_counter()
    done = o.run_queue_prefix(q, k, nthreads=threads)
    t_all = time.perf_counter() - t0
    if k == k1:                          # thread count must not change a bit (R23)
        off2, ids2 = o.memberships()
        if not (np.array_equal(off1, off2) and np.array_equal(ids1, ids2)):
            print("[bench] ERROR: oracle prefix differs between thread counts", file=sys.stderr)
            sys.exit(1)
    evals_all = sum(min(q, n - j * q) for j in range(done))
    evals_1 = sum(min(q, n - j * q) for j in range(done1))
    rate = evals_all / t_all
    total_evals = n * gpu_iterations
    out = {"value": rate, "unit": "node-evals/s", "cores": threads, "kind": "oracle",
           "sample": "the benchmark graph itself (%d nodes, %d edges), queue %d: build and initialisation "
                     "windows at %d threads, then the first %d of %d queues of iteration 1 at %d threads "
                     "(and the first %d at 1 thread), from the same initial state"
                     % (n, o.nedges, q, threads, done, nq, threads, done1),
           "host": hi, "threads": threads,
           "windows_s": {"build": t_build, "init": t_init, "queues_all_cores": t_all, "queues_1_thread": t_1},
           "queues_all_cores": done, "queues_1_thread": done1,
           "node_evals_per_s_1_thread": evals_1 / t_1,
           "end_to_end_estimate_s": t_build + t_init + total_evals / rate,
           "end_to_end_estimate_what": "build + init + n x GPU iteration count / prefix rate at all cores"}
    if golden and "oracle_seconds" in golden:
        out["stored_full_run_s"] = dict(golden["oracle_seconds"], what=golden.get("made_by", ""))
    return out


def stored_oracle(name, q, seed, threshold):
    """The oracle's stored result for (workload, queue size, seed), if one exists."""
    path = os.path.join(ROOT, "tests", "golden", "%s_q%d_seed%d.json" % (name, q, seed))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        gd = json.load(f)
    if gd.get("threshold") != threshold:
        return None
    gd["_file"] = os.path.relpath(path, ROOT)
    return gd


def check_against_oracle(gd, info, off, ids, what):
    """Memberships hash, iteration count and score history against the stored oracle
    result; exits with an error on any difference."""
    import numpy as np
    if gd is None:
        return {"stored_oracle": None}
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(off.astype("<i8")).tobytes())
    h.update(np.ascontiguousarray(ids.astype("<i4")).tobytes())
    ok = (h.hexdigest() == gd["memberships_sha256"] and info["iterations"] == gd["iterations"]
          and [float(w).hex() for w in info["wtilde_hist"]] == gd["wtilde_hist"])
    if not ok:
        print("[bench] ERROR: %s differs from the stored oracle result %s" % (what, gd["_file"]), file=sys.stderr)
        sys.exit(1)
    return {"stored_oracle": gd["_file"], "equal": True}


def start_background_graph(name, seed, outdir):
    """Generate a workload's edge list in a child process (before this process touches
    the GPU), saved as .npy files; returns the process."""
    import subprocess
    code = ("import sys, numpy as np; sys.path.insert(0, %r); import graphgen; "
            "g = graphgen.named_config(%r, seed=%d); np.save(%r, g.src); np.save(%r, g.dst); "
            "open(%r, 'w').write(str(g.n))") % (ROOT, name, seed, os.path.join(outdir, "src.npy"),
                                                 os.path.join(outdir, "dst.npy"), os.path.join(outdir, "n.txt"))
    return subprocess.Popen([sys.executable, "-c", code])


def dense_bench(args, lf, h, torch, proc, outdir):
    """The dense workload (3M nodes, ~117M edges, hubs to 33k) from its pinned host edge
    list: one untimed counter pass, one untimed kernel-timing pass and one timed run,
    checked against the stored oracle result when one exists."""
    import numpy as np
    t0 = time.perf_counter()
    if proc.wait() != 0:
        return {"error": "generator failed"}
    wait_s = time.perf_counter() - t0
    n = int(open(os.path.join(outdir, "n.txt")).read())
    src = torch.from_numpy(np.load(os.path.join(outdir, "src.npy"))).pin_memory()
    dst = torch.from_numpy(np.load(os.path.join(outdir, "dst.npy"))).pin_memory()
    q = WORKLOADS["dense"][1]

    def run(mask):
        h.lf_set_profiling(mask)
        h.load_graph(n, src, dst)
        h.init_communities()
        info = h.run_iterations(q, args.threshold, args.max_iters)
        off, ids = h.get_memberships()
        return info, off, ids

    h.lf_reset_profile()
    run(1 << lf.PROF_COUNTERS_BIT)
    work = h.lf_get_profile()
    h.lf_reset_profile()
    run(True)
    timing = h.lf_get_profile()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info, off, ids = run(0)
    dt = time.perf_counter() - t0
    nn, ne, K = h.lf_get_graph_info()
    gd = stored_oracle("dense", q, args.seed, args.threshold)
    out = {"workload": WORKLOADS["dense"][2], "nodes": nn, "edges": ne, "queue": q, "iterations": info["iterations"],
           "end_to_end_s": dt, "node_evals_per_s": nn * info["iterations"] / dt,
           "generator_wait_s": wait_s, "communities_created": K, "max_degree": int(np.max(np.diff(h.csr()[0]))),
           "kernel_ms_timing_pass": {k: round(v, 3) for k, v in timing["ms"].items()},
           "kernel_rooflines": kernel_rooflines(timing, work),
           "work_per_step": {"node_evals": work["node_evals"], "paths": work["paths"], "apply": work["apply"]}}
    out.update(check_against_oracle(gd, info, off, ids, "dense run"))
    print("[bench] dense: %.3fs, %d iterations, %s" % (dt, info["iterations"], out.get("stored_oracle")),
          file=sys.stderr, flush=True)
    h.lf_set_profiling(0)
    return out


def exact_wcc_bench(h, reps):
    """Exact WCC (triangle-based) of the final partition of the timed steps, next to the
    WCC-hat estimate the iterations optimised."""
    import torch
    h.lf_set_profiling(0)
    r = h.exact_wcc()                                  # warm-up
    times = []
    for _ in range(max(1, reps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r2 = h.exact_wcc()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    if r2["wcc"] != r["wcc"]:
        print("[bench] ERROR: exact WCC differs between calls", file=sys.stderr)
        sys.exit(1)
    sc = h.scores()
    ms = 1000.0 * sum(times) / len(times)
    print("[bench] exact WCC %.6g (WCC-hat %.6g) in %.2f ms" % (r["wcc"], sc["wcc_hat"], ms), file=sys.stderr,
          flush=True)
    return {"ms": ms, "wcc": r["wcc"], "wcc_hat": sc["wcc_hat"], "memberships": int(r["t"].size),
            "triangles": int(sc["triangles"]),
            "what": "lf_exact_wcc of the final partition (host outputs included): oriented triangle pass with "
                    "membership intersections, closing-edge flags, per-membership terms, exact sums"}


def cover_f1_bench(h, g, reps):
    """F1-Score of the final cover against the generator's planted cover."""
    import torch
    ref = g.planted_cover()
    if ref is None:
        return None
    roff = torch.from_numpy(ref[0]).cuda()
    rids = torch.from_numpy(ref[1]).cuda()
    h.lf_set_profiling(0)
    f1 = h.cover_f1(roff, rids)[0]                    # warm-up
    times = []
    for _ in range(max(1, reps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f1b = h.cover_f1(roff, rids)[0]
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    if f1b != f1:
        print("[bench] ERROR: cover F1 differs between calls", file=sys.stderr)
        sys.exit(1)
    ms = 1000.0 * sum(times) / len(times)
    print("[bench] F1 against the planted cover %.4f in %.2f ms" % (f1, ms), file=sys.stderr, flush=True)
    return {"ms": ms, "f1_vs_planted": f1, "reference_memberships": int(ref[1].size),
            "what": "lf_cover_f1 of the final cover against the planted cover (device arrays; per-community "
                    "best F1 and match copied to the host)"}


def postprocess_bench(h, reps):
    """Duplicated / contained community detection on the final cover (not applied)."""
    import torch
    h.lf_set_profiling(0)
    keep, rem = h.postprocess(True, True)             # warm-up
    times = []
    for _ in range(max(1, reps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        keep2, rem2 = h.postprocess(True, True)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    if rem2 != rem:
        print("[bench] ERROR: post-processing differs between calls", file=sys.stderr)
        sys.exit(1)
    ms = 1000.0 * sum(times) / len(times)
    print("[bench] post-processing: %d duplicates, %d contained in %.2f ms" % (rem[0], rem[1], ms),
          file=sys.stderr, flush=True)
    return {"ms": ms, "removed_duplicates": rem[0], "removed_contained": rem[1], "kept": int(keep.sum()),
            "what": "lf_postprocess (duplicates and strictly contained communities) of the final cover, "
                    "keep flags copied to the host, not applied"}


def warm_start_bench(h, reps):
    """Rebuild of the whole state from the final cover of the timed steps (device arrays)
    with lf_init_from_memberships; the rebuilt partition must score exactly the same."""
    import torch
    off, ids = h.get_memberships()
    K = h.lf_get_graph_info()[2]
    want = h.scores()["wtilde"]
    doff = torch.from_numpy(off).cuda()
    dids = torch.from_numpy(ids).cuda()
    h.lf_set_profiling(0)
    h.init_from_memberships(doff, dids, K)          # warm-up (allocations, node statistics kept)
    times = []
    for _ in range(max(1, reps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h.init_from_memberships(doff, dids, K)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    if h.scores()["wtilde"] != want:
        print("[bench] ERROR: warm start changed the partition score", file=sys.stderr)
        sys.exit(1)
    ms = 1000.0 * sum(times) / len(times)
    print("[bench] warm start: %.2f ms for %d memberships" % (ms, ids.size), file=sys.stderr, flush=True)
    return {"ms": ms, "memberships": int(ids.size), "communities": int(K),
            "memberships_per_s": ids.size / (ms * 1e-3), "what": "lf_init_from_memberships of the final "
            "cover (device arrays): checks, slots and in-counts, member lists, exact statistics, score"}


def start_serving_mix(args):
    """Generate the serving mix's graphs in worker processes forked before this process
    touches the GPU (they run only numpy), while the other workloads are measured."""
    import multiprocessing as mp
    import graphgen
    jobs = graphgen.serving_mix(n_jobs=args.serving_jobs, rate=args.serving_rate, seed=args.seed)
    pool = mp.get_context("fork").Pool(max(1, min(8, os.cpu_count() or 1)))
    return jobs, pool, pool.map_async(graphgen.serving_job_graph, jobs, chunksize=16), time.perf_counter()


def serving_bench(args, lf, gen):
    """The serving mix (Poisson arrivals, graphs of uneven size) served two ways on the
    same GPU and trace: the server with continuous batching, and plain one-at-a-time runs
    in arrival order.  Latency = completion - arrival.  Every job's memberships must be
    the same both ways."""
    import numpy as np
    jobs, pool, pending, t0 = gen
    t1 = time.perf_counter()
    graphs = pending.get()
    pool.close()
    pool.join()
    print("[bench] serving mix: %d jobs, %d nodes in all, generated in %.1fs (%.1fs waited)"
          % (len(jobs), sum(g.n for g in graphs), time.perf_counter() - t0, time.perf_counter() - t1),
          file=sys.stderr, flush=True)

    def digest(off, ids):
        return hashlib.sha256(off.tobytes() + ids.tobytes()).hexdigest()

    # continuous batching through the server
    srv = lf.Server(0, hbm_budget=int(args.serving_budget_gib * (1 << 30)), max_batch=args.serving_max_batch)
    srv.set_graph(not args.serving_no_graph)
    lat_b, hashes_b, evals_b = {}, {}, 0
    jid_of = {}
    nxt = 0
    start = time.perf_counter()
    while len(lat_b) < len(jobs):
        now = time.perf_counter() - start
        while nxt < len(jobs) and jobs[nxt]["arrival"] <= now:
            g = graphs[nxt]
            jid_of[srv.submit(g.n, g.src, g.dst, jobs[nxt]["queue"], args.threshold, args.max_iters)] = nxt
            nxt += 1
        if not jid_of:
            time.sleep(max(0.0, min(0.001, jobs[nxt]["arrival"] - now)))
            continue
        srv.tick()
        for jid in srv.take_done():
            r = srv.fetch(jid)
            k = jid_of.pop(jid)
            lat_b[k] = time.perf_counter() - start - jobs[k]["arrival"]
            hashes_b[k] = digest(r[0], r[1])
            evals_b += graphs[k].n * r[2]["iterations"]
    span_b = time.perf_counter() - start
    server_ms = srv.timing()
    srv.close()
    # plain: one job at a time, in arrival order, each alone on the device (on a prefix of
    # the trace when asked; the prefix's arrivals are the trace's own)
    import torch
    n_plain = len(jobs) if args.serving_plain_jobs < 0 else min(args.serving_plain_jobs, len(jobs))
    lat_p, evals_p, same = {}, 0, 0
    start = time.perf_counter()
    for k, (j, g) in enumerate(zip(jobs[:n_plain], graphs[:n_plain])):
        now = time.perf_counter() - start
        if now < j["arrival"]:
            time.sleep(j["arrival"] - now)
        h = lf.Handle(0)
        h.load_graph(g.n, g.src, g.dst).init_communities()
        info = h.run_iterations(j["queue"], args.threshold, args.max_iters)
        off, ids = h.get_memberships()
        h.close()
        lat_p[k] = time.perf_counter() - start - j["arrival"]
        evals_p += g.n * info["iterations"]
        same += digest(off, ids) == hashes_b[k]
    torch.cuda.synchronize()
    span_p = time.perf_counter() - start
    if same != n_plain:
        print("[bench] ERROR: %d of %d served results differ from the plain runs" % (n_plain - same, n_plain),
              file=sys.stderr)
        sys.exit(1)

    def pct(d, p):
        return 1000.0 * float(np.percentile(np.array(list(d.values())), p))
    out = {"jobs": len(jobs), "rate_per_s": args.serving_rate, "graph_replay": not args.serving_no_graph,
           "workload": "serving mix: Poisson arrivals, planted power-law graphs, nodes lognormal(median 2,000, "
                       "sigma 1.2) in [50, 200,000], mean degree 8-40, mixing 0.2-0.4, per-job queue",
           "batched": {"p50_ms": pct(lat_b, 50), "p99_ms": pct(lat_b, 99), "jobs_per_s": len(jobs) / span_b,
                       "node_evals_per_s": evals_b / span_b, "makespan_s": span_b,
                       "server_host_ms": {k: round(v, 1) for k, v in server_ms.items()}},
           "plain": None if n_plain == 0 else
                    {"jobs": n_plain, "p50_ms": pct(lat_p, 50), "p99_ms": pct(lat_p, 99),
                     "jobs_per_s": n_plain / span_p, "node_evals_per_s": evals_p / span_p, "makespan_s": span_p},
           "results_equal": True, "results_compared": n_plain}
    print("[bench] serving: %s" % json.dumps(out), file=sys.stderr, flush=True)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs each graph on one GPU and has no "
              "multi-GPU path (--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import tempfile

    import numpy as np

    import graphgen

    wl = WORKLOADS[args.workload]
    q = args.queue or wl[1]
    dense_dir = dense_proc = None
    if not args.no_dense and args.workload != "dense":
        # generated by a child process while the main workload is measured
        dense_dir = tempfile.mkdtemp(prefix="lf_dense_")
        dense_proc = start_background_graph("dense", args.seed, dense_dir)
    serve_gen = start_serving_mix(args) if args.serving_jobs > 0 else None
    import torch

    import paper_2210_03211_amd as lf
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    g = graphgen.named_config(wl[0], seed=args.seed, scale=args.scale)
    gen_s = time.perf_counter() - t0
    print("[bench] generated %s: n=%d pairs=%d in %.1fs" % (args.workload, g.n, g.npairs, gen_s),
          file=sys.stderr, flush=True)
    # the step starts from the raw edge list in pinned host memory
    src = torch.from_numpy(g.src).pin_memory()
    dst = torch.from_numpy(g.dst).pin_memory()
    h = lf.Handle(0)

    def step(profile_mask=0):
        h.lf_set_profiling(profile_mask)
        h.load_graph(g.n, src, dst)
        h.init_communities()
        info = h.run_iterations(q, args.threshold, args.max_iters)
        off, ids = h.get_memberships()
        return info, off, ids

    tuned = None
    if args.options:
        for kv in args.options.split(","):
            k, v = kv.split("=")
            h.lf_set_option(k.strip(), int(v))
    elif not args.no_autotune:
        h.load_graph(g.n, src, dst)
        h.init_communities()
        tuned = h.autotune(q, 3)
        print("[bench] autotune: %s" % json.dumps(tuned), file=sys.stderr, flush=True)
    for w in range(args.warmup):
        info, off, ids = step()
        print("[bench] warmup %d: %d iterations" % (w, info["iterations"]), file=sys.stderr, flush=True)
    # untimed pass with every kernel timed on its own: which kernel dominates
    h.lf_set_option("prof_stride", 1)
    h.lf_reset_profile()
    step(True)
    timing = h.lf_get_profile()
    dom = max(timing["ms"], key=lambda k: timing["ms"][k] if k.startswith("k_") else -1.0)
    dom_bit = 1 << lf.KERNEL_CLASSES.index(dom)
    print("[bench] per-kernel ms (timing pass): %s" % json.dumps(timing["ms"]), file=sys.stderr, flush=True)
    # untimed pass with the work counters (their atomics would disturb timing)
    h.lf_reset_profile()
    step(1 << lf.PROF_COUNTERS_BIT)
    work = h.lf_get_profile()
    print("[bench] work per step: %s %s" % (json.dumps(work["paths"]), json.dumps(work["apply"])), file=sys.stderr,
          flush=True)
    if args.calibrate_copy_mib:
        # a plain device copy of known size, for scaling the HBM byte counters
        nb = args.calibrate_copy_mib << 20
        a = torch.empty(nb, dtype=torch.uint8, device="cuda")
        b = torch.empty(nb, dtype=torch.uint8, device="cuda")
        a.fill_(1)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print("[bench] copy calibration: %d bytes read, %d written" % (nb, nb), file=sys.stderr, flush=True)
        del a, b

    # timed steps: events around every k-th launch of the dominant kernel only
    h.lf_set_option("prof_stride", max(1, args.event_stride))
    h.lf_reset_profile()
    hashes = set()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = []
    for k in range(args.steps):
        info, off, ids = step(dom_bit)
        iters.append(info["iterations"])
        hashes.add(hashlib.sha256(off.tobytes() + ids.tobytes()).hexdigest())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = h.lf_get_profile()
    h.lf_set_option("prof_stride", 1)
    if len(hashes) != 1:
        print("[bench] ERROR: runs differ", file=sys.stderr)
        sys.exit(1)
    golden = stored_oracle(args.workload, q, args.seed, args.threshold) if args.scale == 1.0 else None
    parity = check_against_oracle(golden, info, off, ids, "timed run")
    n, ne, K = h.lf_get_graph_info()
    ms_per_step = 1000.0 * dt / args.steps
    evals_per_step = n * iters[0]
    value = evals_per_step / (ms_per_step / 1000.0)

    # roofline of the dominant kernel: algorithmic bytes per launch (work counters of one
    # pass / launches per pass) over its average launch time in the timed steps
    launches = prof["launches"][dom]
    avg_ms = prof["ms"][dom] / max(1, launches)
    pass_bytes = kernel_bytes(dom, work)
    per_launch = pass_bytes / max(1, timing["launches"][dom]) if pass_bytes is not None else None
    achieved = per_launch / (avg_ms * 1e-3) / 1e9 if per_launch is not None else None
    traffic = stored_traffic(dom, args.workload, active_options(h))
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": traffic,
            "kernel": dom, "bytes_per_launch": per_launch, "avg_launch_ms": avg_ms, "launches_timed": launches,
            "event_stride": max(1, args.event_stride)}
    try:                                # informative only: never fails the bench line
        cp = copy_peak_gbs(torch)
        roof["achievable_GB_s"] = cp
        roof["frac_of_achievable"] = achieved / cp if (achieved and cp) else None
        print("[bench] device copy: %.0f GB/s" % cp, file=sys.stderr, flush=True)
    except Exception as e:              # noqa: BLE001
        print("[bench] device copy rate not measured: %s" % e, file=sys.stderr, flush=True)
        roof["achievable_GB_s"] = None
        roof["frac_of_achievable"] = None
    out = {
        "metric": "dWCC-hat node-evals/s (whole hot path, end-to-end)",
        "value": value, "unit": "node-evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl[2], "name": args.workload, "nodes": n, "edges": ne, "queue": q,
                   "threshold": args.threshold, "iterations": iters[0], "seed": args.seed,
                   "communities_created": K, "memberships_sha256": next(iter(hashes))[:16]},
        "end_to_end_s": ms_per_step / 1000.0,
        "end_to_end_window": "raw edge list in pinned host memory -> memberships in host memory",
        "parity": parity,
        "kernel_node_evals_per_s": timing["node_evals"] / max(1e-9, sum(timing["ms"][k] for k in EVAL_KERNELS) * 1e-3),
        "kernel_eval_rates": eval_rates(timing, work),
        "work_per_step": {"node_evals": work["node_evals"], "chunks": work["chunks"], "paths": work["paths"],
                          "apply": work["apply"]},
        "kernel_ms_timing_pass": {k: round(v, 3) for k, v in timing["ms"].items()},
        "roofline": roof,
    }
    if tuned is not None:
        out["autotune"] = tuned
    out["options"] = active_options(h)
    out["kernel_rooflines"] = kernel_rooflines(timing, work)
    out["kernel_rooflines"]["triangles"] = triangle_roofline(h, timing["ms"].get("triangles", 0.0))
    out["exact_wcc"] = exact_wcc_bench(h, args.steps)
    out["postprocess"] = postprocess_bench(h, args.steps)
    out["cover_f1"] = cover_f1_bench(h, g, args.steps)
    out["warm_start"] = warm_start_bench(h, args.steps)
    if args.sweep:
        sweep = {}
        for qq in [int(x) for x in args.sweep.split(",") if x]:
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            h.lf_set_profiling(0)
            h.load_graph(g.n, src, dst)
            h.init_communities()
            si = h.run_iterations(qq, args.threshold, args.max_iters)
            soff, sids = h.get_memberships()
            torch.cuda.synchronize()
            s = time.perf_counter() - t1
            sweep[str(qq)] = {"end_to_end_s": s, "iterations": si["iterations"],
                              "node_evals_per_s": n * si["iterations"] / s, "wcc_hat": si["wcc_hat"]}
            gq = stored_oracle(args.workload, qq, args.seed, args.threshold) if args.scale == 1.0 else None
            sweep[str(qq)].update(check_against_oracle(gq, si, soff, sids, "sweep run q=%d" % qq))
            ref = g.planted_cover()
            if ref is not None:
                sweep[str(qq)]["f1_vs_planted"] = h.cover_f1(*ref)[0]
            # per-kernel bandwidth at this queue size: a timed pass and a counter pass
            for mask, key in ((True, "t"), (1 << lf.PROF_COUNTERS_BIT, "w")):
                h.lf_reset_profile()
                h.lf_set_profiling(mask)
                h.load_graph(g.n, src, dst)
                h.init_communities()
                h.run_iterations(qq, args.threshold, args.max_iters)
                if key == "t":
                    tprof = h.lf_get_profile()
                else:
                    wprof = h.lf_get_profile()
            h.lf_set_profiling(0)
            sweep[str(qq)]["kernel_rooflines"] = kernel_rooflines(tprof, wprof)
            print("[bench] sweep q=%d: %.3fs %d iterations %s" % (qq, s, si["iterations"],
                                                                  sweep[str(qq)].get("stored_oracle")),
                  file=sys.stderr, flush=True)
        out["queue_sweep"] = sweep
    if dense_proc is not None:
        out["dense"] = dense_bench(args, lf, h, torch, dense_proc, dense_dir)
        import shutil
        shutil.rmtree(dense_dir, ignore_errors=True)
    h.close()
    if args.serving_jobs > 0:
        out["serving"] = serving_bench(args, lf, serve_gen)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args, g, q, iters[0], golden)
        print("[bench] cpu baseline: %s" % json.dumps(out["cpu_baseline"]), file=sys.stderr, flush=True)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
