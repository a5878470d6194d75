"""Host logic of bench.py (CPU): the one-GPU refusal, the rule that stored rocprofv3 traffic
is reported only for the kernel sources and launch options it was measured with, and the
algorithmic byte model behind the roofline."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def write_traffic(dirpath, sha, options, value=1234567):
    os.makedirs(os.path.join(dirpath, "profiles"), exist_ok=True)
    with open(os.path.join(dirpath, "profiles", "traffic_k_x_w.txt"), "w") as f:
        f.write("# comment: with a colon\n")
        f.write("traffic_bytes_per_launch: %d\n" % value)
        f.write("kernel_sources_sha256: %s\n" % sha)
        f.write("options: %s\n" % options)


def test_stored_traffic_needs_matching_sources_and_options(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_sources_sha", lambda: "abc")
    opts = "wave_table=128,med_table=512"
    assert bench.stored_traffic("k_x", "w", opts) is None          # no file
    write_traffic(str(tmp_path), "abc", opts)
    assert bench.stored_traffic("k_x", "w", opts) == 1234567.0
    assert bench.stored_traffic("k_x", "w") == 1234567.0          # options not checked
    assert bench.stored_traffic("k_x", "w", "wave_table=64,med_table=512") is None
    assert bench.stored_traffic("k_x", "other", opts) is None
    monkeypatch.setattr(bench, "kernel_sources_sha", lambda: "def")
    assert bench.stored_traffic("k_x", "w", opts) is None          # sources changed


def test_kernel_sources_sha_tracks_every_kernel_source(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2210_03211_amd" / "csrc"
    csrc.mkdir(parents=True)
    (tmp_path / "include").mkdir()
    for f in bench.KERNEL_SOURCES:
        (csrc / f).write_text("// " + f + "\n")
    (tmp_path / "include" / "lazyfox.h").write_text("// header\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    base = bench.kernel_sources_sha()
    assert bench.kernel_sources_sha() == base
    for f in bench.KERNEL_SOURCES:
        p = csrc / f
        old = p.read_text()
        p.write_text(old + " ")
        assert bench.kernel_sources_sha() != base, f
        p.write_text(old)
    (tmp_path / "include" / "lazyfox.h").write_text("// header changed\n")
    assert bench.kernel_sources_sha() != base


def test_committed_traffic_file_is_well_formed():
    path = os.path.join(ROOT, "profiles", "traffic_k_eval_big_social.txt")
    if not os.path.exists(path):
        pytest.skip("no stored traffic")
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    fetch = float(kv["fetch_kib_per_dispatch"]) * float(kv["fetch_scale"])
    write = float(kv["write_kib_per_dispatch"]) * float(kv["write_scale"])
    # the scale factors are printed to six decimals
    assert abs((fetch + write) * 1024 / float(kv["traffic_bytes_per_launch"]) - 1.0) < 1e-6
    ratio = float(kv["traffic_bytes_per_launch"]) / float(kv["algorithmic_bytes_per_launch"])
    assert abs(ratio - float(kv["traffic_over_algorithmic"])) < 0.01
    assert kv["kernel"] == "k_eval_big" and kv["workload"] == "social"
    assert sorted(o.split("=")[0] for o in kv["options"].split(",")) == sorted(bench.TRAFFIC_OPTIONS)


def paths(**w):
    z = {"nodes": 0, "neighbours": 0, "visits": 0, "candidates": 0, "own": 0}
    return {p: dict(z, **w.get(p, {})) for p in ("small", "medium", "group", "table")}


APPLY0 = {"moves": 0, "own_slots": 0, "in_units": 0, "in_neighbours": 0, "in_slots": 0, "parts": 0,
          "touched": 0, "members": 0, "member_slots": 0}


def work_of(p, node_evals=0, **apply):
    return {"paths": p, "node_evals": node_evals, "apply": dict(APPLY0, **apply)}


def test_kernel_byte_model():
    """Per-unit bytes of the evaluation: node 16 + 24 and 8 per own membership, neighbour
    4 + 4 + 16, visit 8, candidate 44."""
    p = paths(small={"nodes": 1, "neighbours": 2, "visits": 3, "candidates": 4, "own": 2},
              medium={"nodes": 10}, group={"candidates": 1},
              table={"nodes": 1, "neighbours": 1, "visits": 1, "candidates": 100, "own": 3})
    w = work_of(p)
    # the medium path is evaluated by k_eval
    assert bench.kernel_bytes("k_eval", w) == 40 + 2 * 8 + 2 * 24 + 3 * 8 + 4 * 44 + 10 * 40
    # the table path's candidates are scored in k_big_final, not in k_eval_big
    assert bench.kernel_bytes("k_eval_big", w) == 44 + 40 + 3 * 8 + 24 + 8
    assert bench.kernel_bytes("k_big_final", w) == 100 * 44
    assert bench.kernel_bytes("k_big_tie", w) is None


def test_apply_byte_model():
    w = work_of(paths(), node_evals=100, moves=10, own_slots=20, in_units=30, in_neighbours=40, in_slots=50,
                parts=6, touched=5, members=70, member_slots=80)
    assert bench.kernel_bytes("k_apply", w) == (100 * 24 + 10 * 52 + 20 * 8 + 30 * 24 + 40 * 36 + 50 * 8
                                                + 5 * 24 + 6 * 40)
    assert bench.kernel_bytes("k_refresh", w) == 6 * (40 + 16) + 70 * 20 + 80 * 8 + 5 * 64
    assert bench.kernel_bytes("k_apply_in", w) is None            # no longer launched


def test_kernel_rooflines_divide_bytes_by_event_time():
    p = paths(small={"nodes": 1_000_000}, group={"neighbours": 1_000_000}, table={"candidates": 1_000_000})
    w = work_of(p, node_evals=1_000_000)
    timing = {"ms": {"k_eval": 0.04, "k_eval_big": 0.024, "k_big_final": 0.044, "k_big_tie": 0.0,
                     "k_apply": 0.024},
              "launches": {"k_eval": 1, "k_eval_big": 1, "k_big_final": 1, "k_apply": 1}}
    r = bench.kernel_rooflines(timing, w)
    for k in ("k_eval", "k_eval_big", "k_big_final", "k_apply"):
        assert abs(r[k]["GB_s"] - 1000.0) < 1e-9, k
        assert abs(r[k]["frac"] - 1000.0 / bench.HBM_PEAK_GBS) < 1e-12
    assert abs(r["evaluation"]["GB_s"] - 1000.0) < 1e-9
    assert abs(r["apply"]["GB_s"] - 1000.0) < 1e-9
    timing["ms"]["k_big_tie"] = 0.108
    assert abs(bench.kernel_rooflines(timing, w)["evaluation"]["GB_s"] - 500.0) < 1e-9


def test_triangle_byte_models_on_a_small_graph():
    """B_min and the probe count P = sum over oriented edges u->v of |N+(v)| on a graph
    whose orientation is known: the path 0-1-2 plus the triangle 2-3-4."""
    import numpy as np

    class FakeHandle:
        def csr(self):
            adj = {0: [1], 1: [0, 2], 2: [1, 3, 4], 3: [2, 4], 4: [2, 3]}
            rp = np.zeros(6, np.int64)
            rp[1:] = np.cumsum([len(adj[i]) for i in range(5)])
            return rp, np.concatenate([adj[i] for i in range(5)]).astype(np.int32)
    r = bench.triangle_roofline(FakeHandle(), 1.0)
    # (degree, id) order: 0 (d1), 1 (d2), 3 (d2), 4 (d2), 2 (d3); each edge points to its
    # later end: 0->1, 1->2, 3->2, 4->2, 3->4; out-degrees 0:1, 1:1, 2:0, 3:2, 4:1 and
    # in-degrees 0:0, 1:1, 2:3, 3:0, 4:1, so P = 1*1 (node 1) + 3*0 (node 2) + 1*1 (node 4) = 2
    assert r["probes"] == 2
    assert r["B_min"] == 8 * 6 + 8 * 5 + 8 * 5
    assert r["B_probe"] == 8 * 6 + 4 * 5 + 4 * 2 + 8 * 5 + 8 * 5


def test_oracle_result_check(tmp_path, monkeypatch):
    """A run equal to the stored oracle result passes; any difference exits with an error."""
    import hashlib
    import json
    import numpy as np
    off = np.array([0, 1, 3], np.int64)
    ids = np.array([4, 1, 2], np.int32)
    hs = hashlib.sha256(off.tobytes() + ids.tobytes()).hexdigest()
    gd = {"memberships_sha256": hs, "iterations": 2, "wtilde_hist": [(1.5).hex(), (2.0).hex(), (2.25).hex()],
          "threshold": 0.01, "_file": "x.json"}
    info = {"iterations": 2, "wtilde_hist": np.array([1.5, 2.0, 2.25])}
    assert bench.check_against_oracle(gd, info, off, ids, "t")["equal"] is True
    assert bench.check_against_oracle(None, info, off, ids, "t") == {"stored_oracle": None}
    with pytest.raises(SystemExit):
        bench.check_against_oracle(gd, dict(info, iterations=3), off, ids, "t")
    with pytest.raises(SystemExit):
        bench.check_against_oracle(gd, info, off, np.array([4, 1, 3], np.int32), "t")
    os.makedirs(tmp_path / "tests" / "golden")
    with open(tmp_path / "tests" / "golden" / "w_q8_seed0.json", "w") as f:
        json.dump(dict(gd, threshold=0.01), f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.stored_oracle("w", 8, 0, 0.01)["memberships_sha256"] == hs
    assert bench.stored_oracle("w", 8, 0, 0.02) is None
    assert bench.stored_oracle("w", 16, 0, 0.01) is None


def test_copy_rate_counts_read_and_written_bytes():
    """The achievable-rate probe: 2 x bytes / best copy time (CPU device here; on the GPU the
    same arithmetic with event times)."""
    torch = pytest.importorskip("torch")
    r = bench.copy_peak_gbs(torch, nbytes=1 << 20, reps=3, device="cpu")
    assert r is not None and r > 0.0


def test_eval_rates():
    timing = {"ms": {"k_eval": 500.0, "k_eval_big": 300.0, "k_big_final": 150.0, "k_big_tie": 50.0,
                     "k_refresh": 999.0}, "node_evals": 4_000_000}
    work = {"paths": {"small": {"nodes": 1, "neighbours": 2, "visits": 10_000_000, "candidates": 6_000_000},
                      "table": {"nodes": 1, "neighbours": 2, "visits": 2_000_000, "candidates": 0}}}
    r = bench.eval_rates(timing, work)
    assert r == {"node_evals_per_s": 4_000_000.0, "candidate_evals_per_s": 6_000_000.0,
                 "membership_visits_per_s": 12_000_000.0}
    assert bench.eval_rates({"ms": {}, "node_evals": 1}, work) is None
