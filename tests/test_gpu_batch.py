"""Many graphs advanced together (lf_batch_*) and the serving runtime (lf_server_*) on
the GPU: every graph's result in a batch or a served mix is bit-identical to its result
alone (and to the oracle's), whatever else shares the launches."""
import sys

import numpy as np
import pytest

import graphgen as G

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lf():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2210_03211_amd as lfmod
    lfmod.load_library()
    return lfmod


def path(n):
    return G.Graph(n, np.arange(n - 1, dtype=np.int64), np.arange(1, n, dtype=np.int64))


def graphs():
    """(name, graph, queue size, max_iters): sizes from 30 to 67,000 nodes, a graph without
    triangles (0 iterations) and one cut short by max_iters."""
    return [
        ("gnp80", G.random_gnp(80, 0.12, 7), 7, 50),
        ("sbm2000", G.named_config("tiny_sbm"), 64, 50),
        ("copurchase_1pct", G.named_config("copurchase", scale=0.01), 32, 50),
        ("social_0.2pct", G.named_config("social", scale=0.002), 256, 50),
        ("social_1pct", G.named_config("social", scale=0.01), 1024, 50),
        ("copurchase_20pct", G.named_config("copurchase", scale=0.2), 256, 50),
        ("path30", path(30), 4, 50),
        ("sbm2000_2it", G.named_config("tiny_sbm", seed=3), 16, 2),
    ]


def alone(lf, g, q, max_iters):
    import torch
    h = lf.Handle(0)
    h.load_graph(g.n, torch.from_numpy(g.src).cuda(), torch.from_numpy(g.dst).cuda()).init_communities()
    info = h.run_iterations(q, 0.01, max_iters)
    off, ids = h.memberships()
    return h, info, off, ids


def same_info(a, b):
    assert a["iterations"] == b["iterations"]
    assert a["converged"] == b["converged"] and a["hit_max"] == b["hit_max"]
    assert np.array_equal(a["wtilde_hist"].view(np.int64), b["wtilde_hist"].view(np.int64))
    assert np.array_equal(a["joins"], b["joins"]) and np.array_equal(a["leaves"], b["leaves"])
    assert np.array_equal(a["communities"], b["communities"])
    assert a["wcc_hat"] == b["wcc_hat"]


@pytest.mark.parametrize("graph", [True, False])
def test_batch_equals_alone_and_oracle(lf, graph):
    """Both ways of issuing a step: graph replay (several hundred replays, with the
    members' eager iteration starts and ends in between) and launches one by one."""
    import torch
    import oracle
    oracle.build(force=False)
    gs = graphs()
    ref = {}
    for name, g, q, mi in gs:
        say("alone", name)
        h, info, off, ids = alone(lf, g, q, mi)
        ref[name] = (info, off, ids, h.in_counts())
        h.close()
    # the oracle agrees with the solo runs on the small ones
    for name, g, q, mi in gs[:4] + gs[6:]:
        say("oracle", name)
        o = oracle.Oracle().load_graph(g.n, g.src, g.dst).init_communities()
        oi = o.run_iterations(q, 0.01, mi, mode=oracle.MODE_FAST)
        assert oi["iterations"] == ref[name][0]["iterations"]
        ooff, oids = o.memberships()
        assert np.array_equal(ooff, ref[name][1]) and np.array_equal(oids, ref[name][2])
    say("batch of", len(gs), "graph replay", graph)
    b = lf.Batch(0)
    b.set_graph(graph)
    hs, mids = [], []
    for name, g, q, mi in gs:
        h = lf.Handle(0)
        h.load_graph(g.n, torch.from_numpy(g.src).cuda(), torch.from_numpy(g.dst).cuda()).init_communities()
        hs.append(h)
        mids.append(b.add(h, q, 0.01, mi))
    steps = 0
    while b.step() > 0:
        steps += 1
        assert steps < 100000
    for (name, g, q, mi), h, m in zip(gs, hs, mids):
        say("compare", name)
        info = b.member_info(m)
        assert info is not None
        same_info(info, ref[name][0])
        b.remove(m)
        off, ids = h.memberships()
        assert np.array_equal(off, ref[name][1]) and np.array_equal(ids, ref[name][2])
        assert np.array_equal(h.in_counts(), ref[name][3])
        h.close()
    b.close()


def test_batch_members_join_late_and_leave_early(lf):
    """Members added while others are half-way, and one removed before it finishes: the
    rest are unaffected."""
    import torch
    gs = graphs()[:6]
    ref = {name: alone(lf, g, q, mi)[1:] for name, g, q, mi in gs}
    b = lf.Batch(0)
    hs = {}
    mids = {}

    def add(i):
        name, g, q, mi = gs[i]
        h = lf.Handle(0)
        h.load_graph(g.n, torch.from_numpy(g.src).cuda(), torch.from_numpy(g.dst).cuda()).init_communities()
        hs[name] = h
        mids[name] = b.add(h, q, 0.01, mi)

    add(4)
    add(1)
    for _ in range(3):
        b.step()
    add(0)
    add(5)
    add(3)
    b.step()
    b.remove(mids.pop("social_1pct"))      # leaves before it is done
    hs.pop("social_1pct").close()
    add(2)
    while b.step() > 0:
        pass
    for name, m in mids.items():
        say("compare", name)
        info = b.member_info(m)
        same_info(info, ref[name][0])
        off, ids = hs[name].memberships()
        assert np.array_equal(off, ref[name][1]) and np.array_equal(ids, ref[name][2])
    b.close()


def test_batch_errors(lf):
    b = lf.Batch(0)
    h = lf.Handle(0)
    with pytest.raises(lf.LazyFoxError):
        b.add(h, 16)                       # no graph / communities yet
    g = G.random_gnp(40, 0.2, 1)
    import torch
    h.load_graph(g.n, torch.from_numpy(g.src).cuda(), torch.from_numpy(g.dst).cuda()).init_communities()
    with pytest.raises(lf.LazyFoxError):
        b.add(h, 0)
    m = b.add(h, 8, 0.01, 50)
    assert b.member_info(m) is None
    with pytest.raises(lf.LazyFoxError):
        b.member_info(m + 5)
    b.close()


def serving_jobs(n_jobs, max_n, seed=0):
    jobs = [j for j in G.serving_mix(n_jobs=4 * n_jobs, seed=seed) if j["n"] <= max_n][:n_jobs]
    return [(j, G.serving_job_graph(j)) for j in jobs]


def test_server_mix_equals_alone(lf):
    """A served mix with a budget that admits only a few jobs at a time: each job's
    memberships and run info equal its solo run."""
    jobs = serving_jobs(24, 20000)
    ref = {}
    for j, g in jobs:
        h, info, off, ids = alone(lf, g, j["queue"], 50)
        ref[j["job"]] = (info, off, ids, h.lf_get_memory()[1])
        h.close()
    srv = lf.Server(0, hbm_budget=1 << 30, max_batch=6)
    ids_of = {}
    for j, g in jobs:
        ids_of[srv.submit(g.n, g.src, g.dst, j["queue"], 0.01, 50)] = j["job"]
    done = {}
    ticks = 0
    while True:
        pending = srv.tick()
        st = srv.stats()
        assert st["used"] <= st["budget"] and st["running"] <= 6
        for jid in list(ids_of):
            r = srv.fetch(jid)
            if r is not None:
                done[ids_of.pop(jid)] = r
        ticks += 1
        assert ticks < 200000
        if pending == 0 and not ids_of:
            break
    assert len(done) == len(jobs)
    for j, g in jobs:
        say("job", j["job"], "n", g.n)
        off, ids, info = done[j["job"]]
        same_info(info, ref[j["job"]][0])
        assert np.array_equal(off, ref[j["job"]][1]) and np.array_equal(ids, ref[j["job"]][2])
    srv.close()


def test_server_reserves_at_least_the_device_peak(lf):
    """The footprint the server reserves for a job covers the device memory the same job
    uses at its peak when run alone; a job larger than the whole budget is refused."""
    for j, g in serving_jobs(6, 200000, seed=5):
        h, info, off, ids = alone(lf, g, j["queue"], 50)
        peak = h.lf_get_memory()[1]
        h.close()
        srv = lf.Server(0, hbm_budget=64 << 30, max_batch=4)
        jid = srv.submit(g.n, g.src, g.dst, j["queue"], 0.01, 50)
        srv.tick()
        reserved = srv.stats()["used"]
        say("job n", g.n, "peak", peak, "reserved", reserved)
        assert reserved >= peak
        while srv.tick() > 0:
            pass
        assert srv.fetch(jid) is not None
        srv.close()
    srv = lf.Server(0, hbm_budget=1 << 20, max_batch=4)
    g = G.named_config("tiny_sbm")
    with pytest.raises(lf.LazyFoxError):
        srv.submit(g.n, g.src, g.dst, 64)
    srv.close()


def test_autotune_keeps_results_and_remembers_the_class(lf):
    """The tuner picks options from its candidate lists, leaves the handle at its initial
    clustering, changes no result, and reuses its choice for a graph of the same class."""
    import torch
    h0 = lf.Handle(0)
    h0.lf_autotune_forget()
    for name, q in (("copurchase_1pct", 32), ("social_0.2pct", 256)):
        g = {"copurchase_1pct": G.named_config("copurchase", scale=0.01),
             "social_0.2pct": G.named_config("social", scale=0.002)}[name]
        say("autotune", name)
        ref_h, ref_info, ref_off, ref_ids = alone(lf, g, q, 50)
        ref_h.close()
        h = lf.Handle(0)
        h.load_graph(g.n, torch.from_numpy(g.src).cuda(), torch.from_numpy(g.dst).cuda()).init_communities()
        r = h.autotune(q, 1)
        assert not r["from_cache"] and r["trials"] >= 5 and r["best_ms"] <= r["default_ms"]
        o = r["options"]
        assert o["wave_table"] in (32, 64, 128) and o["med_table"] in (128, 256, 512)
        assert o["grp_table"] in (512, 1024, 2048)
        for k, v in o.items():
            assert h.lf_get_option(k) == v
        info = h.run_iterations(q, 0.01, 50)
        same_info(info, ref_info)
        off, ids = h.memberships()
        assert np.array_equal(off, ref_off) and np.array_equal(ids, ref_ids)
        h2 = lf.Handle(0)
        h2.load_graph(g.n, torch.from_numpy(g.src).cuda(), torch.from_numpy(g.dst).cuda()).init_communities()
        r2 = h2.autotune(q, 1)
        assert r2["from_cache"] and r2["options"] == o
        h.close()
        h2.close()
    h0.lf_autotune_forget()
    h0.close()
