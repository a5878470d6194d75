"""GPU parity on arbitrary tiny raw edge lists (hypothesis; duplicates, both directions,
self-loops, isolated nodes, n from 1).  For each drawn graph and queue size the HIP path
and the oracle must agree bit for bit on the CSR, the node statistics, the initial
clustering, the whole run (score history, move counts, memberships, in-counts, community
table), the exact WCC of the final cover, its post-processing flags and its F1 against the
initial clustering.  Drawn sets of such graphs run through a batch and through the
serving runtime must each give the oracle's result for the graph alone."""
import sys

import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

from raw_graphs import SETTINGS, edge_lists

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lf():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2210_03211_amd as lfmod
    lfmod.load_library()
    return lfmod


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


def bits(a):
    return np.ascontiguousarray(a).view(np.uint8).tobytes()


@SETTINGS
@given(g=edge_lists(), qfrac=st.floats(0.0, 1.0), device_ptr=st.booleans())
def test_raw_tiny_graphs_match_oracle(lf, orc, g, qfrac, device_ptr):
    import torch
    q = max(1, int(round(qfrac * g.n)))
    print("[case] n", g.n, "pairs", g.npairs, "q", q, "device", device_ptr, flush=True)
    sys.stdout.flush()
    h = lf.Handle(0)
    try:
        if device_ptr:
            h.load_graph(g.n, torch.from_numpy(g.src).cuda(), torch.from_numpy(g.dst).cuda())
        else:
            h.load_graph(g.n, g.src, g.dst)
        o = orc.Oracle().load_graph(g.n, g.src, g.dst)
        assert h.n == o.n and h.nedges == o.nedges
        for a, b in zip(h.csr(), o.csr()):
            assert np.array_equal(a, b)
        h.init_communities()
        o.init_communities(1)
        for a, b in zip(h.node_stats(), o.node_stats()):
            assert bits(a) == bits(b)
        off0, ids0 = o.memberships()
        for a, b in zip(h.memberships(), (off0, ids0)):
            assert np.array_equal(a, b)
        hi = h.run_iterations(q, 0.01, 12)
        oi = o.run_iterations(q, 0.01, 12, mode=orc.MODE_FAST)
        assert hi["iterations"] == oi["iterations"]
        assert hi["converged"] == oi["converged"] and hi["hit_max"] == oi["hit_max"]
        for k in ("wtilde_hist", "joins", "leaves", "communities"):
            assert bits(hi[k]) == bits(oi[k]), k
        for a, b in zip(h.memberships(), o.memberships()):
            assert np.array_equal(a, b)
        assert np.array_equal(h.in_counts(), o.in_counts())
        for a, b in zip(h.communities()[:3], o.communities()[:3]):
            assert bits(a) == bits(b)
        a, b = h.exact_wcc(), o.exact_wcc()
        for k in ("wcc_comm", "wcc_node", "t", "vt_out", "vt"):
            assert bits(a[k]) == bits(b[k]), k
        assert bits(np.float64(a["wcc"])) == bits(np.float64(b["wcc"]))
        ka, ra = h.postprocess(True, True)
        kb, rb = o.postprocess(True, True)
        assert ra == rb and np.array_equal(ka, kb)
        fa, fb = h.cover_f1(off0, ids0), o.cover_f1(off0, ids0)
        assert bits(np.float64(fa[0])) == bits(np.float64(fb[0]))
        for x, y in zip(fa[1:], fb[1:]):
            assert bits(x) == bits(y)
    finally:
        h.close()


def oracle_run(orc, g, q, max_iters):
    o = orc.Oracle().load_graph(g.n, g.src, g.dst).init_communities(1)
    info = o.run_iterations(q, 0.01, max_iters, mode=orc.MODE_FAST)
    return info, o.memberships()


def same_run(info, ref):
    assert info["iterations"] == ref["iterations"]
    assert info["converged"] == ref["converged"] and info["hit_max"] == ref["hit_max"]
    for k in ("wtilde_hist", "joins", "leaves", "communities"):
        assert bits(info[k]) == bits(ref[k]), k


jobs = st.lists(st.tuples(edge_lists(), st.floats(0.0, 1.0), st.sampled_from([1, 2, 12])), min_size=1, max_size=5)


@SETTINGS
@given(js=jobs, replay=st.booleans())
def test_raw_tiny_graphs_batched_match_oracle(lf, orc, js, replay):
    """Several drawn graphs advanced together by one batch (graph replay or launches one by
    one): each member's run equals the oracle's run of its graph alone."""
    import torch
    print("[case] batch of", len(js), "n", [g.n for g, _, _ in js], "replay", replay, flush=True)
    b = lf.Batch(0)
    b.set_graph(replay)
    hs, mids, refs = [], [], []
    try:
        for g, qf, mi in js:
            q = max(1, int(round(qf * g.n)))
            h = lf.Handle(0)
            hs.append(h)
            h.load_graph(g.n, torch.from_numpy(g.src).cuda(), torch.from_numpy(g.dst).cuda()).init_communities()
            mids.append(b.add(h, q, 0.01, mi))
            refs.append(oracle_run(orc, g, q, mi))
        steps = 0
        while b.step() > 0:
            steps += 1
            assert steps < 100000
        for h, m, (ref, (ooff, oids)) in zip(hs, mids, refs):
            same_run(b.member_info(m), ref)
            b.remove(m)
            off, ids = h.memberships()
            assert np.array_equal(off, ooff) and np.array_equal(ids, oids)
    finally:
        for h in hs:
            h.close()
        b.close()


@settings(max_examples=40, deadline=None, derandomize=True, database=None)
@given(js=jobs, max_batch=st.integers(1, 3))
def test_raw_tiny_graphs_served_match_oracle(lf, orc, js, max_batch):
    """The same graphs submitted to the serving runtime with few jobs admitted at a time:
    each fetched result equals the oracle's run of its graph alone."""
    print("[case] serve", len(js), "n", [g.n for g, _, _ in js], "max_batch", max_batch, flush=True)
    srv = lf.Server(0, hbm_budget=1 << 30, max_batch=max_batch)
    try:
        want = {}
        for g, qf, mi in js:
            q = max(1, int(round(qf * g.n)))
            want[srv.submit(g.n, g.src, g.dst, q, 0.01, mi)] = oracle_run(orc, g, q, mi)
        done = {}
        ticks = 0
        while True:
            pending = srv.tick()
            for jid in [j for j in want if j not in done]:
                r = srv.fetch(jid)
                if r is not None:
                    done[jid] = r
            ticks += 1
            assert ticks < 100000
            if pending == 0 and len(done) == len(want):
                break
        for jid, (ref, (ooff, oids)) in want.items():
            off, ids, info = done[jid]
            same_run(info, ref)
            assert np.array_equal(off, ooff) and np.array_equal(ids, oids)
    finally:
        srv.close()
