"""Exact WCC of a partition on the GPU (lf_exact_wcc) against the oracle: every
per-membership count and term and every total bit-identical at sizes the oracle finishes
in seconds, and spot checks of sampled nodes at the full social-shaped size."""
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


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


def gpu_handle(lf, g):
    import torch
    h = lf.Handle(0)
    h.load_graph(g.n, torch.from_numpy(g.src).cuda(), torch.from_numpy(g.dst).cuda())
    return h


def random_cover(n, n_comms, seed, hi=3, heavy=()):
    rng = np.random.default_rng(seed)
    per = [rng.choice(n_comms, size=min(40 if x in heavy else int(rng.integers(0, hi + 1)), n_comms),
                      replace=False).astype(np.int32) for x in range(n)]
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum([len(p) for p in per])
    return off, np.concatenate(per).astype(np.int32)


def bits(a):
    a = np.ascontiguousarray(a)
    return a.view(np.uint8).tobytes()


def same_wcc(a, b):
    for k in ("wcc_comm", "wcc_node", "t", "vt_out", "vt"):
        assert a[k].shape == b[k].shape, k
        assert bits(a[k]) == bits(b[k]), k
    assert bits(np.float64(a["wcc"])) == bits(np.float64(b["wcc"]))


def cliques(sizes):
    src, dst, off = [], [], 0
    for s in sizes:
        iu, ju = np.triu_indices(s, 1)
        src.append(iu + off)
        dst.append(ju + off)
        off += s
    return G.Graph(off, np.concatenate(src).astype(np.int64), np.concatenate(dst).astype(np.int64))


CASES = ["sbm_run", "copurchase_run", "random_heavy", "planted_powerlaw", "social_0.2pct_run", "cliques",
         "triangle_free"]


@pytest.mark.parametrize("case", CASES)
def test_exact_wcc_matches_oracle(lf, orc, case):
    if case == "sbm_run":
        g, cover, q = G.named_config("tiny_sbm"), None, 64
    elif case == "copurchase_run":
        g, cover, q = G.named_config("copurchase", scale=0.01), None, 32
    elif case == "random_heavy":
        g, q = G.random_gnp(500, 0.04, 21), None
        cover = random_cover(g.n, 200, 5, heavy={1, 2, 250, 499})
    elif case == "planted_powerlaw":
        g, q = G.named_config("copurchase", scale=0.02, seed=4), None
        cover = g.planted_cover()
    elif case == "social_0.2pct_run":
        g, cover, q = G.named_config("social", scale=0.002), None, 256
    elif case == "cliques":
        g, q = cliques([3, 5, 8, 40]), None
        cover = (np.arange(g.n + 1, dtype=np.int64), np.repeat(np.arange(4), [3, 5, 8, 40]).astype(np.int32))
    else:
        n = 64
        g, q = G.Graph(n, np.arange(n, dtype=np.int64), (np.arange(n, dtype=np.int64) + 1) % n), None
        cover = None
    say("exact wcc", case, "n", g.n)
    o = orc.Oracle().load_graph(g.n, g.src, g.dst)
    h = gpu_handle(lf, g)
    if cover is None:
        o.init_communities()
        h.init_communities()
        if q:
            o.run_iterations(q, 0.01, 50, mode=orc.MODE_FAST)
            h.run_iterations(q, 0.01, 50)
    else:
        o.init_from_memberships(*cover)
        h.init_from_memberships(*cover)
    a = o.exact_wcc()
    b = h.exact_wcc()
    same_wcc(a, b)
    if case == "cliques":
        assert b["wcc"] == float(g.n)
    if case == "triangle_free":
        assert b["wcc"] == 0.0 and not b["t"].any()
    h.close()


def test_exact_wcc_full_size_spot_checks(lf, orc):
    """The social-shaped graph at full size (4M nodes, ~35M edges) with its planted cover
    (generator output, so no oracle input comes from the GPU): the GPU terms of the 40
    highest-degree nodes and of 400 random nodes equal the oracle's per-node evaluation;
    the totals satisfy the bounds of the definition."""
    g = G.named_config("social")
    off, ids = g.planted_cover()
    say("full size exact wcc, n", g.n, "memberships", ids.size)
    h = gpu_handle(lf, g).init_from_memberships(off, ids)
    r = h.exact_wcc()
    hoff, hids = h.memberships()
    assert np.array_equal(hoff, off) and np.array_equal(hids, ids)
    tri = h.lf_get_node_stats()[0]
    node_of = np.repeat(np.arange(g.n), np.diff(off))
    assert np.all(r["wcc_node"] >= 0.0) and np.all(r["wcc_node"] <= 1.0)
    assert np.all(r["t"] <= tri[node_of]) and np.all(r["vt_out"] <= r["vt"][node_of])
    assert 0.0 < r["wcc"] <= float(ids.size)
    say("oracle load + warm start")
    o = orc.Oracle().load_graph(g.n, g.src, g.dst).init_from_memberships(off, ids, -1, 16)
    deg = np.diff(o.csr()[0])
    rng = np.random.default_rng(7)
    sample = np.concatenate([np.argsort(-deg, kind="stable")[:40], rng.choice(g.n, 400, replace=False)])
    sample = sample.astype(np.int32)
    say("oracle sample of", sample.size)
    wn, t, vo, vx = o.wcc_sample(sample)
    sel = np.concatenate([np.arange(off[x], off[x + 1]) for x in sample])
    assert np.array_equal(t, r["t"][sel]) and np.array_equal(vo, r["vt_out"][sel])
    assert np.array_equal(vx, r["vt"][sample])
    assert bits(wn) == bits(r["wcc_node"][sel])
    h.close()
