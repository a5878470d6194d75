"""Warm start from an existing cover (lf_init_from_memberships) on the GPU: the state it
builds and the runs from it equal the oracle's, bit for bit; resuming from saved
memberships continues a run exactly (also at the full social-shaped size)."""
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


def cover_from_lists(n, comms):
    """offsets/ids of a cover given as a list of member arrays (community id = index)."""
    per = [[] for _ in range(n)]
    for c, members in enumerate(comms):
        for x in members:
            per[int(x)].append(c)
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum([len(p) for p in per])
    ids = np.array([c for p in per for c in p], np.int32)
    return off, ids


def random_cover(n, n_comms, seed, lo=0, hi=3, heavy=()):
    """Random cover, ids unsorted per node; nodes in `heavy` get 40 memberships (more
    than a wave evaluation keeps in LDS, so they take the table path)."""
    rng = np.random.default_rng(seed)
    per = []
    for x in range(n):
        k = 40 if x in heavy else int(rng.integers(lo, hi + 1))
        per.append(rng.choice(n_comms, size=min(k, n_comms), replace=False).astype(np.int32))
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum([len(p) for p in per])
    return off, np.concatenate(per).astype(np.int32) if per else np.zeros(0, np.int32)


def gpu_handle(lf, g):
    import torch
    h = lf.Handle(0)
    h.load_graph(g.n, torch.from_numpy(g.src).cuda(), torch.from_numpy(g.dst).cuda())
    return h


def state_of(x):
    off, ids = x.memberships()
    s, m, W = x.communities()[:3]
    return off, ids, x.in_counts(), np.asarray(s), np.asarray(m), np.asarray(W)


def same_state(a, b):
    for u, v in zip(state_of(a), state_of(b)):
        u, v = np.asarray(u), np.asarray(v)
        assert u.shape == v.shape and np.array_equal(u.view(np.uint8), v.view(np.uint8))


def same_run(a, b):
    assert a["iterations"] == b["iterations"]
    assert np.array_equal(np.asarray(a["wtilde_hist"]).view(np.int64), np.asarray(b["wtilde_hist"]).view(np.int64))


def test_warm_start_from_cold_memberships_is_the_cold_start(lf):
    for name, g, q in (("sbm2000", G.named_config("tiny_sbm"), 64),
                       ("copurchase_1pct", G.named_config("copurchase", scale=0.01), 32)):
        say("cold vs warm", name)
        cold = gpu_handle(lf, g).init_communities()
        off, ids = cold.memberships()
        K = cold.lf_get_graph_info()[2]
        warm = gpu_handle(lf, g).init_from_memberships(off, ids, K)
        same_state(cold, warm)
        assert cold.scores()["wtilde"] == warm.scores()["wtilde"]
        same_run(cold.run_iterations(q, 0.01, 50), warm.run_iterations(q, 0.01, 50))
        same_state(cold, warm)
        cold.close()
        warm.close()


@pytest.mark.parametrize("case", ["random_small", "random_heavy", "planted_sbm", "planted_powerlaw"])
def test_warm_start_matches_oracle(lf, orc, case):
    """Covers with gaps in the ids, empty and one-member communities, unsorted lists, nodes
    with 40 memberships; state after the warm start and after the run vs the oracle."""
    if case == "random_small":
        g, q = G.random_gnp(300, 0.04, 11), 16
        off, ids = random_cover(g.n, 120, 1)
        K = 130
    elif case == "random_heavy":
        g, q = G.random_gnp(400, 0.05, 12), 64
        off, ids = random_cover(g.n, 300, 2, heavy={0, 5, 17, 100, 399})
        K = -1
    elif case == "planted_sbm":
        g, q = G.named_config("tiny_sbm", seed=2), 64
        off, ids = cover_from_lists(g.n, g.planted)
        off2, ids2 = g.planted_cover()
        assert np.array_equal(off, off2) and np.array_equal(ids, ids2)
        K = -1
    else:
        g, q = G.named_config("copurchase", scale=0.02, seed=1), 128
        off, ids = g.planted_cover()
        K = -1
    say("warm start", case, "n", g.n, "memberships", ids.size)
    o = orc.Oracle().load_graph(g.n, g.src, g.dst).init_from_memberships(off, ids, K)
    h = gpu_handle(lf, g).init_from_memberships(off, ids, K)
    same_state(o, h)
    assert o.scores()["wtilde"] == h.scores()["wtilde"]
    oi = o.run_iterations(q, 0.01, 30, mode=orc.MODE_FAST)
    hi = h.run_iterations(q, 0.01, 30)
    same_run(oi, hi)
    same_state(o, h)
    h.close()


def test_device_and_host_covers_agree(lf):
    import torch
    g = G.named_config("tiny_sbm")
    off, ids = random_cover(g.n, 500, 3)
    a = gpu_handle(lf, g).init_from_memberships(off, ids)
    b = gpu_handle(lf, g).init_from_memberships(torch.from_numpy(off).cuda(), torch.from_numpy(ids).cuda())
    same_state(a, b)
    same_run(a.run_iterations(32, 0.01, 20), b.run_iterations(32, 0.01, 20))
    same_state(a, b)


def test_resume_continues_the_run(lf):
    """Checkpoint after k iterations, warm start a new handle from the memberships, run on:
    the same iterations, scores and final cover as the uninterrupted run."""
    for name, g, q, ks in (("copurchase_5pct", G.named_config("copurchase", scale=0.05), 256, (1, 2)),
                           ("social_1pct", G.named_config("social", scale=0.01), 1024, (2,))):
        say("resume", name)
        full = gpu_handle(lf, g).init_communities()
        fi = full.run_iterations(q, 0.001, 50)
        assert fi["iterations"] > max(ks)
        for k in ks:
            part = gpu_handle(lf, g).init_communities()
            part.run_iterations(q, 0.001, k)
            off, ids = part.memberships()
            K = part.lf_get_graph_info()[2]
            part.close()
            res = gpu_handle(lf, g).init_from_memberships(off, ids, K)
            assert res.scores()["wtilde"] == fi["wtilde_hist"][k]
            ri = res.run_iterations(q, 0.001, 50 - k)
            assert ri["iterations"] == fi["iterations"] - k
            assert ri["converged"] == fi["converged"] and ri["hit_max"] == fi["hit_max"]
            assert np.array_equal(ri["wtilde_hist"], fi["wtilde_hist"][k:])
            same_state(res, full)
            res.close()
        full.close()


def test_resume_at_full_size(lf):
    """The social-shaped graph at full size (4M nodes, queue 4096): resume after two
    iterations equals the uninterrupted run (a property that holds at any size)."""
    g = G.named_config("social")
    say("full size resume, n", g.n)
    full = gpu_handle(lf, g).init_communities()
    fi = full.run_iterations(4096, 0.01, 50)
    part = gpu_handle(lf, g).init_communities()
    part.run_iterations(4096, 0.01, 2)
    off, ids = part.memberships()
    K = part.lf_get_graph_info()[2]
    part.close()
    res = gpu_handle(lf, g).init_from_memberships(off, ids, K)
    ri = res.run_iterations(4096, 0.01, 48)
    assert ri["iterations"] == fi["iterations"] - 2
    assert ri["converged"] == fi["converged"]
    assert np.array_equal(ri["wtilde_hist"], fi["wtilde_hist"][2:])
    a, b = full.memberships(), res.memberships()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    full.close()
    res.close()


def test_bad_covers_are_refused_and_keep_the_partition(lf):
    g = G.random_gnp(60, 0.1, 4)
    h = gpu_handle(lf, g).init_communities()
    before = state_of(h)
    off = np.arange(g.n + 1, dtype=np.int64)
    bad = [
        (off, np.full(g.n, 7, np.int32), 5),                                         # id >= n_comms
        (off, np.full(g.n, -1, np.int32), -1),                                       # negative id
        (np.concatenate([[0], np.full(g.n, 2, np.int64)]), np.array([3, 3], np.int32), -1),   # twice
        (np.concatenate([[0, 2, 1], np.full(g.n - 2, 2, np.int64)]), np.array([1, 2], np.int32), -1),
    ]
    wrong_total = off.copy()
    wrong_total[-1] += 1
    bad.append((wrong_total, np.zeros(g.n, np.int32), -1))
    for o, i, K in bad:
        with pytest.raises(lf.LazyFoxError):
            h.init_from_memberships(o, i, K)
        for u, v in zip(before, state_of(h)):
            assert np.array_equal(u, v)
    with pytest.raises(ValueError):
        h.init_from_memberships(off[:-1], np.zeros(g.n - 1, np.int32))
    h.run_iterations(8, 0.01, 5)
    h.close()
