"""Post-processing of the final cover on the GPU (lf_postprocess: duplicated and contained
communities) against the oracle, and its defining property at the full social size."""
import random
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


def nested_cover(n, seed, base=40):
    """Random communities plus planted duplicates, strict subsets, supersets, chains."""
    rng = random.Random(seed)
    P = {}
    for c in range(base):
        P[c] = set(rng.sample(range(n), rng.randint(2, 12)))
    k = base
    for _ in range(base // 2):
        a = rng.randrange(base)
        kind = rng.randrange(4)
        if kind == 0:
            P[k] = set(P[a])
        elif kind == 1:
            P[k] = set(rng.sample(sorted(P[a]), max(1, len(P[a]) - rng.randint(1, 3))))
        elif kind == 2:
            P[k] = P[a] | set(rng.sample(range(n), 2))
        else:
            P[k] = P[a] | P[(a + 1) % base]
        k += 1
    off = np.zeros(n + 1, np.int64)
    per = [[] for _ in range(n)]
    for c in sorted(P):
        for x in P[c]:
            per[x].append(c)
    off[1:] = np.cumsum([len(p) for p in per])
    return off, np.array([c for p in per for c in p], np.int32), k + 3


def state_of(x):
    off, ids = x.memberships()
    s, m, W = x.communities()[:3]
    return [np.asarray(a) for a in (off, ids, x.in_counts(), s, m, W)]


def same_state(a, b):
    for u, v in zip(state_of(a), state_of(b)):
        assert u.shape == v.shape and u.view(np.uint8).tobytes() == v.view(np.uint8).tobytes()


FLAGS = [(True, True), (True, False), (False, True)]


@pytest.mark.parametrize("case", ["nested_0", "nested_1", "nested_2", "sbm_run", "copurchase_run",
                                  "social_0.2pct_run", "planted_powerlaw"])
def test_postprocess_matches_oracle(lf, orc, case):
    if case.startswith("nested"):
        seed = int(case[-1])
        g = G.random_gnp(200, 0.05, 40 + seed)
        cover, q = nested_cover(g.n, seed), None
    elif case == "sbm_run":
        g, cover, q = G.named_config("tiny_sbm"), None, 64
    elif case == "copurchase_run":
        g, cover, q = G.named_config("copurchase", scale=0.01), None, 32
    elif case == "social_0.2pct_run":
        g, cover, q = G.named_config("social", scale=0.002), None, 256
    else:
        g, q = G.named_config("copurchase", scale=0.02, seed=4), None
        off, ids = g.planted_cover()
        cover = (off, ids, -1)
    for dup, cont in FLAGS:
        say("postprocess", case, dup, cont)
        o = orc.Oracle().load_graph(g.n, g.src, g.dst)
        h = gpu_handle(lf, g)
        if cover is None:
            o.init_communities().run_iterations(q, 0.01, 50, mode=orc.MODE_FAST)
            h.init_communities().run_iterations(q, 0.01, 50)
        else:
            o.init_from_memberships(*cover)
            h.init_from_memberships(*cover)
        ko, ro = o.postprocess(dup, cont)
        kh, rh = h.postprocess(dup, cont)
        assert ro == rh and np.array_equal(ko, kh)
        ko, ro = o.postprocess(dup, cont, apply=True)
        kh, rh = h.postprocess(dup, cont, apply=True)
        assert ro == rh and np.array_equal(ko, kh)
        same_state(o, h)
        assert o.scores()["wtilde"] == h.scores()["wtilde"]
        h.close()


def test_postprocess_full_size_property(lf):
    """Full social size, the GPU's own final cover: every removed community (a sample) has
    a container among its first member's communities, equal with a lower id or strictly
    larger; no kept community (a sample) has one; after applying, nothing is removed."""
    import torch
    g = G.named_config("social")
    h = gpu_handle(lf, g).init_communities()
    h.run_iterations(4096, 0.01, 50)
    keep, (nd, nc) = h.postprocess(True, True)
    off, ids = h.memberships()
    say("full size: removed", nd, "duplicates,", nc, "contained of", int(keep.size))
    node_of = np.repeat(np.arange(g.n), np.diff(off))
    o = np.argsort(ids, kind="stable")
    cid, cnode = ids[o], node_of[o]
    K = keep.size
    starts = np.searchsorted(cid, np.arange(K + 1))
    members = lambda c: set(cnode[starts[c]:starts[c + 1]].tolist())
    comms_of = lambda x: ids[off[x]:off[x + 1]].tolist()

    def container(c):
        A = members(c)
        x = min(A)
        for b in comms_of(x):
            if b == c:
                continue
            B = members(b)
            if (B == A and b < c) or (A < B):
                return b
        return None

    live = np.flatnonzero(starts[1:] > starts[:-1])
    removed = [c for c in live if not keep[c]]
    kept = [c for c in live if keep[c]]
    assert len(removed) == nd + nc
    rng = np.random.default_rng(3)
    for c in rng.choice(removed, min(200, len(removed)), replace=False) if removed else []:
        assert container(int(c)) is not None
    for c in rng.choice(kept, 500, replace=False):
        assert container(int(c)) is None
    h.postprocess(True, True, apply=True)
    keep2, rem2 = h.postprocess(True, True)
    assert rem2 == (0, 0)
    h.close()
