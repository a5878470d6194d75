"""Property tests of the CPU oracle on arbitrary tiny edge lists (hypothesis, CPU only).

Raw input as the method receives it (Methods, Preprocessing): duplicate edges, both
directions, self-loops and isolated nodes allowed.  Each drawn graph is checked against
the exact brute force, which shares no code with the oracle:

* triangles per node, the local clustering coefficient (one correctly rounded ratio, so
  bit-identical) and the node order of Node Order;
* the greedy Initial Clustering;
* a full LazyFox run (Algorithm 2) for a drawn queue size, skipped when an FP64 near-tie
  could legitimately separate the two;
* for a drawn cover: the warm-started state (in-counts from their definition, WCC-hat as
  an exact rational), the exact WCC terms, the post-processing flags from set definitions
  and the F1-Score against a second drawn cover as exact rationals.
"""
from fractions import Fraction

import numpy as np
from hypothesis import given
from hypothesis import strategies as st

from oracle import brute
from raw_graphs import SETTINGS, covers, edge_lists
from test_oracle_pins import _wcc_check, expected_pp, f1_exact


def memberships_list(o):
    off, ids = o.memberships()
    return [sorted(ids[off[x]:off[x + 1]].tolist()) for x in range(o.n)]


@SETTINGS
@given(g=edge_lists())
def test_node_statistics_and_initial_clustering(oracle_lib, g):
    o = oracle_lib.Oracle().load_graph(g.n, g.src, g.dst).init_communities(1)
    adj = brute.simple_graph(g.n, g.src, g.dst)
    k = brute.triangles(adj)
    ccl = brute.local_cc(adj, k)
    tri, cco, order = o.node_stats()
    assert tri.tolist() == k
    assert cco.tolist() == [float(c) for c in ccl]
    assert order.tolist() == brute.node_order(adj, ccl)
    assert o.scores()["triangles"] * 3 == sum(k)
    P = brute.initial_clustering(adj, brute.node_order(adj, ccl))
    assert memberships_list(o) == [[c for c, C in P.items() if x in C] for x in range(g.n)]


@SETTINGS
@given(g=edge_lists(max_n=11, max_pairs=36), qfrac=st.floats(0.0, 1.0), mode=st.sampled_from([0, 3]))
def test_full_run_against_brute_force(oracle_lib, g, qfrac, mode):
    q = max(1, int(round(qfrac * g.n)))
    b = brute.run(g.n, g.src, g.dst, q, 0.01, 12)
    o = oracle_lib.Oracle().load_graph(g.n, g.src, g.dst).init_communities(1)
    info = o.run_iterations(q, 0.01, 12, mode=mode, nthreads=1, check_every_chunk=True)
    if b["near_tie"]:
        return
    assert memberships_list(o) == b["memberships"]
    assert info["iterations"] == b["iterations"]
    if b["history"][0] > 0:
        cc = o.scores()["cc"]
        for w_o, w_b in zip(info["wtilde_hist"], b["history"]):
            assert abs(w_o / cc - float(w_b)) <= 1e-12 * float(w_b)


@SETTINGS
@given(data=st.data())
def test_covers_against_exact_definitions(oracle_lib, data):
    g = data.draw(edge_lists(max_n=10, max_pairs=30))
    k, off, ids, P = data.draw(covers(g.n))
    kr, roff, rids, Pr = data.draw(covers(g.n, max_comms=5, max_per_node=2))
    o = oracle_lib.Oracle().load_graph(g.n, g.src, g.dst).init_from_memberships(off, ids, k, 1)
    assert o.check_state() == 0
    adj = brute.simple_graph(g.n, g.src, g.dst)
    mo, mi = o.memberships()
    inc = o.in_counts()
    for x in range(g.n):
        assert sorted(mi[mo[x]:mo[x + 1]].tolist()) == sorted(c for c, C in P.items() if x in C)
        for p in range(mo[x], mo[x + 1]):
            assert inc[p] == len(adj[x] & P[int(mi[p])])
    tri = brute.triangles(adj)
    cc = sum(brute.local_cc(adj, tri), Fraction(0)) / g.n
    if cc > 0:
        w = brute.wcc_hat_partition(P, adj, cc)
        sc = o.scores()
        assert abs(sc["wtilde"] / sc["cc"] - float(w)) <= 1e-12 * max(float(w), 1e-300)
    _wcc_check(o, g, P)
    keep, (nd, nc) = o.postprocess(True, True)
    ek, end, enc = expected_pp(P, True, True)
    assert (nd, nc) == (end, enc)
    for c in range(k):
        assert keep[c] == (1 if c in P and ek[c] else 0)
    f1, best, match = o.cover_f1(roff, rids)
    score, per = f1_exact(P, Pr)
    assert abs(f1 - float(score)) <= 1e-15 * max(1.0, float(score))
    for c in range(k):
        if c in per:
            assert best[c] == float(per[c][0]) and match[c] == per[c][1]
        else:
            assert best[c] == 0.0 and match[c] == -1
