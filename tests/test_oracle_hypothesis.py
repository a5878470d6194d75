"""Property tests of the CPU oracle on arbitrary tiny edge lists (hypothesis, CPU only).

Raw input as the method receives it (Methods, Preprocessing): duplicate edges, both
directions, self-loops and isolated nodes allowed.  Each drawn graph is checked against
the exact brute force, which shares no code with the oracle:

* triangles per node, the local clustering coefficient (one correctly rounded ratio, so
  bit-identical) and the node order of Node Order;
* the greedy Initial Clustering;
* a full LazyFox run (Algorithm 2) for a drawn queue size, skipped when an FP64 near-tie
  could legitimately separate the two.
"""
from hypothesis import given
from hypothesis import strategies as st

from oracle import brute
from raw_graphs import SETTINGS, edge_lists


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
