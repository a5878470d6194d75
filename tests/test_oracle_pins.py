"""Pins of the CPU oracle against what the paper and mathematics fix (CPU only).

Each test names the passage it follows.  The oracle is checked against things other than
itself: exact rationals (``fractions``), ``math.fsum``, networkx, textbook identities,
closed forms and brute force on tiny graphs.
"""
import math
import random
from fractions import Fraction

import numpy as np
import pytest

import graphgen as G
from oracle import brute


# ------------------------------------------------------------------ helpers
def cycle(n):
    return G.Graph(n, np.arange(n, dtype=np.int64), (np.arange(n, dtype=np.int64) + 1) % n)


def path(n):
    return G.Graph(n, np.arange(n - 1, dtype=np.int64), np.arange(1, n, dtype=np.int64))


def star(n):
    return G.Graph(n, np.zeros(n - 1, np.int64), np.arange(1, n, dtype=np.int64))


def clique(n, off=0):
    iu, ju = np.triu_indices(n, 1)
    return iu.astype(np.int64) + off, ju.astype(np.int64) + off


def cliques(sizes):
    src, dst, off = [], [], 0
    for s in sizes:
        a, b = clique(s, off)
        src.append(a)
        dst.append(b)
        off += s
    return G.Graph(off, np.concatenate(src), np.concatenate(dst))


def complete(n):
    a, b = clique(n)
    return G.Graph(n, a, b)


def load(oracle_lib, g, relabel=False):
    return oracle_lib.Oracle().load_graph(g.n, g.src, g.dst, relabel=relabel).init_communities(2)


def memberships_list(o):
    off, ids = o.memberships()
    return [sorted(ids[off[x]:off[x + 1]].tolist()) for x in range(o.n)]


# ------------------------------------------------------------------ exact accumulator
def test_exact_sum_matches_fsum_and_fractions(oracle_lib):
    """All decision sums are exact then rounded once: compare with math.fsum (correctly
    rounded) and with the rounded Fraction sum, including heavy cancellation."""
    rng = np.random.default_rng(7)
    for trial in range(200):
        n = int(rng.integers(1, 300))
        kind = trial % 4
        if kind == 0:
            v = rng.random(n)
        elif kind == 1:
            v = rng.standard_normal(n) * 10.0 ** rng.integers(-30, 30, n)
        elif kind == 2:  # cancellation: x, -x pairs plus tiny residue
            x = rng.random(n) * 1e10
            v = np.concatenate([x, -x, rng.random(3) * 1e-40])
        else:  # values of the method's size range: g in (2^-62, 1]
            v = 2.0 ** rng.uniform(-62, 0, n) * np.where(rng.random(n) < 0.5, -1, 1)
        v = rng.permutation(v)
        got = oracle_lib.exact_sum(v)
        assert got == math.fsum(v.tolist())
        assert got == float(sum((Fraction(float(a)) for a in v), Fraction(0)))
    # ties to even: 1 + 2^-53 rounds to 1, 1 + 3*2^-53 rounds up
    assert oracle_lib.exact_sum([1.0, 2.0 ** -53]) == 1.0
    assert oracle_lib.exact_sum([1.0, 2.0 ** -53, 2.0 ** -53, 2.0 ** -53]) == 1.0 + 2.0 ** -51
    assert oracle_lib.exact_sum([]) == 0.0


def test_g_and_density_are_single_roundings(oracle_lib):
    """g(i,d,s) = i(i-1) / ((d-1)(s-1+d-i)) (the estimator with E[t(x,C)] = C(i,2)p,
    E[t(x,V)] = C(d,2)cc, |C\\{x}| = s-1, deg(x,V\\C) = d-i, divided by p/cc) and the
    density 2m/(s(s-1)): each is the correctly rounded value of the exact rational."""
    rnd = random.Random(3)
    for _ in range(2000):
        d = rnd.randint(0, 5000)
        s = rnd.randint(1, 100000)
        i = rnd.randint(0, min(d, s))
        got = oracle_lib.g_term(i, d, s)
        if d < 2 or i < 2:
            assert got == 0.0
        else:
            exact = Fraction(i * (i - 1), (d - 1) * (s - 1 + d - i))
            assert got == float(exact)
            # and it is the paper's WCC-hat(x,C) * cc / p for any p, cc > 0
            p, cc = Fraction(3, 7), Fraction(2, 9)
            w = (Fraction(i * (i - 1), 2) * p) / (Fraction(d * (d - 1), 2) * cc) * Fraction(d, (s - 1) + (d - i))
            assert w * cc / p == exact
        m = rnd.randint(0, s * (s - 1) // 2)
        got_p = oracle_lib.density(s, m)
        assert got_p == (0.0 if s < 2 else float(Fraction(2 * m, s * (s - 1))))


def test_exact_accumulator_ranges_hold_at_the_extremes(oracle_lib):
    """The fixed-point widths rest on three facts, checked at the limits of the integer
    ranges (d, s < 2^31, a member's in-count i <= min(d, s - 1)): a non-zero g lies in
    (2^-62, 1] with its lowest set bit at or above 2^-114; a community score
    p * R(sum g) lies in (2^-124, 2^31) with its lowest set bit at or above 2^-176."""
    top = (1 << 31) - 1
    cases = [(2, top, top), (2, 2, top), (2, top, 3), (top - 1, top, top), (3, 3, 4), (2, 2, 3),
             (1000, 5000, 100000), (2, 5000, 100000)]
    gmin = 1.0
    for i, d, s in cases:
        g = oracle_lib.g_term(i, d, s)
        assert g == float(Fraction(i * (i - 1), (d - 1) * (s - 1 + d - i)))
        assert 2.0 ** -62 < g <= 1.0, (i, d, s, g)
        assert (Fraction(g) * 2 ** 114).denominator == 1
        gmin = min(gmin, g)
    # the smallest density times the smallest sum, and the largest score
    pmin = oracle_lib.density(top, 1)
    assert pmin == float(Fraction(2, top * (top - 1)))
    w = pmin * gmin
    assert 2.0 ** -124 < w and (Fraction(w) * 2 ** 176).denominator == 1
    assert oracle_lib.density(top, top * (top - 1) // 2) == 1.0 and float(top - 1) < 2.0 ** 31


# ------------------------------------------------------------------ preprocessing
def test_load_graph_dedup_selfloops_relabel(oracle_lib):
    """Multi-edges become one edge, self-loops are dropped, rows are sorted; with relabel
    the ids present are compacted in increasing order (Preprocessing)."""
    src = np.array([5, 9, 9, 5, 7, 7, 100, 100], np.int64)
    dst = np.array([9, 5, 5, 7, 5, 7, 9, 100], np.int64)
    o = oracle_lib.Oracle().load_graph(0, src, dst, relabel=True)
    assert o.n == 4 and o.nedges == 3
    assert o.orig_ids().tolist() == [5, 7, 9, 100]
    rp, col = o.csr()
    assert rp.tolist() == [0, 2, 3, 5, 6]
    assert col.tolist() == [1, 2, 0, 0, 3, 2]
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.Oracle().load_graph(3, np.array([0]), np.array([3]))


def test_triangles_brute_force_and_identities(oracle_lib):
    """k_i = number of edges between neighbours of i (Node Order): brute force over all
    triples on small graphs; sum of k = 3T."""
    for seed in range(25):
        g = G.random_gnp(24, 0.3, seed)
        o = load(oracle_lib, g)
        tri, _, _ = o.node_stats()
        adj = brute.simple_graph(g.n, g.src, g.dst)
        assert tri.tolist() == brute.triangles(adj)
        assert o.scores()["triangles"] * 3 == tri.sum()


def test_triangles_trace_identity_and_networkx(oracle_lib):
    """On the 2,000-node planted graph: k_x = (A^3)_xx / 2 and networkx.triangles."""
    nx = pytest.importorskip("networkx")
    g = G.named_config("tiny_sbm")
    o = load(oracle_lib, g)
    tri, ccl, order = o.node_stats()
    rp, col = o.csr()
    A = np.zeros((o.n, o.n))
    rows = np.repeat(np.arange(o.n), np.diff(rp))
    A[rows, col] = 1.0
    a3 = np.einsum("ij,ji->i", A @ A, A)     # exact in float64 at these magnitudes
    assert np.array_equal(a3 / 2, tri.astype(np.float64))
    Gx = nx.Graph()
    Gx.add_nodes_from(range(o.n))
    Gx.add_edges_from(zip(rows.tolist(), col.tolist()))
    t = nx.triangles(Gx)
    assert [t[x] for x in range(o.n)] == tri.tolist()
    # local CC: networkx computes 2t/(d(d-1)) -- the same rational, one rounding
    c = nx.clustering(Gx)
    assert [c[x] for x in range(o.n)] == ccl.tolist()
    # global cc = mean of all local CCs (zeros included)
    cc = o.scores()["cc"]
    # networkx sums sequentially: its error is bounded by n * 2^-53 relative
    assert abs(cc - nx.average_clustering(Gx)) <= o.n * 2.0 ** -53 * cc
    assert cc == math.fsum(ccl.tolist()) / o.n


def test_node_order_closed_forms(oracle_lib):
    """Order: CC descending, ties by degree descending (Node Order), then id ascending."""
    o = load(oracle_lib, path(5))
    assert o.node_stats()[2].tolist() == [1, 2, 3, 0, 4]
    # disjoint cliques: all CC = 1, larger clique (higher degree) first, then by id
    o = load(oracle_lib, cliques([3, 5, 4]))
    assert o.node_stats()[2].tolist() == [3, 4, 5, 6, 7, 8, 9, 10, 11, 0, 1, 2]
    # a triangle with a pendant: 0-1-2 triangle, 2-3; CC(0)=CC(1)=1, CC(2)=1/3, CC(3)=0
    g = G.Graph(4, np.array([0, 1, 2, 2]), np.array([1, 2, 0, 3]))
    o = load(oracle_lib, g)
    tri, ccl, order = o.node_stats()
    assert ccl.tolist() == [1.0, 1.0, 1.0 / 3.0, 0.0]
    assert order.tolist() == [0, 1, 2, 3]
    for seed in range(10):
        g = G.random_gnp(30, 0.2, seed)
        o = load(oracle_lib, g)
        adj = brute.simple_graph(g.n, g.src, g.dst)
        ccx = brute.local_cc(adj, brute.triangles(adj))
        assert o.node_stats()[2].tolist() == brute.node_order(adj, ccx)


def test_initial_clustering_closed_forms(oracle_lib):
    """Greedy initial clustering in node order (Initial Clustering)."""
    o = load(oracle_lib, path(5))           # order 1,2,3,0,4: {1,0,2} then {3,4}
    assert memberships_list(o) == [[0], [0], [0], [1], [1]]
    o = load(oracle_lib, complete(6))
    assert memberships_list(o) == [[0]] * 6
    o = load(oracle_lib, star(7))           # hub first (highest degree): one community
    assert memberships_list(o) == [[0]] * 7
    for seed in range(20):
        g = G.random_gnp(25, 0.15, seed)
        o = load(oracle_lib, g)
        adj = brute.simple_graph(g.n, g.src, g.dst)
        order = brute.node_order(adj, brute.local_cc(adj, brute.triangles(adj)))
        P = brute.initial_clustering(adj, order)
        want = [[c for c, C in P.items() if x in C] for x in range(g.n)]
        assert memberships_list(o) == want


# ------------------------------------------------------------------ WCC-hat closed forms
@pytest.mark.parametrize("n", [3, 4, 5, 10, 17])
def test_complete_graph_closed_form(oracle_lib, n):
    """K_n as one community: every WCC-hat(x,C) = 1 so WCC-hat(P) = n; leaving changes it
    by exactly -3; nothing moves and the run stops after one iteration (rel = 0)."""
    o = load(oracle_lib, complete(n))
    sc = o.scores()
    assert sc["cc"] == 1.0 and sc["wcc_hat"] == float(n)
    for x in range(n):
        ev = o.eval_node(x)
        assert ev["cand"].tolist() == [0] and ev["is_leave"].tolist() == [True]
        assert ev["delta"][0] == -3.0
        assert ev["best_join"] == -1 and ev["best_leave"] == -1
    info = o.run_iterations(2, 0.01, 10, check_every_chunk=True)
    assert info["iterations"] == 1 and info["converged"]
    assert info["wtilde_hist"].tolist() == [float(n), float(n)]


def test_disjoint_cliques_closed_form(oracle_lib):
    """Disjoint cliques of size >= 3: WCC-hat(P) = total size; no join candidate exists and
    every leave is negative, so the run stops after one iteration."""
    g = cliques([3, 4, 6, 5])
    o = load(oracle_lib, g)
    assert o.scores()["wcc_hat"] == 18.0
    info = o.run_iterations(4, 0.01, 10, check_every_chunk=True)
    assert info["iterations"] == 1 and info["joins"].tolist() == [0] and info["leaves"].tolist() == [0]
    # ids follow the node order: the 6-clique (nodes 7-12) first, then 5, 4, 3
    assert memberships_list(o) == [[3]] * 3 + [[2]] * 4 + [[0]] * 6 + [[1]] * 5


@pytest.mark.parametrize("g", [path(9), star(8), cycle(10), G.Graph(3, np.zeros(0, np.int64), np.zeros(0, np.int64))])
def test_triangle_free_closed_form(oracle_lib, g):
    """No triangle: cc = 0, E[t(x,V)] = 0 for every node, WCC-hat = 0; no iteration runs."""
    o = load(oracle_lib, g)
    sc = o.scores()
    assert sc["triangles"] == 0 and sc["cc"] == 0.0 and sc["wcc_hat"] == 0.0
    info = o.run_iterations(3, 0.01, 10)
    assert info["iterations"] == 0 and info["converged"]


# ------------------------------------------------------------------ candidate changes vs exact rationals
def _exact_changes(adj, P, cc, x):
    base = brute.wcc_hat_partition(P, adj, cc)
    _, _, ch = brute._decide(x, P, adj, cc, base)
    return base, {(c, lv): d for c, lv, d in ch}


def test_candidate_changes_match_exact_rationals(oracle_lib):
    """Every join / leave change the oracle computes (cc-free, divided by cc) equals the
    exact WCC-hat(P') - WCC-hat(P) re-evaluated from the definition, within 1e-12."""
    checked = 0
    for seed in range(12):
        g = G.random_gnp(16, 0.35, 100 + seed)
        o = load(oracle_lib, g)
        adj = brute.simple_graph(g.n, g.src, g.dst)
        cc_o = o.scores()["cc"]
        cc = sum(brute.local_cc(adj, brute.triangles(adj)), Fraction(0)) / g.n
        if cc == 0:
            continue
        for rounds in range(2):
            mem = memberships_list(o)
            P = {}
            for x, cs in enumerate(mem):
                for c in cs:
                    P.setdefault(c, set()).add(x)
            for x in range(g.n):
                base, exact = _exact_changes(adj, P, cc, x)
                for mode in (0, 3):
                    ev = o.eval_node(x, mode=mode)
                    got = {(int(c), bool(lv)): d for c, lv, d in zip(ev["cand"], ev["is_leave"], ev["delta"])}
                    assert set(got) == set(exact)
                    for key, d in got.items():
                        want = float(exact[key])
                        assert abs(d / cc_o - want) <= 1e-12 * max(1.0, float(base)), (seed, x, key)
                        checked += 1
            o.run_iterations(4, 0.0, 1)     # advance one iteration, compare again
    assert checked > 500


# ------------------------------------------------------------------ full runs vs brute force
def _compare_runs(oracle_lib, g, q, threshold, mode, sequential=False, max_iters=15):
    b = brute.run(g.n, g.src, g.dst, q, threshold, max_iters, sequential=sequential)
    o = load(oracle_lib, g)
    info = o.run_iterations(q, threshold, max_iters, mode=mode, nthreads=2, check_every_chunk=True)
    if b["near_tie"]:
        return None
    assert memberships_list(o) == b["memberships"]
    assert info["iterations"] == b["iterations"]
    if b["history"][0] > 0:
        cc = o.scores()["cc"]
        for w_o, w_b in zip(info["wtilde_hist"], b["history"]):
            assert abs(w_o / cc - float(w_b)) <= 1e-12 * float(w_b)
    return True


def test_lazyfox_matches_brute_force(oracle_lib):
    """Algorithm 2 on tiny graphs, several queue sizes, both evaluation modes, against the
    exact re-evaluating brute force (skipping runs where FP64 may legitimately differ)."""
    done = 0
    for seed in range(20):
        g = G.random_gnp(15, 0.3, 1000 + seed)
        for q in (2, 5, 15):
            for mode in (0, 3):
                done += bool(_compare_runs(oracle_lib, g, q, 0.01, mode))
    assert done >= 100


def test_queue_size_one_is_fox(oracle_lib):
    """With a queue size of one LazyFox is Fox (Algorithm 1, sequential apply)."""
    done = 0
    for seed in range(20):
        g = G.random_gnp(14, 0.35, 2000 + seed)
        done += bool(_compare_runs(oracle_lib, g, 1, 0.01, 3, sequential=True))
    assert done >= 15


def test_planted_small_graph_vs_brute(oracle_lib):
    """A small planted-overlap graph (two communities sharing nodes) against brute force."""
    rng = np.random.default_rng(5)
    A = set(range(0, 12))
    B = set(range(8, 20))
    e = set()
    for C in (A, B):
        Cl = sorted(C)
        for i in range(len(Cl)):
            for j in range(i + 1, len(Cl)):
                if rng.random() < 0.5:
                    e.add((Cl[i], Cl[j]))
    e.add((0, 19))
    e = sorted(e)
    g = G.Graph(20, np.array([a for a, b in e]), np.array([b for a, b in e]))
    for q in (1, 4, 20):
        assert _compare_runs(oracle_lib, g, q, 0.01, 0) in (True, None)


# ------------------------------------------------------------------ self-consistency
def test_modes_threads_bit_identical_on_planted_graph(oracle_lib):
    """Naive and factored evaluation and any thread count give bit-identical results on the
    2,000-node planted graph (exact sums make every reduction order-free)."""
    g = G.named_config("tiny_sbm")
    outs = []
    for mode, nt in ((0, 1), (3, 1), (3, 8)):
        o = load(oracle_lib, g)
        info = o.run_iterations(64, 0.01, 6, mode=mode, nthreads=nt)
        off, ids = o.memberships()
        outs.append((info["iterations"], info["wtilde_hist"].tobytes(), off.tobytes(), ids.tobytes(),
                     o.in_counts().tobytes()))
    assert outs[0] == outs[1] == outs[2]


def test_state_invariants_every_chunk(oracle_lib):
    """After every chunk: sizes, internal edges, in-counts and exact sums equal a
    from-scratch recount; the community count never rises; a node gains at most one
    membership per iteration; removed communities have fewer than two members."""
    g = G.named_config("copurchase", scale=0.01)
    o = load(oracle_lib, g)
    prev_live = None
    prev = memberships_list(o)
    for it in range(4):
        info = o.run_iterations(32, 0.0, 1, mode=3, check_every_chunk=True)
        assert info["iterations"] == 1
        cur = memberships_list(o)
        for a, b in zip(prev, cur):
            assert len(set(b) - set(a)) <= 1 and len(set(a) - set(b)) <= 1
        s, m, W = o.communities()
        live = int((s >= 2).sum())
        assert not np.any(s == 1)
        if prev_live is not None:
            assert live <= prev_live
        prev_live = live
        prev = cur
    assert o.check_state() == 0


def test_relabel_equivalence(oracle_lib):
    """Dense relabelling is order-preserving: sparse ids give the dense graph's result."""
    g = G.named_config("copurchase", scale=0.005)
    o1 = load(oracle_lib, g)
    i1 = o1.run_iterations(16, 0.01, 5)
    ids = np.unique(np.concatenate([g.src, g.dst]))
    remap = np.full(g.n, -1, np.int64)
    remap[ids] = np.arange(ids.size) * 7 + 1000
    g2 = G.Graph(g.n, remap[g.src], remap[g.dst])
    o2 = oracle_lib.Oracle().load_graph(0, g2.src, g2.dst, relabel=True).init_communities(2)
    i2 = o2.run_iterations(16, 0.01, 5)
    dense = np.full(g.n, -1, np.int64)
    dense[ids] = np.arange(ids.size)
    m1 = memberships_list(o1)
    m2 = memberships_list(o2)
    assert i1["iterations"] == i2["iterations"]
    for x in ids:
        assert m1[x] == m2[dense[x]]


def test_bad_arguments(oracle_lib):
    o = oracle_lib.Oracle()
    with pytest.raises(oracle_lib.OracleError):
        o.run_iterations(4)                      # wrong call order
    o = load(oracle_lib, complete(4))
    for q, th in ((0, 0.01), (4, float("nan")), (4, -1.0)):
        with pytest.raises(oracle_lib.OracleError):
            o.run_iterations(q, th, 5)


def test_generator_is_deterministic():
    a = G.named_config("copurchase", seed=3, scale=0.01)
    b = G.named_config("copurchase", seed=3, scale=0.01)
    assert np.array_equal(a.src, b.src) and np.array_equal(a.dst, b.dst)
    c = G.named_config("copurchase", seed=4, scale=0.01)
    assert not (a.src.size == c.src.size and np.array_equal(a.src, c.src))


# ------------------------------------------------------------------ warm start
def random_cover(n, n_comms, seed, max_per_node=3):
    """Random overlapping cover with gaps in the ids, unsorted per node: (offsets, ids, P)."""
    rng = random.Random(seed)
    P = {}
    per = []
    for x in range(n):
        k = rng.randint(0, max_per_node)
        cs = rng.sample(range(n_comms), k)
        per.append(cs)
        for c in cs:
            P.setdefault(c, set()).add(x)
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum([len(c) for c in per])
    ids = np.array([c for cs in per for c in cs], np.int32)
    return off, ids, P


def test_warm_start_from_greedy_clustering_is_the_cold_start(oracle_lib):
    """Initial Clustering: inserting the greedy clustering as an existing division gives the
    same state and the same run as the greedy start itself."""
    g = G.named_config("tiny_sbm")
    cold = load(oracle_lib, g)
    off, ids = cold.memberships()
    K = cold.communities()[0].size
    warm = oracle_lib.Oracle().load_graph(g.n, g.src, g.dst).init_from_memberships(off, ids, K, 2)
    assert warm.check_state() == 0
    assert np.array_equal(warm.in_counts(), cold.in_counts())
    for a, b in zip(warm.communities(), cold.communities()):
        assert np.array_equal(a, b)
    assert warm.scores()["wtilde"] == cold.scores()["wtilde"]
    ia = cold.run_iterations(64, 0.01, 50)
    ib = warm.run_iterations(64, 0.01, 50)
    assert ia["iterations"] == ib["iterations"]
    assert np.array_equal(ia["wtilde_hist"], ib["wtilde_hist"])
    assert memberships_list(cold) == memberships_list(warm)


def test_warm_start_score_and_in_counts_match_exact_rationals(oracle_lib):
    """WCC-hat subsection: for random overlapping covers (empty and one-member communities
    included), the warm-started in-counts are |N(x) ∩ C| and the partition score is the
    exact rational WCC-hat (times cc) rounded once."""
    for seed in range(10):
        g = G.random_gnp(18, 0.3, 3000 + seed)
        off, ids, P = random_cover(g.n, 9, seed)
        o = oracle_lib.Oracle().load_graph(g.n, g.src, g.dst).init_from_memberships(off, ids, 12, 1)
        assert o.check_state() == 0
        adj = brute.simple_graph(g.n, g.src, g.dst)
        ooff, oids = o.memberships()
        inc = o.in_counts()
        for x in range(g.n):
            cs = oids[ooff[x]:ooff[x + 1]].tolist()
            assert cs == sorted(ids[off[x]:off[x + 1]].tolist())
            for c, i in zip(cs, inc[ooff[x]:ooff[x + 1]].tolist()):
                assert i == len(adj[x] & P[c])
        k = brute.triangles(adj)
        cc = sum(brute.local_cc(adj, k), Fraction(0)) / g.n
        w = brute.wcc_hat_partition(P, adj, cc)
        sc = o.scores()
        assert abs(sc["wtilde"] / sc["cc"] - float(w)) <= 1e-12 * float(w)


def test_warm_start_runs_match_brute_force(oracle_lib):
    """Algorithm 2 from random existing covers against the exact brute force."""
    done = 0
    for seed in range(15):
        g = G.random_gnp(15, 0.3, 4000 + seed)
        off, ids, P = random_cover(g.n, 8, 50 + seed, max_per_node=2)
        for q in (3, 15):
            b = brute.run(g.n, g.src, g.dst, q, 0.01, 15, initial=P)
            o = oracle_lib.Oracle().load_graph(g.n, g.src, g.dst).init_from_memberships(off, ids, -1, 1)
            info = o.run_iterations(q, 0.01, 15, mode=3, nthreads=2, check_every_chunk=True)
            if b["near_tie"]:
                continue
            assert memberships_list(o) == b["memberships"]
            assert info["iterations"] == b["iterations"]
            done += 1
    assert done >= 20


def test_resume_from_memberships_continues_the_run(oracle_lib):
    """Checkpoint and resume: stopping after k iterations and warm-starting from the
    memberships reached gives the uninterrupted run's remaining iterations (the state is a
    function of the memberships; the first resumed iteration compares with the score of the
    partition it starts from, which is the score the uninterrupted run reached)."""
    g = G.named_config("copurchase", scale=0.01)
    full = load(oracle_lib, g)
    fi = full.run_iterations(32, 0.001, 50)
    assert fi["iterations"] >= 4
    for k in (1, 3):
        part = load(oracle_lib, g)
        part.run_iterations(32, 0.001, k)
        off, ids = part.memberships()
        K = part.communities()[0].size
        res = oracle_lib.Oracle().load_graph(g.n, g.src, g.dst).init_from_memberships(off, ids, K, 2)
        assert res.scores()["wtilde"] == fi["wtilde_hist"][k]
        ri = res.run_iterations(32, 0.001, 50 - k)
        assert ri["iterations"] == fi["iterations"] - k
        assert ri["converged"] == fi["converged"] and ri["hit_max"] == fi["hit_max"]
        assert np.array_equal(ri["wtilde_hist"], fi["wtilde_hist"][k:])
        assert memberships_list(res) == memberships_list(full)


def test_warm_start_rejects_bad_covers(oracle_lib):
    g = G.random_gnp(10, 0.4, 1)
    o = oracle_lib.Oracle().load_graph(g.n, g.src, g.dst)
    off = np.arange(g.n + 1, dtype=np.int64)
    with pytest.raises(oracle_lib.OracleError):
        o.init_from_memberships(off, np.full(g.n, 5, np.int32), 3)          # id out of range
    dup = np.concatenate([[0], np.full(g.n, 2, np.int64)])
    with pytest.raises(oracle_lib.OracleError):
        o.init_from_memberships(dup, np.array([1, 1], np.int32), 3)        # node 0 lists 1 twice
    bad_total = off.copy()
    bad_total[-1] += 1
    with pytest.raises(oracle_lib.OracleError):
        o.init_from_memberships(bad_total, np.zeros(g.n, np.int32), 3)     # offsets[n] != total
    with pytest.raises(oracle_lib.OracleError):
        o.init_from_memberships(off[:-1].copy(), np.zeros(g.n - 1, np.int32), 3)   # n offsets


# ------------------------------------------------------------------ exact WCC
def _wcc_check(o, g, P):
    """Oracle WCC terms vs exact rationals for the cover P (dict id -> set) it holds."""
    adj = brute.simple_graph(g.n, g.src, g.dst)
    terms, vt, total = brute.wcc_exact(adj, P)
    r = o.exact_wcc(2)
    off, ids = o.memberships()
    assert np.array_equal(r["vt"], np.array(vt, np.int32))
    for x in range(g.n):
        for p in range(off[x], off[x + 1]):
            t, out, w = terms[(x, int(ids[p]))]
            assert r["t"][p] == t and r["vt_out"][p] == out
            assert abs(r["wcc_node"][p] - float(w)) <= 4e-16 * float(w)
    assert abs(r["wcc"] - float(total)) <= 1e-15 * float(total)
    for c, C in P.items():
        wc = sum((terms[(x, c)][2] for x in C), Fraction(0))
        assert abs(r["wcc_comm"][c] - float(wc)) <= 1e-15 * float(wc)
    return r


def test_exact_wcc_matches_rationals_on_random_covers(oracle_lib):
    """WCC paragraph: t(x,C), vt(x,V), vt(x,V\\C) from their set definitions, WCC(x,C) and
    WCC(P) as exact rationals, for random overlapping covers and for LazyFox results."""
    for seed in range(8):
        g = G.random_gnp(22, 0.35, 5000 + seed)
        off, ids, P = random_cover(g.n, 10, 70 + seed)
        o = oracle_lib.Oracle().load_graph(g.n, g.src, g.dst).init_from_memberships(off, ids, 10, 1)
        _wcc_check(o, g, P)
        o2 = load(oracle_lib, g)
        o2.run_iterations(4, 0.01, 20)
        off2, ids2 = o2.memberships()
        P2 = {}
        for x in range(g.n):
            for c in ids2[off2[x]:off2[x + 1]]:
                P2.setdefault(int(c), set()).add(x)
        _wcc_check(o2, g, P2)


def test_exact_wcc_closed_forms(oracle_lib):
    """Closed forms: a clique as one community rates every node 1 (WCC = n); disjoint
    cliques as communities likewise; a clique split into parts of a and n-a nodes rates a
    node of the first part C(a-1,2)/C(n-1,2); a triangle-free graph rates 0."""
    for n in (3, 5, 9):
        g = complete(n)
        o = oracle_lib.Oracle().load_graph(g.n, g.src, g.dst).init_from_memberships(
            np.arange(n + 1, dtype=np.int64), np.zeros(n, np.int32), 1, 1)
        r = o.exact_wcc(1)
        assert r["wcc"] == float(n) and np.all(r["wcc_node"] == 1.0)
    g = cliques([3, 4, 6])
    comm = np.repeat(np.arange(3), [3, 4, 6]).astype(np.int32)
    o = oracle_lib.Oracle().load_graph(g.n, g.src, g.dst).init_from_memberships(
        np.arange(g.n + 1, dtype=np.int64), comm, 3, 1)
    r = o.exact_wcc(1)
    assert r["wcc"] == 13.0 and list(r["wcc_comm"]) == [3.0, 4.0, 6.0]
    n, a = 10, 4
    g = complete(n)
    comm = np.array([0] * a + [1] * (n - a), np.int32)
    o = oracle_lib.Oracle().load_graph(g.n, g.src, g.dst).init_from_memberships(
        np.arange(n + 1, dtype=np.int64), comm, 2, 1)
    r = o.exact_wcc(1)
    b2 = lambda v: v * (v - 1) // 2
    assert np.all(r["wcc_node"][:a] == b2(a - 1) / b2(n - 1))
    assert np.all(r["wcc_node"][a:] == b2(n - a - 1) / b2(n - 1))
    for g in (cycle(12), star(8), path(9)):
        o = load(oracle_lib, g)
        r = o.exact_wcc(1)
        assert r["wcc"] == 0.0 and not r["t"].any() and not r["vt"].any()


def test_exact_wcc_bounds_and_sample(oracle_lib):
    """0 <= WCC(x,C) <= 1 (vt(x,V) <= |C\\{x}| + vt(x,V\\C)), t(x,C) <= t(x,V),
    vt(x,V\\C) <= vt(x,V); the per-node spot check equals the full pass."""
    g = G.named_config("copurchase", scale=0.01)
    o = load(oracle_lib, g)
    o.run_iterations(32, 0.01, 5)
    r = o.exact_wcc(4)
    off, ids = o.memberships()
    tri, _, _ = o.node_stats()
    node_of = np.repeat(np.arange(g.n), np.diff(off))
    assert np.all(r["wcc_node"] >= 0) and np.all(r["wcc_node"] <= 1.0)
    assert np.all(r["t"] <= tri[node_of]) and np.all(r["vt_out"] <= r["vt"][node_of])
    rng = np.random.default_rng(0)
    sample = rng.choice(g.n, 50, replace=False).astype(np.int32)
    wn, t, vo, vx = o.wcc_sample(sample)
    sel = np.concatenate([np.arange(off[x], off[x + 1]) for x in sample])
    assert np.array_equal(wn, r["wcc_node"][sel]) and np.array_equal(t, r["t"][sel])
    assert np.array_equal(vo, r["vt_out"][sel]) and np.array_equal(vx, r["vt"][sample])


# ------------------------------------------------------------------ post-processing
def cover_arrays(n, P):
    """(offsets, ids) of a cover given as dict id -> set of nodes."""
    per = [[] for _ in range(n)]
    for c in sorted(P):
        for x in P[c]:
            per[x].append(c)
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum([len(p) for p in per])
    return off, np.array([c for p in per for c in p], np.int32)


def nested_cover(n, seed):
    """Random communities plus planted duplicates (equal member sets, higher and lower ids),
    strict subsets and supersets, a chain A < B < C and a singleton."""
    rng = random.Random(seed)
    P = {}
    for c in range(12):
        P[c] = set(rng.sample(range(n), rng.randint(2, 8)))
    P[12] = set(P[3])                       # duplicate of 3 (higher id)
    P[13] = set(rng.sample(sorted(P[4]), max(1, len(P[4]) - 2)))   # strict subset of 4
    P[14] = P[5] | {rng.randrange(n)}       # superset (or duplicate) of 5
    a = set(rng.sample(range(n), 3))
    P[15], P[16], P[17] = a, a | {0, 1}, a | {0, 1, 2, 3}   # chain
    P[18] = set(P[16])                      # duplicate inside the chain
    P[19] = {rng.randrange(n)}              # one member
    return P


def expected_pp(P, dup, cont):
    keep, nd, nc = {}, 0, 0
    for a, A in P.items():
        d = dup and any(b < a and B == A for b, B in P.items() if b != a)
        s = cont and any(A < B for b, B in P.items() if b != a)
        keep[a] = not (d or s)
        nd += d
        nc += (s and not d)
    return keep, nd, nc


def test_postprocess_matches_set_definitions(oracle_lib):
    """Post-processing: duplicates (equal member sets, the lowest id stays) and strictly
    contained communities removed, each rule alone and both, against Python sets."""
    for seed in range(12):
        g = G.random_gnp(30, 0.2, 6000 + seed)
        P = nested_cover(g.n, seed)
        off, ids = cover_arrays(g.n, P)
        for dup, cont in ((True, True), (True, False), (False, True)):
            o = oracle_lib.Oracle().load_graph(g.n, g.src, g.dst).init_from_memberships(off, ids, 25, 1)
            keep, (nd, nc) = o.postprocess(dup, cont)
            ek, end, enc = expected_pp(P, dup, cont)
            assert (nd, nc) == (end, enc)
            for c in range(25):
                assert keep[c] == (1 if c in P and ek[c] else 0)


def test_postprocess_apply_rebuilds_the_cover(oracle_lib):
    """Applying the removal leaves exactly the kept communities, a consistent state, and
    the exact-rational WCC-hat of the remaining cover."""
    g = G.random_gnp(30, 0.25, 77)
    P = nested_cover(g.n, 3)
    off, ids = cover_arrays(g.n, P)
    o = oracle_lib.Oracle().load_graph(g.n, g.src, g.dst).init_from_memberships(off, ids, 25, 1)
    keep, _ = o.postprocess(True, True, apply=True)
    assert o.check_state() == 0
    Q = {c: C for c, C in P.items() if keep[c]}
    assert memberships_list(o) == [sorted(c for c, C in Q.items() if x in C) for x in range(g.n)]
    adj = brute.simple_graph(g.n, g.src, g.dst)
    k = brute.triangles(adj)
    cc = sum(brute.local_cc(adj, k), Fraction(0)) / g.n
    w = brute.wcc_hat_partition(Q, adj, cc)
    sc = o.scores()
    assert abs(sc["wtilde"] / sc["cc"] - float(w)) <= 1e-12 * float(w)
    keep2, rem2 = o.postprocess(True, True)
    assert rem2 == (0, 0) and np.array_equal(keep2, keep)


# ------------------------------------------------------------------ cover F1
def f1_exact(Pd, Pr):
    """F1-Score(P', P) from the paper's precision / recall form, as Fractions: (score,
    {c': (max F1, lowest reference id reaching it or -1)})."""
    per = {}
    for c, A in Pd.items():
        if not A:
            continue
        bestv, arg = Fraction(0), -1
        for r in sorted(Pr):
            B = Pr[r]
            i = len(A & B)
            if not B or i == 0:
                continue
            p, q = Fraction(i, len(A)), Fraction(i, len(B))
            f = 2 * p * q / (p + q)
            if arg < 0 or f > bestv:
                bestv, arg = f, r
        per[c] = (bestv, arg)
    score = sum((v[0] for v in per.values()), Fraction(0)) / len(per) if per else Fraction(0)
    return score, per


def test_cover_f1_matches_rationals(oracle_lib):
    """F1-Score for Overlapping Communities: every community's best match and the average
    against exact rationals, for random and LazyFox covers against random and planted
    reference covers."""
    for seed in range(8):
        g = G.random_gnp(40, 0.2, 7000 + seed)
        off, ids, Pd = random_cover(g.n, 15, 80 + seed)
        roff, rids, Pr = random_cover(g.n, 12, 90 + seed, max_per_node=2)
        for lazy in (False, True):
            if lazy:
                o = load(oracle_lib, g)
                o.run_iterations(8, 0.01, 20)
                mo, mi = o.memberships()
                Pd = {}
                for x in range(g.n):
                    for c in mi[mo[x]:mo[x + 1]]:
                        Pd.setdefault(int(c), set()).add(x)
            else:
                o = oracle_lib.Oracle().load_graph(g.n, g.src, g.dst).init_from_memberships(off, ids, 15, 1)
            f1, best, match = o.cover_f1(roff, rids)
            score, per = f1_exact(Pd, Pr)
            assert f1 == math.fsum(float(v[0]) for v in per.values()) / max(1, len(per))
            assert abs(f1 - float(score)) <= 1e-15 * max(1.0, float(score))
            for c in range(best.size):
                if c in per:
                    assert best[c] == float(per[c][0]) and match[c] == per[c][1]
                else:
                    assert best[c] == 0.0 and match[c] == -1


def test_cover_f1_closed_forms(oracle_lib):
    """Identical covers score 1; communities that are parts of one reference community of
    all n nodes score 2s/(s+n) each; a reference meeting nothing scores 0; bad covers are
    refused."""
    g = G.named_config("tiny_sbm")
    o = load(oracle_lib, g)
    off, ids = o.memberships()
    assert o.cover_f1(off, ids)[0] == 1.0
    g = cliques([3, 4, 6])
    comm = np.repeat(np.arange(3), [3, 4, 6]).astype(np.int32)
    o = oracle_lib.Oracle().load_graph(g.n, g.src, g.dst).init_from_memberships(
        np.arange(g.n + 1, dtype=np.int64), comm, 3, 1)
    f1, best, match = o.cover_f1(np.arange(g.n + 1, dtype=np.int64), np.zeros(g.n, np.int32))
    assert list(best) == [6 / 16, 8 / 17, 12 / 19] and list(match) == [0, 0, 0]
    assert f1 == math.fsum([6 / 16, 8 / 17, 12 / 19]) / 3
    f1, best, match = o.cover_f1(np.zeros(g.n + 1, np.int64), np.zeros(0, np.int32))
    assert f1 == 0.0 and not best.any() and np.all(match == -1)
    dup = np.concatenate([[0], np.full(g.n, 2, np.int64)])
    with pytest.raises(oracle_lib.OracleError):
        o.cover_f1(dup, np.array([1, 1], np.int32))


def test_queue_prefix_runs_stop_after_the_stated_queues(oracle_lib):
    """Timing samples (run_queue_prefix): the first k queues of iteration 1 are evaluated
    and applied exactly as in the full run, and the run stops there.  The prefix state
    passes the from-scratch state check, and applying the same prefix with the factored
    mode at several threads gives the same memberships as the naive mode at one."""
    g = G.named_config("tiny_sbm")
    covers = []
    for mode, threads in ((oracle_lib.MODE_NAIVE, 1), (oracle_lib.MODE_FAST, 4)):
        o = load(oracle_lib, g)
        assert o.run_queue_prefix(64, 5, mode=mode, nthreads=threads) == 5
        assert o.check_state() == 0
        covers.append(o.memberships())
    assert np.array_equal(covers[0][0], covers[1][0]) and np.array_equal(covers[0][1], covers[1][1])
    o = load(oracle_lib, g)
    # a limit beyond the queues of one iteration ends with that iteration
    assert o.run_queue_prefix(64, 10_000) == (g.n + 63) // 64
    full = load(oracle_lib, g)
    full.run_iterations(64, 0.0, 1)
    assert np.array_equal(o.memberships()[1], full.memberships()[1])
