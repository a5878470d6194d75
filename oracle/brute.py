"""Exact-rational brute force for tiny graphs (TEST INFRASTRUCTURE ONLY).

Everything is recomputed from scratch from the paper's own formulas with
``fractions.Fraction`` -- no maintained state, no factoring, no floating point in any
decision:

* triangles k_i by checking every node triple; the local clustering coefficient
  CC(i) = k_i / (d_i (d_i - 1) / 2) (0 when d_i <= 1) and the node order by decreasing CC,
  ties by decreasing degree (Methods, "Node Order"), then by increasing id;
* the global cc as the mean of all local CCs (WCC-hat subsection);
* the greedy initial clustering (Methods, "Initial Clustering");
* WCC-hat(x, C) = E[t(x,C)] / E[t(x,V)] * deg(x,V) / (|C \\ {x}| + deg(x, V \\ C)) with
  E[t(x,C)] = C(deg(x,C), 2) p, E[t(x,V)] = C(deg(x,V), 2) cc and p the community's
  density, 0 when E[t(x,V)] = 0; WCC-hat(C) and WCC-hat(P) as plain sums;
* a join / leave change is the difference WCC-hat(P') - WCC-hat(P) of two full
  re-evaluations of the partition (Methods, "Node Changes");
* Fox (Algorithm 1: decide and apply node by node) and LazyFox (Algorithm 2: a queue of q
  nodes decided on one partition, then applied together), the relative stopping test and
  the removal of communities with fewer than two members after every iteration.

Only usable for graphs of a few dozen nodes.
"""
from __future__ import annotations

from fractions import Fraction
from itertools import combinations


def simple_graph(n, src, dst):
    """Adjacency sets: self-loops dropped, duplicate edges merged (Methods, Preprocessing)."""
    adj = [set() for _ in range(n)]
    for a, b in zip(src, dst):
        a, b = int(a), int(b)
        if a != b:
            adj[a].add(b)
            adj[b].add(a)
    return adj


def triangles(adj):
    n = len(adj)
    k = [0] * n
    for a, b, c in combinations(range(n), 3):
        if b in adj[a] and c in adj[a] and c in adj[b]:
            k[a] += 1
            k[b] += 1
            k[c] += 1
    return k


def local_cc(adj, k):
    out = []
    for x, nb in enumerate(adj):
        d = len(nb)
        out.append(Fraction(k[x], d * (d - 1) // 2) if d > 1 else Fraction(0))
    return out


def node_order(adj, ccl):
    return sorted(range(len(adj)), key=lambda x: (-ccl[x], -len(adj[x]), x))


def initial_clustering(adj, order):
    comm_of = [-1] * len(adj)
    P = {}
    for x in order:
        if comm_of[x] >= 0:
            continue
        c = len(P)
        P[c] = {x}
        comm_of[x] = c
        for y in adj[x]:
            if comm_of[y] < 0:
                comm_of[y] = c
                P[c].add(y)
    return P


def binom2(v):
    return Fraction(v * (v - 1), 2)


def wcc_hat_node(x, C, adj, cc):
    d = len(adj[x])
    i = len(adj[x] & C)
    s = len(C)
    m = sum(len(adj[y] & C) for y in C) // 2
    p = Fraction(2 * m, s * (s - 1)) if s >= 2 else Fraction(0)
    et_xc = binom2(i) * p
    et_xv = binom2(d) * cc
    if et_xv == 0:
        return Fraction(0)
    return et_xc / et_xv * Fraction(d, (s - 1) + (d - i))


def wcc_hat_partition(P, adj, cc):
    return sum((wcc_hat_node(x, C, adj, cc) for C in P.values() for x in C), Fraction(0))


def _decide(x, P, adj, cc, base):
    """Best join and best leave of x on partition P (exact), plus all candidate changes."""
    mine = [c for c, C in P.items() if x in C]
    near = sorted({c for c, C in P.items() if x not in C and (adj[x] & C)})
    changes = []
    best_join, best_jd = -1, None
    for c in near:
        Q = dict(P)
        Q[c] = P[c] | {x}
        d = wcc_hat_partition(Q, adj, cc) - base
        changes.append((c, False, d))
        if d > 0 and (best_jd is None or d > best_jd):
            best_join, best_jd = c, d
    best_leave, best_ld = -1, None
    for c in sorted(mine):
        Q = dict(P)
        Q[c] = P[c] - {x}
        d = wcc_hat_partition(Q, adj, cc) - base
        changes.append((c, True, d))
        if d > 0 and (best_ld is None or d > best_ld):
            best_leave, best_ld = c, d
    return best_join, best_leave, changes


def _near_tie(changes, scale):
    """True if FP64 could legitimately decide differently: a change within 1e-12*scale of 0,
    or two competing positive changes within 1e-12*scale of each other."""
    eps = Fraction(1, 10 ** 12) * max(scale, Fraction(1))
    for leave in (False, True):
        vals = sorted(d for c, lv, d in changes if lv == leave)
        for v in vals:
            if v != 0 and abs(v) < eps:
                return True
            if v == 0:
                continue
        pos = [v for v in vals if v > 0]
        for a, b in zip(pos, pos[1:]):
            if b - a < eps:
                return True
    return False


def _apply(P, x, join, leave):
    if leave >= 0:
        P[leave] = P[leave] - {x}
    if join >= 0:
        P[join] = P[join] | {x}


def _end_iteration(P):
    for c in list(P):
        if len(P[c]) < 2:
            del P[c]


def run(n, src, dst, queue_size, threshold=0.01, max_iters=50, sequential=False, initial=None):
    """LazyFox (or Fox with sequential=True) on a tiny graph, exactly.  ``initial`` (a dict
    community id -> set of nodes) replaces the greedy initial clustering (warm start).

    Returns dict(memberships (per node sorted community ids), iterations, history of
    WCC-hat(P) (Fractions), cc, order, triangles, near_tie flag).
    """
    adj = simple_graph(n, src, dst)
    k = triangles(adj)
    ccl = local_cc(adj, k)
    cc = sum(ccl, Fraction(0)) / n if n else Fraction(0)
    order = node_order(adj, ccl)
    P = initial_clustering(adj, order) if initial is None else {c: set(C) for c, C in initial.items()}
    hist = [wcc_hat_partition(P, adj, cc) if cc > 0 else Fraction(0)]
    near_tie = False
    its = 0
    theta = Fraction(threshold)
    if cc > 0:
        for _ in range(max_iters):
            if sequential:
                # Algorithm 1: each node's best leave and best join are applied before
                # the next node is considered
                for x in order:
                    base = wcc_hat_partition(P, adj, cc)
                    j, l, ch = _decide(x, P, adj, cc, base)
                    near_tie |= _near_tie(ch, base)
                    _apply(P, x, j, l)
            else:
                # Algorithm 2: a queue of q nodes is decided on the same partition, then
                # all changes are applied together
                for s in range(0, n, queue_size):
                    chunk = order[s:s + queue_size]
                    base = wcc_hat_partition(P, adj, cc)
                    dec = []
                    for x in chunk:
                        j, l, ch = _decide(x, P, adj, cc, base)
                        near_tie |= _near_tie(ch, base)
                        dec.append((x, j, l))
                    for x, j, l in dec:
                        _apply(P, x, j, l)
            _end_iteration(P)
            its += 1
            w = wcc_hat_partition(P, adj, cc)
            prev = hist[-1]
            hist.append(w)
            if prev == 0 or (w - prev) / prev < theta:
                if prev != 0 and abs((w - prev) / prev - theta) < Fraction(1, 10 ** 12):
                    near_tie = True
                break
    mem = [sorted(c for c, C in P.items() if x in C) for x in range(n)]
    return dict(memberships=mem, iterations=its, history=hist, cc=cc, order=order,
                triangles=k, near_tie=near_tie, partition=P, adj=adj)


def wcc_exact(adj, P):
    """WCC of cover P (dict id -> set of nodes) from its definition (WCC paragraph of the
    WCC-hat subsection), exactly: per membership (x, C) the tuple (t(x,C), vt(x, V\\C),
    WCC(x,C) as a Fraction), vt(x, V) per node, and WCC(P)."""
    n = len(adj)
    tri = triangles(adj)
    closes = [{y for y in adj[x] if adj[x] & adj[y]} for x in range(n)]
    terms = {}
    for c, C in P.items():
        for x in C:
            t = sum(1 for y in adj[x] & C for z in adj[x] & C if y < z and z in adj[y])
            out = len(closes[x] - C)
            w = Fraction(t, tri[x]) * Fraction(len(closes[x]), len(C) - 1 + out) if tri[x] else Fraction(0)
            terms[(x, c)] = (t, out, w)
    return terms, [len(s) for s in closes], sum((v[2] for v in terms.values()), Fraction(0))
