"""Seeded synthetic graph generators (shared input source for the oracle and the GPU path).

This module holds no part of the community-detection method: it only draws edge lists.
Every generator is a pure function of its parameters and an integer seed
(numpy PCG64), so the oracle and the GPU library can be fed the same bytes.

Workloads (stand-ins for the paper's SNAP inputs, which are not reproduced):

* ``planted_sbm``   overlapping stochastic block model (small parity graph, 2,000 nodes);
* ``planted_powerlaw``  LFR-style planted-overlap graph: power-law degrees, power-law
  community sizes, several memberships per node, mixing parameter mu;
* ``serving_mix``   a Poisson-arriving stream of small planted power-law graphs.

Edge lists are returned raw (int64 ``src``, ``dst``): they may contain duplicate edges
and both directions of an edge, which the consumers must remove (the paper's input is a
possibly multi-edge list that preprocessing turns into a simple graph).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Graph", "planted_sbm", "planted_powerlaw", "serving_mix", "named_config",
    "CONFIGS", "random_gnp", "solve_cutoff",
]


@dataclasses.dataclass
class Graph:
    n: int
    src: np.ndarray          # int64 [npairs]
    dst: np.ndarray          # int64 [npairs]
    planted: list | None = None   # planted communities (list of int64 arrays), for reference only
    meta: dict = dataclasses.field(default_factory=dict)
    planted_pairs: tuple | None = None   # planted memberships as (node, community) int64 arrays

    def planted_cover(self):
        """Planted memberships as (offsets int64[n + 1], community ids int32), per node in
        ascending id order; None if the generator plants none."""
        if self.planted_pairs is None:
            return None
        node, comm = self.planted_pairs
        o = np.lexsort((comm, node))
        off = np.zeros(self.n + 1, np.int64)
        np.cumsum(np.bincount(node, minlength=self.n), out=off[1:])
        return off, comm[o].astype(np.int32)

    @property
    def npairs(self) -> int:
        return int(self.src.shape[0])

    def simple_edge_count(self) -> int:
        a = np.minimum(self.src, self.dst)
        b = np.maximum(self.src, self.dst)
        keep = a != b
        key = a[keep] * np.int64(self.n) + b[keep]
        return int(np.unique(key).shape[0])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def random_gnp(n: int, p: float, seed: int) -> Graph:
    """Erdos-Renyi G(n, p) (small test graphs)."""
    rng = _rng(seed)
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.shape[0]) < p
    return Graph(n, iu[keep].astype(np.int64), ju[keep].astype(np.int64))


# ---------------------------------------------------------------- power-law helpers
def _pareto_floor(rng, size, expo, lo, hi):
    """floor of a continuous power law x^-expo on [lo, hi+1) (inverse-CDF draw)."""
    u = rng.random(size)
    a = 1.0 - expo
    x = (lo ** a + u * ((hi + 1.0) ** a - lo ** a)) ** (1.0 / a)
    return np.minimum(np.floor(x), hi).astype(np.int64)


def _pareto_mean(expo, lo, hi):
    # mean of floor(x) for x ~ power law on [lo, hi+1): integrate piecewise per integer cell
    a = 1.0 - expo
    z = (hi + 1.0) ** a - lo ** a
    ks = np.arange(int(math.floor(lo)), int(hi) + 1, dtype=np.float64)
    lo_k = np.maximum(ks, lo)
    hi_k = ks + 1.0
    mass = (hi_k ** a - lo_k ** a) / z
    return float(np.sum(ks * mass))


def solve_cutoff(expo: float, dmax: int, target_mean: float, lo_bound: float = 1.0) -> float:
    """Real-valued lower cutoff c such that E[floor(x)] = target_mean, x ~ x^-expo on [c, dmax+1)."""
    lo, hi = lo_bound, float(dmax)
    if _pareto_mean(expo, lo, dmax) >= target_mean:
        return lo
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        if _pareto_mean(expo, mid, dmax) < target_mean:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def _pair_stubs(rng, owner, group):
    """Configuration model: random perfect matching of stubs inside each group.

    owner: node id of each stub; group: group id of each stub (same length).
    Returns (u, v) arrays of matched stub owners (one unmatched stub per odd group dropped).
    """
    if owner.size == 0:
        e = np.zeros(0, np.int64)
        return e, e
    key = rng.random(owner.size)
    order = np.lexsort((key, group))
    g = group[order]
    o = owner[order]
    start = np.ones(g.size, dtype=bool)
    start[1:] = g[1:] != g[:-1]
    first = np.maximum.accumulate(np.where(start, np.arange(g.size), 0))
    rel = np.arange(g.size) - first
    left = (rel % 2 == 0)
    has_right = np.zeros(g.size, dtype=bool)
    has_right[:-1] = (g[1:] == g[:-1])
    left &= has_right
    idx = np.nonzero(left)[0]
    return o[idx], o[idx + 1]


def _assign_memberships(rng, n, mcount, sizes):
    """Pair membership stubs of nodes with community slots (LFR style, no duplicates).

    Returns (node, comm) membership pairs.
    """
    node_stubs = np.repeat(np.arange(n, dtype=np.int64), mcount)
    comm_slots = np.repeat(np.arange(sizes.size, dtype=np.int64), sizes)
    tot = min(node_stubs.size, comm_slots.size)
    node_stubs = rng.permutation(node_stubs)[:tot]
    comm_slots = rng.permutation(comm_slots)[:tot]
    key = node_stubs * np.int64(sizes.size) + comm_slots
    key = np.unique(key)
    return key // sizes.size, key % sizes.size


def _membership_matrix(n, mnode, mcomm, width):
    order = np.lexsort((mcomm, mnode))
    mnode, mcomm = mnode[order], mcomm[order]
    counts = np.bincount(mnode, minlength=n)
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
    pos = np.arange(mnode.size) - starts[mnode]
    M = np.full((n, width), -1, dtype=np.int64)
    keep = pos < width
    M[mnode[keep], pos[keep]] = mcomm[keep]
    return M, counts


def planted_powerlaw(n, target_edges, deg_exp, deg_max, deg_min_floor, mem_max, size_exp,
                     size_min, size_max, mu, seed, mem_ratio=0.5, excess=1.04, cap_intra=False):
    """LFR-style planted-overlap graph with power-law degrees and community sizes.

    1. degrees: floor of a continuous power law (exponent deg_exp, max deg_max); the lower
       cutoff is solved so that the mean degree reaches 2*target_edges/n (the edge count is
       the binding constraint);
    2. memberships per node: truncated geometric on 1..mem_max (ratio mem_ratio);
    3. community sizes: power law (size_exp) on [size_min, size_max], summing to the
       membership count; memberships paired with community slots at random;
    4. (1-mu)*d intra stubs split over the node's communities, matched by a configuration
       model inside each community; mu*d inter stubs matched globally, pairs that share a
       community rejected.  With cap_intra a node's stubs in a community are capped at the
       community's size minus one and the rest become inter stubs, so that a hub whose
       communities are smaller than its degree still realises its degree.
    """
    rng = _rng(seed)
    target_mean = 2.0 * target_edges / n * excess   # excess: multi-edges are dropped later
    cut = solve_cutoff(deg_exp, deg_max, target_mean, lo_bound=float(deg_min_floor))
    deg = _pareto_floor(rng, n, deg_exp, cut, deg_max)

    ms = np.arange(1, mem_max + 1)
    pm = mem_ratio ** (ms - 1.0)
    pm /= pm.sum()
    mcount = rng.choice(ms, size=n, p=pm).astype(np.int64)
    total = int(mcount.sum())
    smax = min(size_max, n)
    smin = min(size_min, smax)
    sizes = []
    acc = 0
    while acc < total:
        s = _pareto_floor(rng, 4096, size_exp, float(smin), smax)
        c = np.cumsum(s) + acc
        k = int(np.searchsorted(c, total, side="left"))
        if k < s.size:
            sizes.append(s[:k + 1])
            acc = int(c[k])
            break
        sizes.append(s)
        acc = int(c[-1])
    sizes = np.concatenate(sizes)
    mnode, mcomm = _assign_memberships(rng, n, mcount, sizes)
    M, mc = _membership_matrix(n, mnode, mcomm, mem_max)

    # intra stubs, split evenly over the node's communities (first ones get the remainder)
    intra = np.rint((1.0 - mu) * deg).astype(np.int64)
    intra = np.where(mc > 0, intra, 0)
    inter = deg - intra
    mcs = np.maximum(mc, 1)
    base = intra // mcs
    rem = intra % mcs
    stub_owner = []
    stub_group = []
    for j in range(mem_max):
        has = mc > j
        cnt = np.where(has, base + (j < rem), 0)
        if cap_intra:
            room = np.where(has, sizes[np.maximum(M[:, j], 0)] - 1, 0)
            over = np.maximum(cnt - room, 0)
            cnt = cnt - over
            inter = inter + over
        owners = np.repeat(np.arange(n, dtype=np.int64), cnt)
        stub_owner.append(owners)
        stub_group.append(M[owners, j])
    u1, v1 = _pair_stubs(rng, np.concatenate(stub_owner), np.concatenate(stub_group))

    owners = np.repeat(np.arange(n, dtype=np.int64), inter)
    u2, v2 = _pair_stubs(rng, owners, np.zeros(owners.size, np.int64))
    share = np.zeros(u2.size, dtype=bool)
    for a in range(mem_max):
        ca = M[u2, a]
        for b in range(mem_max):
            share |= (ca >= 0) & (ca == M[v2, b])
    u2, v2 = u2[~share], v2[~share]

    src = np.concatenate([u1, u2])
    dst = np.concatenate([v1, v2])
    perm = rng.permutation(src.size)
    src, dst = src[perm], dst[perm]
    # both directions present for a random half of the pairs (exercises dedup/canonicalisation)
    flip = rng.random(src.size) < 0.5
    src, dst = np.where(flip, dst, src), np.where(flip, src, dst)
    meta = dict(kind="planted_powerlaw", n=n, deg_exp=deg_exp, deg_max=deg_max, cutoff=cut,
                mem_max=mem_max, size_exp=size_exp, size_min=smin, size_max=smax, mu=mu,
                seed=seed, communities=int(sizes.size), raw_pairs=int(src.size))
    return Graph(n, src.astype(np.int64), dst.astype(np.int64), None, meta,
                 (mnode.astype(np.int64), mcomm.astype(np.int64)))


def planted_sbm(n=2000, ncomm=20, size_lo=50, size_hi=200, p_two=0.2, p_in=0.15, mix=0.2, seed=0):
    """Overlapping stochastic block model.

    ncomm communities with sizes U{size_lo..size_hi}; each node is in 1 community (prob
    1-p_two) or 2 (prob p_two); every pair inside a community is an edge with prob p_in;
    random pairs that share no community are added until inter/(intra+inter) = mix.
    """
    rng = _rng(seed)
    sizes = rng.integers(size_lo, size_hi + 1, size=ncomm).astype(np.int64)
    mcount = np.where(rng.random(n) < p_two, 2, 1).astype(np.int64)
    total = int(mcount.sum())
    # rescale the community sizes to the membership count (keeps U-shape proportions)
    scaled = np.maximum(2, np.floor(sizes * (total / sizes.sum()))).astype(np.int64)
    while scaled.sum() < total:
        scaled[rng.integers(0, ncomm)] += 1
    mnode, mcomm = _assign_memberships(rng, n, mcount, scaled)
    M, _ = _membership_matrix(n, mnode, mcomm, 2)
    planted = [mnode[mcomm == c] for c in range(ncomm)]
    us, vs = [], []
    for members in planted:
        members = np.sort(members)
        iu, ju = np.triu_indices(members.size, 1)
        keep = rng.random(iu.size) < p_in
        us.append(members[iu[keep]])
        vs.append(members[ju[keep]])
    u1, v1 = np.concatenate(us), np.concatenate(vs)
    key = np.unique(np.minimum(u1, v1) * n + np.maximum(u1, v1))
    intra = key.size
    want_inter = int(round(intra * mix / (1.0 - mix)))
    got = []
    have = 0
    while have < want_inter:
        a = rng.integers(0, n, size=2 * (want_inter - have) + 64)
        b = rng.integers(0, n, size=a.size)
        share = (a == b)
        for i in range(2):
            for j in range(2):
                share |= (M[a, i] >= 0) & (M[a, i] == M[b, j])
        a, b = a[~share], b[~share]
        k = np.unique(np.minimum(a, b) * n + np.maximum(a, b))
        k = np.setdiff1d(k, key)
        if got:
            k = np.setdiff1d(k, np.concatenate(got))
        k = rng.permutation(k)[: want_inter - have]
        got.append(k)
        have += k.size
    inter_keys = np.concatenate(got) if got else np.zeros(0, np.int64)
    allk = np.concatenate([key, inter_keys])
    allk = rng.permutation(allk)
    src, dst = allk // n, allk % n
    flip = rng.random(src.size) < 0.5
    src, dst = np.where(flip, dst, src), np.where(flip, src, dst)
    meta = dict(kind="planted_sbm", n=n, ncomm=ncomm, p_in=p_in, mix=mix, seed=seed,
                intra=int(intra), inter=int(inter_keys.size))
    return Graph(n, src.astype(np.int64), dst.astype(np.int64), planted, meta,
                 (mnode.astype(np.int64), mcomm.astype(np.int64)))


# ---------------------------------------------------------------- named workloads
CONFIGS = {
    # 2,000 nodes, 20 overlapping communities (50-200), 1-2 memberships (0.8/0.2),
    # intra-edge probability 0.15, inter/(intra+inter) = 0.2; queue 64
    "tiny_sbm": dict(queue=64),
    # co-purchase-shaped: 335,000 nodes, ~926,000 edges, exponent 2.5, max 550,
    # memberships 1-3, community sizes power law 1.5 on [5, 500], mixing 0.3; queue 256
    "copurchase": dict(queue=256),
    # social-shaped: 4,000,000 nodes, ~35,000,000 edges, exponent 2.3, min >= 2, max 15,000,
    # memberships 1-4, sizes [10, 3000], mixing 0.4; queue swept 1k-64k
    "social": dict(queue=4096),
    # dense heavy-tail: 3,000,000 nodes, ~117,000,000 edges, exponent 2.1, max 33,000,
    # memberships 1-5, sizes [10, 3000], mixing 0.5
    "dense": dict(queue=16384),
}


def named_config(name: str, seed: int = 0, scale: float = 1.0) -> Graph:
    """Build a named workload. ``scale`` < 1 shrinks node and edge counts proportionally
    (same degree law and structure) for quick tests."""
    if name == "tiny_sbm":
        return planted_sbm(seed=seed)
    if name == "copurchase":
        n = max(1000, int(335_000 * scale))
        return planted_powerlaw(n, 926_000 * n / 335_000, 2.5, 550, 1, 3, 1.5, 5, 500, 0.3, seed,
                                excess=1.133)
    if name == "social":
        n = max(1000, int(4_000_000 * scale))
        return planted_powerlaw(n, 35_000_000 * n / 4_000_000, 2.3, 15_000, 2, 4, 1.5, 10, 3000,
                                0.4, seed, excess=1.10, cap_intra=True)
    if name == "dense":
        n = max(1000, int(3_000_000 * scale))
        return planted_powerlaw(n, 117_000_000 * n / 3_000_000, 2.1, 33_000, 2, 5, 1.5, 10, 3000,
                                0.5, seed, excess=1.2)
    raise KeyError(name)


def serving_mix(n_jobs=10_000, rate=200.0, seed=0):
    """Poisson-arriving serving jobs: list of (arrival_s, job_params).

    Node count lognormal(median 2,000, sigma 1.2) clipped to [50, 200,000]; mean degree
    U[8, 40]; mixing U[0.2, 0.4]; degree exponent 2.5 with max min(n-1, 1000);
    memberships 1-3; community sizes power law 1.5 on [5, min(500, n/2)].
    The per-job queue size depends only on the job: clamp(2^round(log2(n/32)), 16, 4096).
    """
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_jobs)
    arrivals = np.cumsum(gaps)
    ns = np.clip(np.exp(rng.normal(math.log(2000.0), 1.2, size=n_jobs)), 50, 200_000).astype(int)
    degs = rng.uniform(8, 40, size=n_jobs)
    mus = rng.uniform(0.2, 0.4, size=n_jobs)
    jobs = []
    for j in range(n_jobs):
        n = int(ns[j])
        q = int(min(4096, max(16, 2 ** round(math.log2(n / 32.0)))))
        jobs.append(dict(job=j, arrival=float(arrivals[j]), n=n, mean_deg=float(degs[j]),
                         mu=float(mus[j]), queue=q, seed=j))
    return jobs


def serving_job_graph(job: dict) -> Graph:
    n = job["n"]
    dmax = int(min(n - 1, 1000))
    smax = int(max(5, min(500, n // 2)))
    return planted_powerlaw(n, job["mean_deg"] * n / 2.0, 2.5, dmax, 1, 3, 1.5, min(5, smax), smax,
                            job["mu"], 1_000_003 + job["seed"])
