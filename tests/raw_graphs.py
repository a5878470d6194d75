"""Hypothesis strategy of tiny raw edge lists for the property tests (test input only: it
draws graphs and holds no part of the method)."""
import numpy as np
from hypothesis import HealthCheck, settings
from hypothesis import strategies as st

import graphgen as G


@st.composite
def edge_lists(draw, max_n=12, max_pairs=40):
    """A simple graph drawn with a drawn density (so triangles are common), then written
    out as a raw list: each edge in a drawn direction, some edges repeated, some
    self-loops added."""
    n = draw(st.integers(1, max_n))
    every = [(a, b) for a in range(n) for b in range(a + 1, n)]
    if every:
        density = draw(st.sampled_from([0.15, 0.3, 0.5, 0.8]))
        u = draw(st.lists(st.floats(0.0, 1.0), min_size=len(every), max_size=len(every)))
        edges = [e for e, ue in zip(every, u) if ue < density]
    else:
        edges = []
    edges = edges[:max_pairs]
    flip = draw(st.lists(st.booleans(), min_size=len(edges), max_size=len(edges)))
    pairs = [(b, a) if f else (a, b) for (a, b), f in zip(edges, flip)]
    if edges:
        pairs += draw(st.lists(st.sampled_from(pairs), max_size=4))
    pairs += [(x, x) for x in draw(st.lists(st.integers(0, n - 1), max_size=2))]
    order = draw(st.permutations(range(len(pairs))))
    pairs = [pairs[i] for i in order]
    src = np.array([a for a, b in pairs], np.int64)
    dst = np.array([b for a, b in pairs], np.int64)
    return G.Graph(n, src, dst)


SETTINGS = settings(max_examples=150, deadline=None, derandomize=True, database=None,
                    suppress_health_check=[HealthCheck.too_slow])


@st.composite
def covers(draw, n, max_comms=8, max_per_node=3):
    """A cover of n nodes as a dict community id -> set of nodes: each node lists up to
    max_per_node distinct ids drawn from [0, max_comms), in drawn order."""
    k = draw(st.integers(1, max_comms))
    per = [draw(st.lists(st.integers(0, k - 1), max_size=max_per_node, unique=True)) for _ in range(n)]
    P = {}
    for x, cs in enumerate(per):
        for c in cs:
            P.setdefault(c, set()).add(x)
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum([len(cs) for cs in per])
    ids = np.array([c for cs in per for c in cs], np.int32)
    return k, off, ids, P
