"""GPU parity on arbitrary tiny raw edge lists (hypothesis; duplicates, both directions,
self-loops, isolated nodes, n from 1).  For each drawn graph and queue size the HIP path
and the oracle must agree bit for bit on the CSR, the node statistics, the initial
clustering, the whole run (score history, move counts, memberships, in-counts, community
table), the exact WCC of the final cover, its post-processing flags and its F1 against the
initial clustering."""
import sys

import numpy as np
import pytest
from hypothesis import given
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
