"""Failure handling of the C ABI on the GPU library, forced from the host: caller buffers
that are too small, a serving job larger than the whole device budget, the integer-range
guards of the graph loader, and a run that stops at max_iters.  Every case either fails
before any kernel is launched or runs ordinary, in-bounds kernels."""
import ctypes as C
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


def test_membership_buffers_too_small(lf):
    """LF_ERANGE when the capacity is below the membership count; the query call still
    reports the count, and the handle's state is untouched."""
    say("ERANGE memberships")
    g = G.named_config("tiny_sbm")
    h = gpu_handle(lf, g).init_communities()
    h.run_iterations(64, 0.01, 3)
    off0, ids0 = h.memberships()
    inc0 = h.in_counts()
    tot = C.c_int64()
    assert h.L.lf_get_memberships(h.h, None, None, 0, C.byref(tot)) == 0
    assert tot.value == ids0.size > 0
    off = np.zeros(g.n + 1, np.int64)
    ids = np.zeros(tot.value, np.int32)
    rc = h.L.lf_get_memberships(h.h, C.c_void_p(off.ctypes.data), C.c_void_p(ids.ctypes.data), tot.value - 1,
                                C.byref(tot))
    assert rc == lf.LF_ERANGE and tot.value == ids0.size
    assert not ids.any()                                  # nothing written
    assert "capacity" in h.L.lf_last_error(h.h).decode()
    inc = np.zeros(tot.value, np.int32)
    assert h.L.lf_get_in_counts(h.h, C.c_void_p(inc.ctypes.data), tot.value - 1) == lf.LF_ERANGE
    off1, ids1 = h.memberships()
    assert np.array_equal(off0, off1) and np.array_equal(ids0, ids1)
    assert np.array_equal(inc0, h.in_counts())
    h.close()


def test_loader_integer_range_guards(lf):
    """n or the pair count at 2^31 - 1 or beyond is refused with LF_EOVERFLOW before the
    edge arrays are read; a previously loaded graph is kept."""
    say("EOVERFLOW load")
    g = G.random_gnp(50, 0.2, 3)
    h = gpu_handle(lf, g)
    src = np.zeros(4, np.int64)
    dst = np.ones(4, np.int64)
    for n, npairs in ((1 << 31, 4), ((1 << 31) - 1, 4), (8, 1 << 31), (8, (1 << 31) - 1)):
        rc = h.L.lf_load_graph(h.h, n, npairs, C.c_void_p(src.ctypes.data), C.c_void_p(dst.ctypes.data), 0)
        assert rc == lf.LF_EOVERFLOW, (n, npairs)
    assert h.n == g.n
    h.init_communities()
    assert h.memberships()[0].size == g.n + 1
    h.close()


def test_run_stops_at_max_iters(lf, orc):
    """threshold 0 keeps the run going while anything improves: with max_iters = 2 both the
    GPU and the oracle stop after two iterations, not converged, hit_max set, same cover."""
    say("max_iters reached")
    g = G.named_config("copurchase", scale=0.01)
    h = gpu_handle(lf, g).init_communities()
    o = orc.Oracle().load_graph(g.n, g.src, g.dst).init_communities()
    a = h.run_iterations(32, 0.0, 2)
    b = o.run_iterations(32, 0.0, 2, mode=orc.MODE_FAST)
    assert a["iterations"] == b["iterations"] == 2
    assert a["hit_max"] and b["hit_max"] and not a["converged"] and not b["converged"]
    assert a["wtilde"] == b["wtilde"]
    for u, v in zip(h.memberships(), o.memberships()):
        assert np.array_equal(u, v)
    h.close()


def test_server_refuses_job_beyond_budget(lf):
    """A job whose estimated footprint exceeds the whole budget is refused at submission
    (LF_ENOMEM) and leaves nothing queued or reserved."""
    say("server ENOMEM")
    srv = lf.Server(0, hbm_budget=1 << 16, max_batch=4)
    g = G.named_config("tiny_sbm")
    with pytest.raises(lf.LazyFoxError) as e:
        srv.submit(g.n, g.src, g.dst, 64, 0.01, 50)
    assert e.value.code == lf.LF_ENOMEM
    st = srv.stats()
    assert st["used"] == 0 and st["queued"] == 0 and st["running"] == 0
    srv.close()


def test_server_fetch_buffers_too_small(lf):
    """Fetching a done job into buffers below its membership count is LF_ERANGE and keeps
    the job; a fetch with enough room then returns the solo run's result."""
    say("server ERANGE")
    g = G.random_gnp(300, 0.03, 9)
    srv = lf.Server(0, hbm_budget=1 << 30, max_batch=4)
    jid = srv.submit(g.n, g.src, g.dst, 16, 0.01, 50)
    ticks = 0
    while srv.tick() > 0:
        ticks += 1
        assert ticks < 100000
    tot = C.c_int64()
    assert srv.L.lf_server_fetch(srv.s, jid, None, None, 0, C.byref(tot), None) == 0
    assert tot.value > 0
    off = np.zeros(g.n + 1, np.int64)
    ids = np.zeros(tot.value, np.int32)
    rc = srv.L.lf_server_fetch(srv.s, jid, C.c_void_p(off.ctypes.data), C.c_void_p(ids.ctypes.data),
                               tot.value - 1, C.byref(tot), None)
    assert rc == lf.LF_ERANGE
    r = srv.fetch(jid)
    assert r is not None
    h = gpu_handle(lf, g).init_communities()
    h.run_iterations(16, 0.01, 50)
    ho, hi = h.memberships()
    assert np.array_equal(r[0], ho) and np.array_equal(r[1], hi)
    h.close()
    srv.close()
