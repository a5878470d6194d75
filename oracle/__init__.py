"""CPU oracle for the LazyFox hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
may import this package.  The product library (``paper_2210_03211_amd``) never does, and
the two share no code: this package wraps ``lfo.c`` (plain C, built with gcc,
``-ffp-contract=off``) and ``brute.py`` (exact rationals, tiny graphs only).

``build()`` compiles ``liblfo.so`` next to this file.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lfo.c")
_LIB = os.path.join(_HERE, "liblfo.so")

LFO_RELABEL = 1
MODE_NAIVE = 0          # re-sum every candidate community; re-count touched in-counts
MODE_FAST = 3           # exact S+/S- with corrections; incremental in-counts (same bits)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared",
               "-fPIC", "-std=gnu11", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class RunInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("hit_max", C.c_int32),
                ("pad", C.c_int32), ("wcc_hat", C.c_double), ("wtilde", C.c_double),
                ("wtilde_hist", C.POINTER(C.c_double)), ("joins", C.POINTER(C.c_int64)),
                ("leaves", C.POINTER(C.c_int64)), ("communities", C.POINTER(C.c_int64))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        vp, i64, i32, u32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_uint32, C.c_double
        L.lfo_create.restype = vp
        L.lfo_destroy.argtypes = [vp]
        L.lfo_last_error.restype = C.c_char_p
        L.lfo_last_error.argtypes = [vp]
        L.lfo_load_graph.argtypes = [vp, i64, i64, vp, vp, u32]
        L.lfo_init_communities.argtypes = [vp, C.c_int]
        L.lfo_init_from_memberships.argtypes = [vp, vp, vp, i64, i32, C.c_int]
        L.lfo_exact_wcc.argtypes = [vp, C.c_int, vp, vp, vp, vp, vp, vp]
        L.lfo_wcc_sample.argtypes = [vp, vp, i64, vp, vp, vp, vp]
        L.lfo_postprocess.argtypes = [vp, u32, vp, vp, C.c_int]
        L.lfo_cover_f1.argtypes = [vp, vp, vp, i64, vp, vp, vp]
        L.lfo_run_iterations.argtypes = [vp, i32, dbl, i32, i32, i32, i32, C.POINTER(RunInfo)]
        L.lfo_check_state.argtypes = [vp]
        L.lfo_check_state.restype = i64
        L.lfo_set_chunk_limit.argtypes = [vp, i64]
        L.lfo_set_chunk_limit.restype = None
        L.lfo_chunks_done.argtypes = [vp]
        L.lfo_chunks_done.restype = i64
        L.lfo_num_nodes.argtypes = [vp]
        L.lfo_num_nodes.restype = i64
        L.lfo_num_edges.argtypes = [vp]
        L.lfo_num_edges.restype = i64
        L.lfo_num_communities_created.argtypes = [vp]
        L.lfo_num_communities_created.restype = i32
        L.lfo_get_csr.argtypes = [vp, vp, vp]
        L.lfo_get_orig_ids.argtypes = [vp, vp]
        L.lfo_get_node_stats.argtypes = [vp, vp, vp, vp]
        L.lfo_get_scores.argtypes = [vp, vp, vp, vp, vp]
        L.lfo_get_memberships.argtypes = [vp, vp, vp, i64, vp]
        L.lfo_get_communities.argtypes = [vp, vp, vp, vp]
        L.lfo_get_in_counts.argtypes = [vp, vp, i64]
        L.lfo_eval_node.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp]
        L.lfo_exact_sum.argtypes = [vp, i64]
        L.lfo_exact_sum.restype = dbl
        L.lfo_g.argtypes = [i64, i64, i64]
        L.lfo_g.restype = dbl
        L.lfo_density.argtypes = [i64, i64]
        L.lfo_density.restype = dbl
        L.lfo_xs_error.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


class OracleError(RuntimeError):
    pass


class Oracle:
    """One graph's oracle state (mirrors the product C-ABI: load, init, run, get)."""

    def __init__(self):
        self.L = lib()
        self.h = self.L.lfo_create()

    def close(self):
        if self.h:
            self.L.lfo_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != 0:
            raise OracleError("%s failed (%d): %s" % (what, rc, self.L.lfo_last_error(self.h).decode()))

    def load_graph(self, n, src, dst, relabel=False):
        src = np.ascontiguousarray(src, dtype=np.int64)
        dst = np.ascontiguousarray(dst, dtype=np.int64)
        self._check(self.L.lfo_load_graph(self.h, int(n), int(src.size), _p(src), _p(dst),
                                          LFO_RELABEL if relabel else 0), "load_graph")
        return self

    @property
    def n(self):
        return int(self.L.lfo_num_nodes(self.h))

    @property
    def nedges(self):
        return int(self.L.lfo_num_edges(self.h))

    def init_communities(self, nthreads=None):
        nthreads = nthreads or min(8, os.cpu_count() or 1)
        self._check(self.L.lfo_init_communities(self.h, int(nthreads)), "init_communities")
        return self

    def init_from_memberships(self, offsets, ids, n_comms=-1, nthreads=None):
        """Warm start: the given cover (offsets[n + 1], ids) replaces the greedy initial
        clustering; ids in [0, n_comms) (n_comms < 0: largest id + 1)."""
        nthreads = nthreads or min(8, os.cpu_count() or 1)
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        if offsets.size != self.n + 1:
            raise OracleError("init_from_memberships: %d offsets for %d nodes" % (offsets.size, self.n))
        self._check(self.L.lfo_init_from_memberships(self.h, _p(offsets), _p(ids), int(ids.size),
                                                     int(n_comms), int(nthreads)), "init_from_memberships")
        return self

    def run_iterations(self, queue_size, threshold=0.01, max_iters=50, mode=MODE_FAST,
                       nthreads=None, check_every_chunk=False):
        nthreads = nthreads or min(8, os.cpu_count() or 1)
        hist = np.zeros(max_iters + 1, np.float64)
        joins = np.zeros(max(1, max_iters), np.int64)
        leaves = np.zeros(max(1, max_iters), np.int64)
        comms = np.zeros(max(1, max_iters), np.int64)
        info = RunInfo()
        info.wtilde_hist = hist.ctypes.data_as(C.POINTER(C.c_double))
        info.joins = joins.ctypes.data_as(C.POINTER(C.c_int64))
        info.leaves = leaves.ctypes.data_as(C.POINTER(C.c_int64))
        info.communities = comms.ctypes.data_as(C.POINTER(C.c_int64))
        rc = self.L.lfo_run_iterations(self.h, int(queue_size), float(threshold), int(max_iters),
                                       int(mode), int(nthreads), int(bool(check_every_chunk)),
                                       C.byref(info))
        self._check(rc, "run_iterations")
        it = info.iterations
        return dict(iterations=it, converged=bool(info.converged), hit_max=bool(info.hit_max),
                    wcc_hat=info.wcc_hat, wtilde=info.wtilde, wtilde_hist=hist[: it + 1].copy(),
                    joins=joins[:it].copy(), leaves=leaves[:it].copy(),
                    communities=comms[:it].copy())

    def run_queue_prefix(self, queue_size, chunks, mode=MODE_FAST, nthreads=None):
        """Timing sample: evaluate and apply the first `chunks` queues of the first
        iteration and stop there (the state is left mid-iteration).  Returns the number of
        queues done."""
        self.L.lfo_set_chunk_limit(self.h, int(chunks))
        try:
            self.run_iterations(queue_size, 0.0, 1, mode=mode, nthreads=nthreads)
        finally:
            self.L.lfo_set_chunk_limit(self.h, 0)
        return int(self.L.lfo_chunks_done(self.h))

    def exact_wcc(self, nthreads=None):
        """Exact WCC of the current partition: dict(wcc, per-community wcc_comm[K], and per
        membership in the memberships() order: wcc_node, t (t(x,C)), vt_out (vt(x, V\\C));
        vt[n] = vt(x, V))."""
        nthreads = nthreads or min(8, os.cpu_count() or 1)
        off, ids = self.memberships()
        K = int(self.L.lfo_num_communities_created(self.h))
        tot = ids.size
        wcc = C.c_double()
        wc = np.zeros(max(1, K), np.float64)
        wn = np.zeros(max(1, tot), np.float64)
        t = np.zeros(max(1, tot), np.int32)
        vo = np.zeros(max(1, tot), np.int32)
        vx = np.zeros(max(1, self.n), np.int32)
        self._check(self.L.lfo_exact_wcc(self.h, int(nthreads), C.byref(wcc), _p(wc), _p(wn), _p(t), _p(vo), _p(vx)),
                    "exact_wcc")
        return dict(wcc=wcc.value, wcc_comm=wc[:K], wcc_node=wn[:tot], t=t[:tot], vt_out=vo[:tot], vt=vx[:self.n])

    def wcc_sample(self, nodes):
        """WCC terms of the listed nodes only: (wcc_node, t, vt_out) over their memberships
        (ascending ids, node after node) and vt per node."""
        nodes = np.ascontiguousarray(nodes, dtype=np.int32)
        off, ids = self.memberships()
        tot = int(sum(off[x + 1] - off[x] for x in nodes))
        wn = np.zeros(max(1, tot), np.float64)
        t = np.zeros(max(1, tot), np.int32)
        vo = np.zeros(max(1, tot), np.int32)
        vx = np.zeros(max(1, nodes.size), np.int32)
        self._check(self.L.lfo_wcc_sample(self.h, _p(nodes), int(nodes.size), _p(wn), _p(t), _p(vo), _p(vx)),
                    "wcc_sample")
        return wn[:tot], t[:tot], vo[:tot], vx[:nodes.size]

    def postprocess(self, duplicates=True, contained=True, apply=False, nthreads=None):
        """Duplicated / contained community removal: (keep[K] uint8, (removed as duplicates,
        removed as contained)); apply=True also rebuilds the state without them."""
        nthreads = nthreads or min(8, os.cpu_count() or 1)
        K = int(self.L.lfo_num_communities_created(self.h))
        keep = np.zeros(max(1, K), np.uint8)
        rem = np.zeros(2, np.int64)
        flags = (1 if duplicates else 0) | (2 if contained else 0) | (4 if apply else 0)
        self._check(self.L.lfo_postprocess(self.h, flags, _p(keep), _p(rem), int(nthreads)), "postprocess")
        return keep[:K], (int(rem[0]), int(rem[1]))

    def cover_f1(self, offsets, ids):
        """F1-Score of the current partition against a reference cover: (f1, best[K],
        match[K])."""
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        if offsets.size != self.n + 1:
            raise OracleError("cover_f1: %d offsets for %d nodes" % (offsets.size, self.n))
        K = int(self.L.lfo_num_communities_created(self.h))
        f1 = C.c_double()
        best = np.zeros(max(1, K), np.float64)
        match = np.zeros(max(1, K), np.int32)
        self._check(self.L.lfo_cover_f1(self.h, _p(offsets), _p(ids), int(ids.size), C.byref(f1), _p(best),
                                        _p(match)), "cover_f1")
        return f1.value, best[:K], match[:K]

    def check_state(self):
        return int(self.L.lfo_check_state(self.h))

    def csr(self):
        n, ne = self.n, self.nedges
        rp = np.zeros(n + 1, np.int64)
        col = np.zeros(2 * ne, np.int32)
        self._check(self.L.lfo_get_csr(self.h, _p(rp), _p(col)), "get_csr")
        return rp, col

    def orig_ids(self):
        ids = np.zeros(self.n, np.int64)
        self._check(self.L.lfo_get_orig_ids(self.h, _p(ids)), "get_orig_ids")
        return ids

    def node_stats(self):
        n = self.n
        tri = np.zeros(n, np.int64)
        ccl = np.zeros(n, np.float64)
        order = np.zeros(n, np.int32)
        self._check(self.L.lfo_get_node_stats(self.h, _p(tri), _p(ccl), _p(order)), "get_node_stats")
        return tri, ccl, order

    def scores(self):
        w, cc, wt = C.c_double(), C.c_double(), C.c_double()
        T = C.c_int64()
        self._check(self.L.lfo_get_scores(self.h, C.byref(w), C.byref(cc), C.byref(T), C.byref(wt)),
                    "get_scores")
        return dict(wcc_hat=w.value, cc=cc.value, triangles=T.value, wtilde=wt.value)

    def memberships(self):
        tot = C.c_int64()
        self._check(self.L.lfo_get_memberships(self.h, None, None, 0, C.byref(tot)), "get_memberships")
        off = np.zeros(self.n + 1, np.int64)
        ids = np.zeros(max(1, tot.value), np.int32)
        self._check(self.L.lfo_get_memberships(self.h, _p(off), _p(ids), ids.size, C.byref(tot)),
                    "get_memberships")
        return off, ids[: tot.value]

    def in_counts(self):
        off, ids = self.memberships()
        inc = np.zeros(max(1, ids.size), np.int32)
        self._check(self.L.lfo_get_in_counts(self.h, _p(inc), inc.size), "get_in_counts")
        return inc[: ids.size]

    def communities(self):
        K = int(self.L.lfo_num_communities_created(self.h))
        s = np.zeros(max(1, K), np.int32)
        m = np.zeros(max(1, K), np.int64)
        W = np.zeros(max(1, K), np.float64)
        self._check(self.L.lfo_get_communities(self.h, _p(s), _p(m), _p(W)), "get_communities")
        return s[:K], m[:K], W[:K]

    def eval_node(self, x, mode=MODE_NAIVE, cap=4096):
        comm = np.zeros(cap, np.int32)
        delta = np.zeros(cap, np.float64)
        leave = np.zeros(cap, np.int32)
        nc, bj, bl = C.c_int32(), C.c_int32(), C.c_int32()
        jd, ld = C.c_double(), C.c_double()
        self._check(self.L.lfo_eval_node(self.h, int(x), int(mode), cap, _p(comm), _p(delta), _p(leave),
                                         C.byref(nc), C.byref(bj), C.byref(jd), C.byref(bl),
                                         C.byref(ld)), "eval_node")
        k = nc.value
        return dict(cand=comm[:k].copy(), delta=delta[:k].copy(), is_leave=leave[:k].astype(bool),
                    best_join=bj.value, join_delta=jd.value, best_leave=bl.value,
                    leave_delta=ld.value)


def exact_sum(values) -> float:
    v = np.ascontiguousarray(values, dtype=np.float64)
    return float(lib().lfo_exact_sum(_p(v), v.size))


def g_term(i, d, s) -> float:
    return float(lib().lfo_g(int(i), int(d), int(s)))


def density(s, m) -> float:
    return float(lib().lfo_density(int(s), int(m)))


def run_graph(graph, queue_size, threshold=0.01, max_iters=50, mode=MODE_FAST, nthreads=None,
              relabel=False):
    """Convenience: the whole path on a graphgen.Graph; returns (oracle, run-info dict)."""
    o = Oracle().load_graph(graph.n, graph.src, graph.dst, relabel=relabel)
    o.init_communities(nthreads)
    info = o.run_iterations(queue_size, threshold, max_iters, mode=mode, nthreads=nthreads)
    return o, info
