"""ctypes binding of liblazyfox.so: one Python method per C entry point, same names."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblazyfox.so")

LF_OK, LF_EINVAL, LF_ESTATE, LF_ENOMEM, LF_EDEVICE, LF_ERANGE, LF_EOVERFLOW = 0, -1, -2, -3, -4, -5, -6
LF_EAGAIN, LF_EINTERNAL = -7, -8
LF_RELABEL = 1
LF_DEVICE_PTR = 2
OPTIONS = {"tri_lds_cap": 1, "hub_blocks": 3, "refresh_blocks": 4, "wave_table": 5, "med_table": 6,
           "grp_table": 7, "prof_stride": 8}
KERNEL_CLASSES = ["build", "triangles", "order", "init_clustering", "k_eval", "k_eval_big", "k_big_final",
                  "k_big_tie", "k_apply", "k_apply_in", "k_refresh", "iteration_end"]
PROF_COUNTERS_BIT = 16
PATHS = ["small", "medium", "group", "table"]
APPLY_WORK = ["moves", "own_slots", "in_units", "in_neighbours", "in_slots", "parts", "touched", "members",
              "member_slots"]


class LazyFoxError(RuntimeError):
    def __init__(self, code, what, text):
        super().__init__("%s failed (status %d): %s" % (what, code, text))
        self.code = code


class RunInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("hit_max", C.c_int32),
                ("pad", C.c_int32), ("wcc_hat", C.c_double), ("wtilde", C.c_double),
                ("wtilde_hist", C.POINTER(C.c_double)), ("joins", C.POINTER(C.c_int64)),
                ("leaves", C.POINTER(C.c_int64)), ("communities", C.POINTER(C.c_int64))]


class TuneResult(C.Structure):
    _fields_ = [("value", C.c_int64 * 5), ("default_ms", C.c_float), ("best_ms", C.c_float),
                ("trials", C.c_int32), ("from_cache", C.c_int32)]


class Profile(C.Structure):
    _fields_ = [("launches", C.c_int64 * 12), ("ms", C.c_double * 12), ("chunks", C.c_int64),
                ("node_evals", C.c_int64), ("visits", C.c_int64), ("candidates", C.c_int64),
                ("path_nodes", C.c_int64 * 4), ("path_neighbours", C.c_int64 * 4),
                ("path_visits", C.c_int64 * 4), ("path_candidates", C.c_int64 * 4),
                ("path_own", C.c_int64 * 4), ("apply_work", C.c_int64 * 9)]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def load_library():
    """Load liblazyfox.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError("liblazyfox.so is not built (run `python -m paper_2210_03211_amd.build` "
                          "or __graft_entry__.build()); the HIP library is required")
    # PyTorch's ROCm wheels carry a HIP runtime of their own: when both are in the process,
    # torch's must have initialised the device before the library is loaded, or the
    # library's runtime finds no device
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
    except ImportError:
        pass
    L = C.CDLL(_LIB_PATH)
    vp, i32, i64, u32, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_double
    sig = {
        "lf_create": [C.POINTER(vp), C.c_int, vp, u32],
        "lf_destroy": [vp],
        "lf_load_graph": [vp, i64, i64, vp, vp, u32],
        "lf_init_communities": [vp],
        "lf_init_from_memberships": [vp, vp, vp, i64, i32, u32],
        "lf_exact_wcc": [vp, C.POINTER(dbl), vp, vp, vp, vp, vp],
        "lf_postprocess": [vp, u32, vp, vp],
        "lf_cover_f1": [vp, vp, vp, i64, u32, C.POINTER(dbl), vp, vp],
        "lf_run_iterations": [vp, i32, dbl, i32, C.POINTER(RunInfo)],
        "lf_get_memberships": [vp, vp, vp, i64, C.POINTER(i64)],
        "lf_get_graph_info": [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)],
        "lf_get_csr": [vp, vp, vp, vp],
        "lf_get_node_stats": [vp, vp, vp, vp],
        "lf_get_scores": [vp, vp, vp, vp, vp],
        "lf_get_communities": [vp, vp, vp, vp],
        "lf_get_in_counts": [vp, vp, i64],
        "lf_set_profiling": [vp, C.c_int],
        "lf_get_profile": [vp, C.POINTER(Profile)],
        "lf_reset_profile": [vp],
        "lf_debug_exact_sum": [vp, vp, i64, C.POINTER(dbl)],
        "lf_exact_sum_noalloc": [vp, vp, i64, C.POINTER(dbl)],
        "lf_debug_sort_pairs": [vp, vp, vp, i64, i32],
        "lf_debug_sort_pairs_u32": [vp, vp, vp, i64],
        "lf_debug_exclusive_scan": [vp, vp, i32, vp, i64],
        "lf_set_option": [vp, C.c_int, i64],
        "lf_get_option": [vp, C.c_int, C.POINTER(i64)],
        "lf_get_memory": [vp, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)],
        "lf_batch_create": [C.POINTER(vp), C.c_int, vp],
        "lf_batch_add": [vp, vp, i32, dbl, i32, C.POINTER(i32)],
        "lf_batch_step": [vp, C.POINTER(i32)],
        "lf_batch_member_info": [vp, i32, C.POINTER(RunInfo)],
        "lf_batch_remove": [vp, i32],
        "lf_batch_destroy": [vp],
        "lf_batch_set_graph": [vp, i32],
        "lf_server_create": [C.POINTER(vp), C.c_int, vp, C.c_uint64, i32],
        "lf_server_submit": [vp, i64, i64, vp, vp, i32, dbl, i32, C.POINTER(i64)],
        "lf_server_tick": [vp, C.POINTER(i32)],
        "lf_server_poll": [vp, i64, C.POINTER(i32)],
        "lf_server_fetch": [vp, i64, vp, vp, i64, C.POINTER(i64), C.POINTER(RunInfo)],
        "lf_server_stats": [vp, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.POINTER(i32), C.POINTER(i32)],
        "lf_server_destroy": [vp],
        "lf_server_timing": [vp, C.POINTER(C.c_double)],
        "lf_server_take_done": [vp, vp, i32, C.POINTER(i32)],
        "lf_server_set_graph": [vp, i32],
        "lf_autotune": [vp, i32, i32, C.POINTER(TuneResult)],
        "lf_autotune_forget": [],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    for name in ("lf_last_error", "lf_batch_last_error", "lf_server_last_error"):
        f = getattr(L, name)
        f.argtypes = [vp]
        f.restype = C.c_char_p
    _lib = L
    return L


def _ptr(a):
    """(address, is_device) of a numpy array or a torch tensor."""
    if isinstance(a, np.ndarray):
        return a.ctypes.data, False
    if hasattr(a, "data_ptr"):
        return a.data_ptr(), bool(a.is_cuda)
    raise TypeError("expected a numpy array or a torch tensor")


def _current_stream(device):
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)
    except ImportError:
        pass
    return None


class Handle:
    """One graph's device-resident LazyFox state (``lf_handle``)."""

    def __init__(self, device: int = 0, stream=None):
        self.L = load_library()
        self.h = C.c_void_p()
        if stream is None:
            stream = _current_stream(device)
        elif hasattr(stream, "cuda_stream"):
            stream = C.c_void_p(stream.cuda_stream)
        rc = self.L.lf_create(C.byref(self.h), int(device), stream, 0)
        if rc != 0:
            raise LazyFoxError(rc, "lf_create", "device %d unavailable" % device)
        self.device = device

    # -- lifetime ------------------------------------------------------------------
    def lf_destroy(self):
        if self.h:
            self.L.lf_destroy(self.h)
            self.h = C.c_void_p()

    close = lf_destroy

    def __del__(self):
        try:
            self.lf_destroy()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.lf_destroy()

    def _check(self, rc, what):
        if rc != 0:
            raise LazyFoxError(rc, what, self.L.lf_last_error(self.h).decode(errors="replace"))

    # -- C entry points ------------------------------------------------------------
    def lf_load_graph(self, n, src, dst, relabel=False):
        ps, ds = _ptr(src)
        pd, dd = _ptr(dst)
        if ds != dd:
            raise ValueError("src and dst must both be host or both be device arrays")
        for a in (src, dst):
            if str(getattr(a, "dtype", "")) not in ("int64", "torch.int64"):
                raise TypeError("edge arrays must be int64")
        npairs = int(src.shape[0])
        if int(dst.shape[0]) != npairs:
            raise ValueError("src and dst differ in length")
        flags = (LF_RELABEL if relabel else 0) | (LF_DEVICE_PTR if ds else 0)
        self._check(self.L.lf_load_graph(self.h, int(n), npairs, C.c_void_p(ps), C.c_void_p(pd), flags),
                    "lf_load_graph")
        return self

    load_graph = lf_load_graph

    def lf_init_communities(self):
        self._check(self.L.lf_init_communities(self.h), "lf_init_communities")
        return self

    init_communities = lf_init_communities

    def lf_init_from_memberships(self, offsets, comm_ids, n_comms=-1):
        """Warm start from an existing cover: offsets int64[n + 1], comm_ids int32 (both
        numpy arrays or both device tensors); n_comms < 0 takes the largest id + 1."""
        po, do = _ptr(offsets)
        pc, dc = _ptr(comm_ids)
        if do != dc:
            raise ValueError("offsets and comm_ids must both be host or both be device arrays")
        if str(getattr(offsets, "dtype", "")) not in ("int64", "torch.int64"):
            raise TypeError("offsets must be int64")
        if str(getattr(comm_ids, "dtype", "")) not in ("int32", "torch.int32"):
            raise TypeError("comm_ids must be int32")
        n = self.lf_get_graph_info()[0]
        if int(offsets.shape[0]) != n + 1:
            raise ValueError("offsets must have n + 1 = %d entries" % (n + 1))
        total = int(comm_ids.shape[0])
        self._check(self.L.lf_init_from_memberships(self.h, C.c_void_p(po), C.c_void_p(pc), total, int(n_comms),
                                                    LF_DEVICE_PTR if do else 0), "lf_init_from_memberships")
        return self

    init_from_memberships = lf_init_from_memberships

    def lf_exact_wcc(self):
        """Exact WCC of the current partition: dict(wcc, wcc_comm[K], per membership in the
        memberships() order wcc_node, t, vt_out; vt[n])."""
        n, _, K = self.lf_get_graph_info()
        off, ids = self.lf_get_memberships()
        tot = ids.size
        wcc = C.c_double()
        wc = np.zeros(max(1, K), np.float64)
        wn = np.zeros(max(1, tot), np.float64)
        t = np.zeros(max(1, tot), np.int32)
        vo = np.zeros(max(1, tot), np.int32)
        vx = np.zeros(max(1, n), np.int32)
        self._check(self.L.lf_exact_wcc(self.h, C.byref(wcc), C.c_void_p(wc.ctypes.data), C.c_void_p(wn.ctypes.data),
                                        C.c_void_p(t.ctypes.data), C.c_void_p(vo.ctypes.data),
                                        C.c_void_p(vx.ctypes.data)), "lf_exact_wcc")
        return dict(wcc=wcc.value, wcc_comm=wc[:K], wcc_node=wn[:tot], t=t[:tot], vt_out=vo[:tot], vt=vx[:n])

    exact_wcc = lf_exact_wcc

    def lf_postprocess(self, duplicates=True, contained=True, apply=False):
        """Duplicated / contained community removal: (keep[K] uint8, (removed as duplicates,
        removed as contained)); apply=True also takes them out of the partition."""
        K = self.lf_get_graph_info()[2]
        keep = np.zeros(max(1, K), np.uint8)
        rem = np.zeros(2, np.int64)
        flags = (1 if duplicates else 0) | (2 if contained else 0) | (4 if apply else 0)
        self._check(self.L.lf_postprocess(self.h, flags, C.c_void_p(keep.ctypes.data), C.c_void_p(rem.ctypes.data)),
                    "lf_postprocess")
        return keep[:K], (int(rem[0]), int(rem[1]))

    postprocess = lf_postprocess

    def lf_cover_f1(self, offsets, ids):
        """F1-Score of the current partition against a reference cover (offsets int64[n + 1],
        ids int32; numpy or device tensors): (f1, best[K], match[K])."""
        po, do = _ptr(offsets)
        pc, dc = _ptr(ids)
        if do != dc:
            raise ValueError("offsets and ids must both be host or both be device arrays")
        if str(getattr(offsets, "dtype", "")) not in ("int64", "torch.int64"):
            raise TypeError("offsets must be int64")
        if str(getattr(ids, "dtype", "")) not in ("int32", "torch.int32"):
            raise TypeError("ids must be int32")
        n, _, K = self.lf_get_graph_info()
        if int(offsets.shape[0]) != n + 1:
            raise ValueError("offsets must have n + 1 = %d entries" % (n + 1))
        f1 = C.c_double()
        best = np.zeros(max(1, K), np.float64)
        match = np.zeros(max(1, K), np.int32)
        self._check(self.L.lf_cover_f1(self.h, C.c_void_p(po), C.c_void_p(pc), int(ids.shape[0]),
                                       LF_DEVICE_PTR if do else 0, C.byref(f1), C.c_void_p(best.ctypes.data),
                                       C.c_void_p(match.ctypes.data)), "lf_cover_f1")
        return f1.value, best[:K], match[:K]

    cover_f1 = lf_cover_f1

    def lf_run_iterations(self, queue_size, threshold=0.01, max_iters=50):
        hist = np.zeros(max_iters + 1, np.float64)
        joins = np.zeros(max(1, max_iters), np.int64)
        leaves = np.zeros(max(1, max_iters), np.int64)
        comms = np.zeros(max(1, max_iters), np.int64)
        info = RunInfo()
        info.wtilde_hist = hist.ctypes.data_as(C.POINTER(C.c_double))
        info.joins = joins.ctypes.data_as(C.POINTER(C.c_int64))
        info.leaves = leaves.ctypes.data_as(C.POINTER(C.c_int64))
        info.communities = comms.ctypes.data_as(C.POINTER(C.c_int64))
        self._check(self.L.lf_run_iterations(self.h, int(queue_size), float(threshold), int(max_iters),
                                             C.byref(info)), "lf_run_iterations")
        it = info.iterations
        return dict(iterations=it, converged=bool(info.converged), hit_max=bool(info.hit_max),
                    wcc_hat=info.wcc_hat, wtilde=info.wtilde, wtilde_hist=hist[: it + 1].copy(),
                    joins=joins[:it].copy(), leaves=leaves[:it].copy(), communities=comms[:it].copy())

    run_iterations = lf_run_iterations

    def lf_get_graph_info(self):
        n, ne, k = C.c_int64(), C.c_int64(), C.c_int64()
        self._check(self.L.lf_get_graph_info(self.h, C.byref(n), C.byref(ne), C.byref(k)), "lf_get_graph_info")
        return n.value, ne.value, k.value

    @property
    def n(self):
        return self.lf_get_graph_info()[0]

    @property
    def nedges(self):
        return self.lf_get_graph_info()[1]

    def lf_get_memberships(self):
        tot = C.c_int64()
        self._check(self.L.lf_get_memberships(self.h, None, None, 0, C.byref(tot)), "lf_get_memberships")
        n = self.n
        off = np.zeros(n + 1, np.int64)
        ids = np.zeros(max(1, tot.value), np.int32)
        self._check(self.L.lf_get_memberships(self.h, C.c_void_p(off.ctypes.data), C.c_void_p(ids.ctypes.data),
                                              ids.size, C.byref(tot)), "lf_get_memberships")
        return off, ids[: tot.value]

    get_memberships = lf_get_memberships
    memberships = lf_get_memberships

    def lf_get_in_counts(self):
        off, ids = self.lf_get_memberships()
        inc = np.zeros(max(1, ids.size), np.int32)
        self._check(self.L.lf_get_in_counts(self.h, C.c_void_p(inc.ctypes.data), inc.size), "lf_get_in_counts")
        return inc[: ids.size]

    in_counts = lf_get_in_counts

    def lf_get_csr(self):
        n, ne, _ = self.lf_get_graph_info()
        rp = np.zeros(n + 1, np.int64)
        col = np.zeros(max(1, 2 * ne), np.int32)
        ids = np.zeros(max(1, n), np.int64)
        self._check(self.L.lf_get_csr(self.h, C.c_void_p(rp.ctypes.data), C.c_void_p(col.ctypes.data),
                                      C.c_void_p(ids.ctypes.data)), "lf_get_csr")
        return rp, col[: 2 * ne], ids[:n]

    def csr(self):
        rp, col, _ = self.lf_get_csr()
        return rp, col

    def orig_ids(self):
        return self.lf_get_csr()[2]

    def lf_get_node_stats(self):
        n = self.n
        tri = np.zeros(max(1, n), np.int64)
        ccl = np.zeros(max(1, n), np.float64)
        order = np.zeros(max(1, n), np.int32)
        self._check(self.L.lf_get_node_stats(self.h, C.c_void_p(tri.ctypes.data), C.c_void_p(ccl.ctypes.data),
                                             C.c_void_p(order.ctypes.data)), "lf_get_node_stats")
        return tri[:n], ccl[:n], order[:n]

    node_stats = lf_get_node_stats

    def lf_get_scores(self):
        w, cc, wt = C.c_double(), C.c_double(), C.c_double()
        T = C.c_int64()
        self._check(self.L.lf_get_scores(self.h, C.byref(w), C.byref(cc), C.byref(T), C.byref(wt)),
                    "lf_get_scores")
        return dict(wcc_hat=w.value, cc=cc.value, triangles=T.value, wtilde=wt.value)

    scores = lf_get_scores

    def lf_get_communities(self):
        K = self.lf_get_graph_info()[2]
        s = np.zeros(max(1, K), np.int32)
        m = np.zeros(max(1, K), np.int64)
        W = np.zeros(max(1, K), np.float64)
        self._check(self.L.lf_get_communities(self.h, C.c_void_p(s.ctypes.data), C.c_void_p(m.ctypes.data),
                                              C.c_void_p(W.ctypes.data)), "lf_get_communities")
        return s[:K], m[:K], W[:K]

    communities = lf_get_communities

    def lf_set_profiling(self, mask=True):
        """mask: kernels to time (bit i = KERNEL_CLASSES[i]; bit PROF_COUNTERS_BIT adds the
        per-path work counters); True = every kernel without the counters, 0 = off."""
        if mask is True:
            mask = (1 << len(KERNEL_CLASSES)) - 1
        self._check(self.L.lf_set_profiling(self.h, int(mask)), "lf_set_profiling")

    def lf_reset_profile(self):
        self._check(self.L.lf_reset_profile(self.h), "lf_reset_profile")

    def lf_get_profile(self):
        p = Profile()
        self._check(self.L.lf_get_profile(self.h, C.byref(p)), "lf_get_profile")
        return dict(launches={k: int(p.launches[i]) for i, k in enumerate(KERNEL_CLASSES)},
                    ms={k: float(p.ms[i]) for i, k in enumerate(KERNEL_CLASSES)},
                    chunks=int(p.chunks), node_evals=int(p.node_evals), visits=int(p.visits),
                    candidates=int(p.candidates),
                    paths={name: dict(nodes=int(p.path_nodes[i]), neighbours=int(p.path_neighbours[i]),
                                      visits=int(p.path_visits[i]), candidates=int(p.path_candidates[i]),
                                      own=int(p.path_own[i]))
                           for i, name in enumerate(PATHS)},
                apply={name: int(p.apply_work[i]) for i, name in enumerate(APPLY_WORK)})

    def lf_set_option(self, name, value):
        self._check(self.L.lf_set_option(self.h, OPTIONS[name], int(value)), "lf_set_option")
        return self

    def lf_get_option(self, name):
        v = C.c_int64()
        self._check(self.L.lf_get_option(self.h, OPTIONS[name], C.byref(v)), "lf_get_option")
        return v.value

    def lf_autotune(self, queue_size, trial_iters=2):
        """Tune the path thresholds and launch shapes on this graph (see lazyfox.h)."""
        r = TuneResult()
        self._check(self.L.lf_autotune(self.h, int(queue_size), int(trial_iters), C.byref(r)), "lf_autotune")
        names = ("wave_table", "med_table", "grp_table", "hub_blocks", "refresh_blocks")
        return dict(options=dict(zip(names, list(r.value))), default_ms=r.default_ms, best_ms=r.best_ms,
                    trials=r.trials, from_cache=bool(r.from_cache))

    autotune = lf_autotune

    def lf_autotune_forget(self):
        self._check(self.L.lf_autotune_forget(), "lf_autotune_forget")

    def lf_get_memory(self):
        b, p = C.c_uint64(), C.c_uint64()
        self._check(self.L.lf_get_memory(self.h, C.byref(b), C.byref(p)), "lf_get_memory")
        return b.value, p.value

    def lf_debug_exact_sum(self, values_dev):
        p, is_dev = _ptr(values_dev)
        if not is_dev:
            raise ValueError("lf_debug_exact_sum takes a device array")
        out = C.c_double()
        self._check(self.L.lf_debug_exact_sum(self.h, C.c_void_p(p), int(values_dev.numel()), C.byref(out)),
                    "lf_debug_exact_sum")
        return out.value

    def lf_exact_sum_noalloc(self, values_dev):
        """lf_debug_exact_sum on the library's fixed device scratch (allocates nothing)."""
        p, is_dev = _ptr(values_dev)
        if not is_dev:
            raise ValueError("lf_exact_sum_noalloc takes a device array")
        return self._noalloc_raw(values_dev, int(values_dev.numel()))

    def _noalloc_raw(self, values_dev, n):
        out = C.c_double()
        self._check(self.L.lf_exact_sum_noalloc(self.h, C.c_void_p(_ptr(values_dev)[0]), int(n), C.byref(out)),
                    "lf_exact_sum_noalloc")
        return out.value

    def lf_debug_sort_pairs(self, keys_dev, vals_dev=None, end_bit=64):
        """Stable radix sort in place of uint64 keys (as int64 tensor bits) and int32 values."""
        kp, kd = _ptr(keys_dev)
        vp_, vd = _ptr(vals_dev) if vals_dev is not None else (0, True)
        if not (kd and vd):
            raise ValueError("lf_debug_sort_pairs takes device arrays")
        self._check(self.L.lf_debug_sort_pairs(self.h, C.c_void_p(kp), C.c_void_p(vp_) if vals_dev is not None
                                               else None, int(keys_dev.numel()), int(end_bit)),
                    "lf_debug_sort_pairs")

    def lf_debug_sort_pairs_u32(self, keys_dev, vals_dev):
        """Stable radix sort in place of uint32 keys (as int32 tensor bits) and int32 values."""
        kp, kd = _ptr(keys_dev)
        vp_, vd = _ptr(vals_dev)
        if not (kd and vd):
            raise ValueError("lf_debug_sort_pairs_u32 takes device arrays")
        self._check(self.L.lf_debug_sort_pairs_u32(self.h, C.c_void_p(kp), C.c_void_p(vp_), int(keys_dev.numel())),
                    "lf_debug_sort_pairs_u32")

    def lf_debug_exclusive_scan(self, in_dev, out_dev):
        """out[i] = sum of in[0..i) (int64) for an int32 or int64 device array."""
        ip, idv = _ptr(in_dev)
        op, odv = _ptr(out_dev)
        if not (idv and odv):
            raise ValueError("lf_debug_exclusive_scan takes device arrays")
        self._check(self.L.lf_debug_exclusive_scan(self.h, C.c_void_p(ip), int(in_dev.element_size()),
                                                   C.c_void_p(op), int(in_dev.numel())),
                    "lf_debug_exclusive_scan")


def _run_info_arrays(max_iters):
    hist = np.zeros(max_iters + 1, np.float64)
    joins = np.zeros(max(1, max_iters), np.int64)
    leaves = np.zeros(max(1, max_iters), np.int64)
    comms = np.zeros(max(1, max_iters), np.int64)
    info = RunInfo()
    info.wtilde_hist = hist.ctypes.data_as(C.POINTER(C.c_double))
    info.joins = joins.ctypes.data_as(C.POINTER(C.c_int64))
    info.leaves = leaves.ctypes.data_as(C.POINTER(C.c_int64))
    info.communities = comms.ctypes.data_as(C.POINTER(C.c_int64))
    return info, hist, joins, leaves, comms


def _run_info_dict(info, hist, joins, leaves, comms):
    it = info.iterations
    return dict(iterations=it, converged=bool(info.converged), hit_max=bool(info.hit_max),
                wcc_hat=info.wcc_hat, wtilde=info.wtilde, wtilde_hist=hist[: it + 1].copy(),
                joins=joins[:it].copy(), leaves=leaves[:it].copy(), communities=comms[:it].copy())


class Batch:
    """Many graphs advanced together, one queue of each per step (``lf_batch``)."""

    def __init__(self, device: int = 0, stream=None):
        self.L = load_library()
        self.b = C.c_void_p()
        if stream is None:
            stream = _current_stream(device)
        elif hasattr(stream, "cuda_stream"):
            stream = C.c_void_p(stream.cuda_stream)
        rc = self.L.lf_batch_create(C.byref(self.b), int(device), stream)
        if rc != 0:
            raise LazyFoxError(rc, "lf_batch_create", "device %d unavailable" % device)
        self._max_iters = {}

    def _check(self, rc, what):
        if rc != 0:
            raise LazyFoxError(rc, what, self.L.lf_batch_last_error(self.b).decode(errors="replace"))

    def lf_batch_add(self, handle, queue_size, threshold=0.01, max_iters=50):
        mid = C.c_int32()
        self._check(self.L.lf_batch_add(self.b, handle.h, int(queue_size), float(threshold), int(max_iters),
                                        C.byref(mid)), "lf_batch_add")
        self._max_iters[mid.value] = int(max_iters)
        return mid.value

    add = lf_batch_add

    def lf_batch_step(self):
        running = C.c_int32()
        self._check(self.L.lf_batch_step(self.b, C.byref(running)), "lf_batch_step")
        return running.value

    step = lf_batch_step

    def lf_batch_member_info(self, member):
        """Run info of a finished member (as Handle.run_iterations returns), None while it runs."""
        arrays = _run_info_arrays(self._max_iters.get(member, 1))
        rc = self.L.lf_batch_member_info(self.b, int(member), C.byref(arrays[0]))
        if rc == LF_EAGAIN:
            return None
        self._check(rc, "lf_batch_member_info")
        return _run_info_dict(*arrays)

    member_info = lf_batch_member_info

    def lf_batch_remove(self, member):
        self._check(self.L.lf_batch_remove(self.b, int(member)), "lf_batch_remove")

    remove = lf_batch_remove

    def lf_batch_set_graph(self, on=True):
        self._check(self.L.lf_batch_set_graph(self.b, 1 if on else 0), "lf_batch_set_graph")

    set_graph = lf_batch_set_graph

    def lf_batch_destroy(self):
        if self.b:
            self.L.lf_batch_destroy(self.b)
            self.b = C.c_void_p()

    close = lf_batch_destroy

    def lf_batch_last_error(self):
        return self.L.lf_batch_last_error(self.b).decode(errors="replace")

    def __del__(self):
        try:
            self.lf_batch_destroy()
        except Exception:
            pass


class Server:
    """Serving runtime (``lf_server``): jobs admitted by device-memory footprint into a
    shared batch as they arrive, results copied back as they finish."""

    def __init__(self, device: int = 0, hbm_budget: int = 32 << 30, max_batch: int = 256, stream=None):
        self.L = load_library()
        self.s = C.c_void_p()
        if stream is None:
            stream = _current_stream(device)
        elif hasattr(stream, "cuda_stream"):
            stream = C.c_void_p(stream.cuda_stream)
        rc = self.L.lf_server_create(C.byref(self.s), int(device), stream, int(hbm_budget), int(max_batch))
        if rc != 0:
            raise LazyFoxError(rc, "lf_server_create", "device %d unavailable" % device)
        self._max_iters = {}
        self._n = {}

    def _check(self, rc, what):
        if rc != 0:
            raise LazyFoxError(rc, what, self.L.lf_server_last_error(self.s).decode(errors="replace"))

    def lf_server_submit(self, n, src, dst, queue_size, threshold=0.01, max_iters=50):
        src = np.ascontiguousarray(src, dtype=np.int64)
        dst = np.ascontiguousarray(dst, dtype=np.int64)
        if src.shape != dst.shape:
            raise ValueError("src and dst differ in length")
        jid = C.c_int64()
        self._check(self.L.lf_server_submit(self.s, int(n), int(src.size), C.c_void_p(src.ctypes.data),
                                            C.c_void_p(dst.ctypes.data), int(queue_size), float(threshold),
                                            int(max_iters), C.byref(jid)), "lf_server_submit")
        self._max_iters[jid.value] = int(max_iters)
        self._n[jid.value] = int(n)
        return jid.value

    submit = lf_server_submit

    def lf_server_tick(self):
        pending = C.c_int32()
        self._check(self.L.lf_server_tick(self.s, C.byref(pending)), "lf_server_tick")
        return pending.value

    tick = lf_server_tick

    def lf_server_poll(self, job):
        st = C.c_int32()
        self._check(self.L.lf_server_poll(self.s, int(job), C.byref(st)), "lf_server_poll")
        return st.value

    poll = lf_server_poll

    def lf_server_take_done(self, capacity=4096):
        """Ids of the jobs that finished or failed since the last call."""
        ids = np.zeros(max(1, capacity), np.int64)
        cnt = C.c_int32()
        self._check(self.L.lf_server_take_done(self.s, C.c_void_p(ids.ctypes.data), int(capacity), C.byref(cnt)),
                    "lf_server_take_done")
        return [int(x) for x in ids[: cnt.value]]

    take_done = lf_server_take_done

    def lf_server_fetch(self, job):
        """(offsets, community ids, run info) of a done job; None while it is not done."""
        arrays = _run_info_arrays(self._max_iters.get(job, 1))
        total = C.c_int64()
        rc = self.L.lf_server_fetch(self.s, int(job), None, None, 0, C.byref(total), C.byref(arrays[0]))
        if rc == LF_EAGAIN:
            return None
        self._check(rc, "lf_server_fetch")
        off = np.zeros(self._n[job] + 1, np.int64)
        ids = np.zeros(max(1, total.value), np.int32)
        self._check(self.L.lf_server_fetch(self.s, int(job), C.c_void_p(off.ctypes.data), C.c_void_p(ids.ctypes.data),
                                           ids.size, C.byref(total), None), "lf_server_fetch")
        del self._max_iters[job], self._n[job]
        return off, ids[: total.value], _run_info_dict(*arrays)

    fetch = lf_server_fetch

    def lf_server_stats(self):
        used, budget = C.c_uint64(), C.c_uint64()
        running, queued = C.c_int32(), C.c_int32()
        self._check(self.L.lf_server_stats(self.s, C.byref(used), C.byref(budget), C.byref(running),
                                           C.byref(queued)), "lf_server_stats")
        return dict(used=used.value, budget=budget.value, running=running.value, queued=queued.value)

    stats = lf_server_stats

    def lf_server_timing(self):
        ms = (C.c_double * 14)()
        self._check(self.L.lf_server_timing(self.s, ms), "lf_server_timing")
        return dict(zip(("admit_ms", "step_ms", "retire_ms", "handover_ms", "tick_ms", "step_wait_ms", "steps",
                         "member_steps", "step_phase_ms", "step_params_ms", "step_launch_ms", "phases_plain",
                         "phases_captured", "phases_replayed"), list(ms)))

    timing = lf_server_timing

    def lf_server_set_graph(self, on=True):
        self._check(self.L.lf_server_set_graph(self.s, 1 if on else 0), "lf_server_set_graph")

    set_graph = lf_server_set_graph

    def lf_server_destroy(self):
        if self.s:
            self.L.lf_server_destroy(self.s)
            self.s = C.c_void_p()

    close = lf_server_destroy

    def lf_server_last_error(self):
        return self.L.lf_server_last_error(self.s).decode(errors="replace")

    def __del__(self):
        try:
            self.lf_server_destroy()
        except Exception:
            pass
