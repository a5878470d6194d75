"""MI355X-native LazyFox hot path (overlapping community detection, arXiv 2210.03211).

Thin Python binding over ``liblazyfox.so`` (C ABI in ``include/lazyfox.h``): every step of
the path runs in the library's HIP kernels; this module only marshals arguments.  If the
library has not been built, importing the binding raises -- there is no CPU fallback.

    import paper_2210_03211_amd as lf
    h = lf.Handle()                       # on cuda:0, torch's current stream
    h.load_graph(n, src, dst)             # numpy int64 (host) or torch int64 cuda tensors
    h.init_communities()
    info = h.run_iterations(queue_size=4096, threshold=0.01, max_iters=50)
    offsets, comm_ids = h.get_memberships()
"""
from ._native import (  # noqa: F401
    Handle, Batch, Server, LazyFoxError, RunInfo, Profile, library_path, load_library,
    LF_OK, LF_EINVAL, LF_ESTATE, LF_ENOMEM, LF_EDEVICE, LF_ERANGE, LF_EOVERFLOW, LF_EAGAIN, LF_EINTERNAL,
    LF_RELABEL, LF_DEVICE_PTR, KERNEL_CLASSES, OPTIONS, PROF_COUNTERS_BIT, PATHS,
)

__all__ = ["Handle", "Batch", "Server", "LazyFoxError", "RunInfo", "Profile", "library_path", "load_library"]
