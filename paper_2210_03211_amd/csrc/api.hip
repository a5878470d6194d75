// api.hip -- the C ABI declared in include/lazyfox.h.
#include <math.h>
#include <stdlib.h>

#include <mutex>

#include "lf_internal.h"

// Scratch of lf_exact_sum_noalloc: the block partial sums, the range flag and the rounded
// result of the exact sum.  Each GPU the library runs on holds its own copy until the
// process ends; host code uses only the per-device address resolved below, never the
// array's name (which is a host-side stand-in).
#define LF_NOALLOC_SCRATCH_BYTES 32768
static __device__ __align__(256) unsigned char scratch[LF_NOALLOC_SCRATCH_BYTES];
static_assert(sizeof(X192) * LF_EXACT_PARTIALS + 256 + sizeof(double) <= LF_NOALLOC_SCRATCH_BYTES,
              "the no-allocation scratch holds the partials, the flag and the result");
#define LF_MAX_DEVICES 64
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[LF_MAX_DEVICES];

// Address of this device's scratch, resolved once per device with that device current.
static int resolve_scratch(int device)
{
    if (device < 0 || device >= LF_MAX_DEVICES) return LF_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return LF_OK;
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
        (void)hipGetLastError();
        return LF_EDEVICE;
    }
    g_scratch_ptr[device] = p;
    return LF_OK;
}

static void *scratch_of(int device)
{
    if (device < 0 || device >= LF_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

extern "C" {

// Releases what a handle under construction already holds (lf_create's failure paths;
// the handle is zero-initialised, so members not created yet are null).
static int create_failed(lf_handle *h, int rc)
{
    if (h->hrep) lf_host_release(h->hrep, sizeof(long long) * 16);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h->allocs;
    delete h->alloc_sizes;
    delete h->tmp_chunks;
    delete h->evpool;
    delete h->evkind;
    delete h->evlaunch;
    free(h);
    return rc;
}

int lf_create(lf_handle **out, int device, void *hip_stream, uint32_t flags)
{
    (void)flags;
    if (!out) return LF_EINVAL;
    *out = nullptr;
    lf_handle *h = (lf_handle *)calloc(1, sizeof(lf_handle));
    if (!h) return LF_ENOMEM;
    h->allocs = new std::vector<void *>();
    h->alloc_sizes = new std::vector<size_t>();
    h->tmp_chunks = new std::vector<TmpChunk>();
    h->evpool = new std::vector<hipEvent_t>();
    h->evkind = new std::vector<int>();
    h->evlaunch = new std::vector<int>();
    h->device = device;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return create_failed(h, LF_EDEVICE);
    if (hipSetDevice(device) != hipSuccess) return create_failed(h, LF_EDEVICE);
    if (resolve_scratch(device) != LF_OK) return create_failed(h, LF_EDEVICE);
    if (hip_stream) {
        h->stream = (hipStream_t)hip_stream;
        h->own_stream = false;
    } else {
        if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) {
            h->stream = nullptr;
            return create_failed(h, LF_EDEVICE);
        }
        h->own_stream = true;
    }
    if (hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess)
        return create_failed(h, LF_EDEVICE);
    if (lf_host_alloc((void **)&h->hrep, sizeof(long long) * 16) != LF_OK) {
        h->hrep = nullptr;
        return create_failed(h, LF_ENOMEM);
    }
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    h->eval_wave_cap = 128;
    h->eval_med_cap = 512;
    h->eval_grp_cap = 2048;
    h->prof_stride = 1;
    h->hub_blocks = 2 * cus;
    h->refresh_blocks = 2 * cus;
    h->K = -1;
    *out = h;
    return LF_OK;
}

int lf_destroy(lf_handle *h)
{
    if (!h) return LF_OK;
    (void)hipSetDevice(h->device);
    (void)hipStreamSynchronize(h->stream);
    lf_phase_graphs_drop(h);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    // the handle's work has completed on its stream: its blocks can serve other handles
    for (size_t k = 0; k < h->allocs->size(); k++) lf_dev_release(h->device, (*h->allocs)[k], (*h->alloc_sizes)[k]);
    delete h->allocs;
    delete h->alloc_sizes;
    delete h->tmp_chunks;
    for (hipEvent_t e : *h->evpool) (void)hipEventDestroy(e);
    delete h->evpool;
    delete h->evkind;
    delete h->evlaunch;
    (void)hipEventDestroy(h->ev0);
    (void)hipEventDestroy(h->ev1);
    if (h->own_stream) (void)hipStreamDestroy(h->stream);
    if (h->hqoff) lf_host_release(h->hqoff, sizeof(long long) * h->hqoff_len);
    if (h->hrep) lf_host_release(h->hrep, sizeof(long long) * 16);
    free(h);
    return LF_OK;
}

const char *lf_last_error(lf_handle *h) { return h ? h->err : "null handle"; }

static void reset_graph(lf_handle *h)
{
    lf_free_partition(h);
    void **ptrs[] = {(void **)&h->rowptr, (void **)&h->col, (void **)&h->deg, (void **)&h->orig_id,
                     (void **)&h->tri, (void **)&h->ccl, (void **)&h->order, (void **)&h->rank,
                     (void **)&h->col_rank};
    for (void **p : ptrs) {
        lf_dev_free(h, *p);
        *p = nullptr;
    }
    h->n = h->ne = 0;
    h->K = -1;
    h->state = 0;
    h->cc = 0.0;
    h->T = 0;
    h->Wt = 0.0;
}

int lf_load_graph(lf_handle *h, int64_t n, int64_t n_pairs, const int64_t *src, const int64_t *dst,
                  uint32_t flags)
{
    if (!h) return LF_EINVAL;
    LF_HIP(h, hipSetDevice(h->device));
    if (n_pairs < 0 || (!(flags & LF_RELABEL) && n < 0))
        return lf_set_error(h, LF_EINVAL, "negative size");
    if (n_pairs > 0 && (!src || !dst)) return lf_set_error(h, LF_EINVAL, "null edge arrays");
    if (n_pairs >= (1ll << 31) - 1) return lf_set_error(h, LF_EOVERFLOW, "n_pairs >= 2^31 - 1");
    if (!(flags & LF_RELABEL) && n >= (1ll << 31) - 1)
        return lf_set_error(h, LF_EOVERFLOW, "n >= 2^31 - 1");
    reset_graph(h);
    LF_HIP(h, hipStreamSynchronize(h->stream));
    LF_TRY(lf_prof_begin(h, LF_K_BUILD));
    int rc = lf_build_graph(h, n, n_pairs, (const long long *)src, (const long long *)dst, flags);
    if (rc != LF_OK) {
        char keep[512];
        memcpy(keep, h->err, sizeof keep);
        reset_graph(h);
        memcpy(h->err, keep, sizeof keep);
        return rc;
    }
    LF_TRY(lf_prof_end(h, LF_K_BUILD, 8));
    LF_TRY(lf_prof_flush(h));
    h->state = 1;
    return LF_OK;
}

int lf_init_communities(lf_handle *h)
{
    if (!h) return LF_EINVAL;
    if (h->state < 1) return lf_set_error(h, LF_ESTATE, "lf_load_graph has not been called");
    LF_HIP(h, hipSetDevice(h->device));
    if (h->state == 1 || !h->order) {
        void **ptrs[] = {(void **)&h->tri, (void **)&h->ccl, (void **)&h->order, (void **)&h->rank,
                     (void **)&h->col_rank};
        for (void **p : ptrs) {
            lf_dev_free(h, *p);
            *p = nullptr;
        }
        LF_TRY(lf_node_stats(h));
    }
    h->state = 1;
    LF_TRY(lf_initial_clustering(h));
    h->state = 2;
    return LF_OK;
}

int lf_init_from_memberships(lf_handle *h, const int64_t *offsets, const int32_t *comm_ids, int64_t total,
                             int32_t n_comms, uint32_t flags)
{
    if (!h) return LF_EINVAL;
    if (h->state < 1) return lf_set_error(h, LF_ESTATE, "lf_load_graph has not been called");
    if (!offsets || total < 0 || (total > 0 && !comm_ids))
        return lf_set_error(h, LF_EINVAL, "null cover arrays or negative total");
    if (total + h->n >= (1ll << 31) - 1) return lf_set_error(h, LF_EOVERFLOW, "cover too large");
    LF_HIP(h, hipSetDevice(h->device));
    if (h->state == 1 || !h->order) {
        void **ptrs[] = {(void **)&h->tri, (void **)&h->ccl, (void **)&h->order, (void **)&h->rank,
                     (void **)&h->col_rank};
        for (void **p : ptrs) {
            lf_dev_free(h, *p);
            *p = nullptr;
        }
        h->state = 1;
        LF_TRY(lf_node_stats(h));
    }
    TmpScope tmp_scope(h);
    const long long *doff = (const long long *)offsets;
    const int *dids = comm_ids;
    if (!(flags & LF_DEVICE_PTR)) {          // host arrays: staged into device temporaries
        long long *o = nullptr;
        int *c = nullptr;
        LF_TRY(lf_tmp_alloc(h, (void **)&o, sizeof(long long) * (h->n + 1)));
        LF_TRY(lf_tmp_alloc(h, (void **)&c, sizeof(int) * (total > 0 ? total : 1)));
        LF_HIP(h, hipMemcpyAsync(o, offsets, sizeof(long long) * (h->n + 1), hipMemcpyHostToDevice, h->stream));
        if (total > 0)
            LF_HIP(h, hipMemcpyAsync(c, comm_ids, sizeof(int) * total, hipMemcpyHostToDevice, h->stream));
        doff = o;
        dids = c;
    }
    LF_TRY(lf_partition_from_cover(h, doff, dids, total, n_comms));
    h->state = 2;
    return LF_OK;
}

int lf_run_iterations(lf_handle *h, int32_t queue_size, double threshold, int32_t max_iters, lf_run_info *out)
{
    if (!h) return LF_EINVAL;
    if (queue_size < 1 || isnan(threshold) || threshold < 0.0 || max_iters < 0)
        return lf_set_error(h, LF_EINVAL, "bad argument (queue_size %d, threshold %g, max_iters %d)", queue_size,
                            threshold, max_iters);
    if (h->state < 2) return lf_set_error(h, LF_ESTATE, "lf_init_communities has not been called");
    LF_HIP(h, hipSetDevice(h->device));
    return lf_iterate(h, queue_size, threshold, max_iters, out);
}

int lf_get_memberships(lf_handle *h, int64_t *offsets, int32_t *comm_ids, int64_t capacity, int64_t *total)
{
    if (!h || !total) return LF_EINVAL;
    if (h->state < 2) return lf_set_error(h, LF_ESTATE, "no communities yet");
    LF_HIP(h, hipSetDevice(h->device));
    long long tot = 0;
    int rc = lf_fetch_memberships(h, (long long *)offsets, comm_ids, capacity, &tot,
                                  nullptr);
    *total = tot;
    return rc;
}

int lf_get_in_counts(lf_handle *h, int32_t *in, int64_t capacity)
{
    if (!h || !in) return LF_EINVAL;
    if (h->state < 2) return lf_set_error(h, LF_ESTATE, "no communities yet");
    LF_HIP(h, hipSetDevice(h->device));
    std::vector<long long> off((size_t)h->n + 1);
    long long tot = 0;
    return lf_fetch_memberships(h, off.data(), nullptr, capacity, &tot, in);
}

int lf_get_graph_info(lf_handle *h, int64_t *n, int64_t *nedges, int64_t *ncommunities)
{
    if (!h) return LF_EINVAL;
    if (n) *n = h->n;
    if (nedges) *nedges = h->ne;
    if (ncommunities) *ncommunities = h->state >= 2 ? h->K : -1;
    return LF_OK;
}

int lf_get_csr(lf_handle *h, int64_t *rowptr, int32_t *col, int64_t *orig_ids)
{
    if (!h) return LF_EINVAL;
    if (h->state < 1) return lf_set_error(h, LF_ESTATE, "no graph loaded");
    LF_HIP(h, hipSetDevice(h->device));
    // blocking copies go through the null stream, which does not wait for a non-blocking one
    LF_HIP(h, hipStreamSynchronize(h->stream));
    if (rowptr) LF_HIP(h, hipMemcpy(rowptr, h->rowptr, sizeof(long long) * (h->n + 1), hipMemcpyDeviceToHost));
    if (col && h->ne > 0) LF_HIP(h, hipMemcpy(col, h->col, sizeof(int) * 2 * h->ne, hipMemcpyDeviceToHost));
    if (orig_ids && h->n > 0) LF_HIP(h, hipMemcpy(orig_ids, h->orig_id, sizeof(long long) * h->n, hipMemcpyDeviceToHost));
    return LF_OK;
}

int lf_get_node_stats(lf_handle *h, int64_t *tri, double *cc_local, int32_t *order)
{
    if (!h) return LF_EINVAL;
    if (h->state < 2) return lf_set_error(h, LF_ESTATE, "lf_init_communities has not been called");
    LF_HIP(h, hipSetDevice(h->device));
    LF_HIP(h, hipStreamSynchronize(h->stream));
    size_t n = (size_t)h->n;
    if (n == 0) return LF_OK;
    if (tri) LF_HIP(h, hipMemcpy(tri, h->tri, sizeof(long long) * n, hipMemcpyDeviceToHost));
    if (cc_local) LF_HIP(h, hipMemcpy(cc_local, h->ccl, sizeof(double) * n, hipMemcpyDeviceToHost));
    if (order) LF_HIP(h, hipMemcpy(order, h->order, sizeof(int) * n, hipMemcpyDeviceToHost));
    return LF_OK;
}

int lf_get_scores(lf_handle *h, double *wcc_hat, double *cc, int64_t *triangles, double *wtilde)
{
    if (!h) return LF_EINVAL;
    if (h->state < 2) return lf_set_error(h, LF_ESTATE, "lf_init_communities has not been called");
    if (cc) *cc = h->cc;
    if (triangles) *triangles = h->T;
    if (wtilde) *wtilde = h->Wt;
    if (wcc_hat) *wcc_hat = h->cc > 0.0 ? h->Wt / h->cc : 0.0;
    return LF_OK;
}

int lf_get_communities(lf_handle *h, int32_t *size, int64_t *internal_edges, double *score)
{
    if (!h) return LF_EINVAL;
    if (h->state < 2) return lf_set_error(h, LF_ESTATE, "lf_init_communities has not been called");
    LF_HIP(h, hipSetDevice(h->device));
    LF_HIP(h, hipStreamSynchronize(h->stream));
    size_t K = (size_t)h->K;
    if (K == 0) return LF_OK;
    std::vector<CommRec> rec(K);
    LF_HIP(h, hipMemcpy(rec.data(), h->cr, sizeof(CommRec) * K, hipMemcpyDeviceToHost));
    for (size_t c = 0; c < K; c++) {
        if (size) size[c] = rec[c].s;
        if (internal_edges) internal_edges[c] = rec[c].m;
        if (score) score[c] = rec[c].W;
    }
    return LF_OK;
}

int lf_set_profiling(lf_handle *h, int mask)
{
    if (!h) return LF_EINVAL;
    h->profiling = mask & ((1 << (LF_PROF_COUNTERS_BIT + 1)) - 1);
    return LF_OK;
}

int lf_get_profile(lf_handle *h, lf_profile *out)
{
    if (!h || !out) return LF_EINVAL;
    *out = h->prof;
    return LF_OK;
}

int lf_reset_profile(lf_handle *h)
{
    if (!h) return LF_EINVAL;
    memset(&h->prof, 0, sizeof h->prof);
    return LF_OK;
}

int lf_set_option(lf_handle *h, int option, int64_t value)
{
    if (!h) return LF_EINVAL;
    switch (option) {
    case LF_OPT_TRI_LDS_CAP:
        if (value < 0 || value > (1 << 24)) break;
        h->tri_lds_cap = (int)value;
        return LF_OK;
    case LF_OPT_HUB_BLOCKS:
        if (value < 1 || value > 65536) break;
        h->hub_blocks = (int)value;
        return LF_OK;
    case LF_OPT_REFRESH_BLOCKS:
        if (value < 1 || value > 65536) break;
        h->refresh_blocks = (int)value;
        return LF_OK;
    case LF_OPT_WAVE_TABLE:
        if (value < 16 || value > 128 || (value & (value - 1))) break;
        h->eval_wave_cap = (int)value;
        return LF_OK;
    case LF_OPT_MED_TABLE:
        if (value < 16 || value > 512 || (value & (value - 1))) break;
        h->eval_med_cap = (int)value;
        return LF_OK;
    case LF_OPT_GRP_TABLE:
        if (value < 16 || value > 2048 || (value & (value - 1))) break;
        h->eval_grp_cap = (int)value;
        return LF_OK;
    case LF_OPT_PROF_STRIDE:
        if (value < 1 || value > 65536) break;
        h->prof_stride = (int)value;
        memset(h->prof_seq, 0, sizeof h->prof_seq);
        return LF_OK;
    default:
        return lf_set_error(h, LF_EINVAL, "unknown option %d", option);
    }
    return lf_set_error(h, LF_EINVAL, "option %d: value %lld out of range", option, (long long)value);
}

int lf_get_option(lf_handle *h, int option, int64_t *value)
{
    if (!h || !value) return LF_EINVAL;
    switch (option) {
    case LF_OPT_TRI_LDS_CAP: *value = h->tri_lds_cap; return LF_OK;
    case LF_OPT_HUB_BLOCKS: *value = h->hub_blocks; return LF_OK;
    case LF_OPT_REFRESH_BLOCKS: *value = h->refresh_blocks; return LF_OK;
    case LF_OPT_WAVE_TABLE: *value = h->eval_wave_cap; return LF_OK;
    case LF_OPT_MED_TABLE: *value = h->eval_med_cap; return LF_OK;
    case LF_OPT_GRP_TABLE: *value = h->eval_grp_cap; return LF_OK;
    case LF_OPT_PROF_STRIDE: *value = h->prof_stride; return LF_OK;
    default: return lf_set_error(h, LF_EINVAL, "unknown option %d", option);
    }
}

int lf_debug_exact_sum(lf_handle *h, const double *values_dev, int64_t n, double *out)
{
    if (!h || !out || n < 0 || (n > 0 && !values_dev)) return LF_EINVAL;
    LF_HIP(h, hipSetDevice(h->device));
    return lf_exact_sum_dev(h, values_dev, n, out);
}

int lf_exact_sum_noalloc(lf_handle *h, const double *values_dev, int64_t n, double *out)
{
    if (!h || !out || n < 0 || (n > 0 && !values_dev)) return LF_EINVAL;
    if (n > LF_NOALLOC_MAX_VALUES)
        return lf_set_error(h, LF_EINVAL, "lf_exact_sum_noalloc: n = %lld exceeds the maximum 2^40",
                            (long long)n);
    LF_HIP(h, hipSetDevice(h->device));
    unsigned char *sp = (unsigned char *)scratch_of(h->device);
    if (!sp) return lf_set_error(h, LF_EDEVICE, "no-allocation scratch not resolved for device %d", h->device);
    X192 *part = (X192 *)sp;
    int *err = (int *)(sp + sizeof(X192) * LF_EXACT_PARTIALS);
    double *dout = (double *)(sp + sizeof(X192) * LF_EXACT_PARTIALS + 256);
    return lf_exact_sum_run(h, values_dev, n, out, part, err, dout);
}

int lf_debug_sort_pairs(lf_handle *h, uint64_t *keys_dev, int32_t *vals_dev, int64_t n, int32_t end_bit)
{
    if (!h || n < 0 || (n > 0 && !keys_dev) || end_bit < 0 || end_bit > 64) return LF_EINVAL;
    if (n >= (1ll << 31)) return lf_set_error(h, LF_EOVERFLOW, "n >= 2^31");
    LF_HIP(h, hipSetDevice(h->device));
    return lf_sort_dev_u64(h, (unsigned long long *)keys_dev, (int *)vals_dev, n, end_bit);
}

int lf_debug_sort_pairs_u32(lf_handle *h, uint32_t *keys_dev, int32_t *vals_dev, int64_t n)
{
    if (!h || n < 0 || (n > 0 && (!keys_dev || !vals_dev))) return LF_EINVAL;
    if (n >= (1ll << 31)) return lf_set_error(h, LF_EOVERFLOW, "n >= 2^31");
    LF_HIP(h, hipSetDevice(h->device));
    return lf_sort_dev_u32(h, (unsigned *)keys_dev, (int *)vals_dev, n);
}

int lf_debug_exclusive_scan(lf_handle *h, const void *in_dev, int32_t in_bytes, int64_t *out_dev, int64_t n)
{
    if (!h || n < 0 || (in_bytes != 4 && in_bytes != 8) || (n > 0 && (!in_dev || !out_dev))) return LF_EINVAL;
    LF_HIP(h, hipSetDevice(h->device));
    return lf_scan_dev(h, in_dev, in_bytes, (long long *)out_dev, n);
}

}  // extern "C"
