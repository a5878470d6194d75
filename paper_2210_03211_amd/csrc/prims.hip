// prims.hip -- library primitives: device radix sorts and prefix sums (hipCUB), plus
// the handle's allocation registry and error/profiling helpers.
#include <stdarg.h>

#include <hipcub/hipcub.hpp>

#include "lf_internal.h"

int lf_set_error(lf_handle *h, int code, const char *fmt, ...)
{
    if (h) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(h->err, sizeof h->err, fmt, ap);
        va_end(ap);
    }
    return code;
}

int lf_dev_alloc(lf_handle *h, void **p, size_t bytes)
{
    *p = nullptr;
    if (bytes == 0) bytes = 256;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return lf_set_error(h, LF_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    h->allocs->push_back(*p);
    h->alloc_sizes->push_back(bytes);
    h->dev_bytes += bytes;
    if (h->dev_bytes > h->dev_bytes_peak) h->dev_bytes_peak = h->dev_bytes;
    return LF_OK;
}

void lf_dev_free(lf_handle *h, void *p)
{
    if (!p) return;
    for (size_t k = 0; k < h->allocs->size(); k++)
        if ((*h->allocs)[k] == p) {
            h->dev_bytes -= (*h->alloc_sizes)[k];
            (*h->allocs)[k] = h->allocs->back();
            (*h->alloc_sizes)[k] = h->alloc_sizes->back();
            h->allocs->pop_back();
            h->alloc_sizes->pop_back();
            break;
        }
    (void)hipFree(p);
}

// Scratch arena of a handle: temporaries of one host routine are carved from chunks the
// handle keeps, so iteration starts and ends allocate nothing once warm (hipFree would
// synchronise the whole device).  Marks and releases nest like a stack; memory handed out
// after a release is only used by work queued later on the same stream.
int lf_tmp_alloc(lf_handle *h, void **p, size_t bytes)
{
    *p = nullptr;
    bytes = (bytes + 255) & ~(size_t)255;
    if (bytes == 0) bytes = 256;
    std::vector<TmpChunk> &ch = *h->tmp_chunks;
    while (true) {
        if (h->tmp_chunk < (int)ch.size()) {
            TmpChunk &c = ch[h->tmp_chunk];
            if (h->tmp_off + bytes <= c.size) {
                *p = (char *)c.ptr + h->tmp_off;
                h->tmp_off += bytes;
                return LF_OK;
            }
            if (h->tmp_off == 0) {                  // an unused chunk that is too small
                lf_dev_free(h, c.ptr);
                c.ptr = nullptr;
                size_t want = bytes > 2 * c.size ? bytes : 2 * c.size;
                LF_TRY(lf_dev_alloc(h, &c.ptr, want));
                c.size = want;
                continue;
            }
            h->tmp_chunk++;
            h->tmp_off = 0;
            continue;
        }
        size_t last = ch.empty() ? 0 : ch.back().size;
        size_t want = bytes;
        if (want < 2 * last) want = 2 * last;
        if (want < ((size_t)4 << 20)) want = (size_t)4 << 20;
        TmpChunk c;
        LF_TRY(lf_dev_alloc(h, &c.ptr, want));
        c.size = want;
        ch.push_back(c);
    }
}

TmpMark lf_tmp_mark(lf_handle *h) { return TmpMark{h->tmp_chunk, h->tmp_off}; }

void lf_tmp_release(lf_handle *h, TmpMark m)
{
    h->tmp_chunk = m.chunk;
    h->tmp_off = m.off;
}

int lf_ensure_tmp(lf_handle *h, size_t bytes)
{
    if (bytes <= h->tmp_bytes) return LF_OK;
    if (h->tmp) {
        LF_HIP(h, hipStreamSynchronize(h->stream));
        lf_dev_free(h, h->tmp);
        h->tmp = nullptr;
    }
    size_t want = bytes + bytes / 4 + 4096;
    LF_TRY(lf_dev_alloc(h, &h->tmp, want));
    h->tmp_bytes = want;
    return LF_OK;
}

static bool prof_on(lf_handle *h, int kind) { return kind < LF_K_COUNT && ((h->profiling >> kind) & 1); }

int lf_prof_begin(lf_handle *h, int kind) { return lf_prof_begin_on(h, kind, h->stream); }
int lf_prof_end(lf_handle *h, int kind, int launches) { return lf_prof_end_on(h, kind, launches, h->stream); }

int lf_prof_begin_on(lf_handle *h, int kind, hipStream_t st)
{
    if (!prof_on(h, kind)) return LF_OK;
    if (h->evused >= 4096) LF_TRY(lf_prof_flush(h));
    size_t need = 2 * (size_t)(h->evused + 1);
    while (h->evpool->size() < need) {
        hipEvent_t e;
        LF_HIP(h, hipEventCreate(&e));
        h->evpool->push_back(e);
    }
    LF_HIP(h, hipEventRecord((*h->evpool)[2 * h->evused], st));
    return LF_OK;
}

int lf_prof_end_on(lf_handle *h, int kind, int launches, hipStream_t st)
{
    if (!prof_on(h, kind)) return LF_OK;
    LF_HIP(h, hipEventRecord((*h->evpool)[2 * h->evused + 1], st));
    if ((int)h->evkind->size() <= h->evused) {
        h->evkind->push_back(kind);
        h->evlaunch->push_back(launches);
    } else {
        (*h->evkind)[h->evused] = kind;
        (*h->evlaunch)[h->evused] = launches;
    }
    h->evused++;
    return LF_OK;
}

int lf_prof_flush(lf_handle *h)
{
    if (h->evused == 0) return LF_OK;
    for (int k = 0; k < h->evused; k++) {       // pairs may sit on different streams
        float ms = 0.f;
        LF_HIP(h, hipEventSynchronize((*h->evpool)[2 * k + 1]));
        LF_HIP(h, hipEventElapsedTime(&ms, (*h->evpool)[2 * k], (*h->evpool)[2 * k + 1]));
        int kind = (*h->evkind)[k];
        h->prof.ms[kind] += ms;
        h->prof.launches[kind] += (*h->evlaunch)[k];
    }
    h->evused = 0;
    return LF_OK;
}

int lf_sort_u64(lf_handle *h, unsigned long long *keys, unsigned long long *keys_alt, long long n,
                int end_bit, unsigned long long **result)
{
    *result = keys;
    if (n <= 1) return LF_OK;
    hipcub::DoubleBuffer<unsigned long long> db(keys, keys_alt);
    size_t bytes = 0;
    LF_HIP(h, hipcub::DeviceRadixSort::SortKeys(nullptr, bytes, db, (int)n, 0, end_bit, h->stream));
    LF_TRY(lf_ensure_tmp(h, bytes));
    bytes = h->tmp_bytes;
    LF_HIP(h, hipcub::DeviceRadixSort::SortKeys(h->tmp, bytes, db, (int)n, 0, end_bit, h->stream));
    *result = db.Current();
    return LF_OK;
}

int lf_sort_pairs_u64_i32(lf_handle *h, unsigned long long *keys, unsigned long long *keys_alt,
                          int *vals, int *vals_alt, long long n, int end_bit,
                          unsigned long long **rkeys, int **rvals)
{
    *rkeys = keys;
    *rvals = vals;
    if (n <= 1) return LF_OK;
    hipcub::DoubleBuffer<unsigned long long> dk(keys, keys_alt);
    hipcub::DoubleBuffer<int> dv(vals, vals_alt);
    size_t bytes = 0;
    LF_HIP(h, hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, dk, dv, (int)n, 0, end_bit, h->stream));
    LF_TRY(lf_ensure_tmp(h, bytes));
    bytes = h->tmp_bytes;
    LF_HIP(h, hipcub::DeviceRadixSort::SortPairs(h->tmp, bytes, dk, dv, (int)n, 0, end_bit, h->stream));
    *rkeys = dk.Current();
    *rvals = dv.Current();
    return LF_OK;
}

int lf_sort_pairs_u32_i32(lf_handle *h, unsigned *keys, unsigned *keys_alt, int *vals,
                          int *vals_alt, long long n, unsigned **rkeys, int **rvals)
{
    *rkeys = keys;
    *rvals = vals;
    if (n <= 1) return LF_OK;
    hipcub::DoubleBuffer<unsigned> dk(keys, keys_alt);
    hipcub::DoubleBuffer<int> dv(vals, vals_alt);
    size_t bytes = 0;
    LF_HIP(h, hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, dk, dv, (int)n, 0, 32, h->stream));
    LF_TRY(lf_ensure_tmp(h, bytes));
    bytes = h->tmp_bytes;
    LF_HIP(h, hipcub::DeviceRadixSort::SortPairs(h->tmp, bytes, dk, dv, (int)n, 0, 32, h->stream));
    *rkeys = dk.Current();
    *rvals = dv.Current();
    return LF_OK;
}

int lf_exclusive_scan_i64(lf_handle *h, const long long *in, long long *out, long long n)
{
    if (n <= 0) return LF_OK;
    size_t bytes = 0;
    LF_HIP(h, hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, in, out, (int)n, h->stream));
    LF_TRY(lf_ensure_tmp(h, bytes));
    bytes = h->tmp_bytes;
    LF_HIP(h, hipcub::DeviceScan::ExclusiveSum(h->tmp, bytes, in, out, (int)n, h->stream));
    return LF_OK;
}

struct I32ToI64 {
    __host__ __device__ long long operator()(const int &v) const { return (long long)v; }
};

int lf_exclusive_scan_i32_to_i64(lf_handle *h, const int *in, long long *out, long long n)
{
    if (n <= 0) return LF_OK;
    hipcub::TransformInputIterator<long long, I32ToI64, const int *> it(in, I32ToI64());
    size_t bytes = 0;
    LF_HIP(h, hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, it, out, (int)n, h->stream));
    LF_TRY(lf_ensure_tmp(h, bytes));
    bytes = h->tmp_bytes;
    LF_HIP(h, hipcub::DeviceScan::ExclusiveSum(h->tmp, bytes, it, out, (int)n, h->stream));
    return LF_OK;
}
