// f1.hip -- F1-Score of the current partition against a reference cover (Methods, "F1-Score
// for Overlapping Communities"): every detected community C' is matched to the reference
// community C with the largest F1(C', C), the harmonic mean of precision |C n C'| / |C'|
// and recall |C n C'| / |C|, i.e. the rational 2 |C n C'| / (|C| + |C'|), evaluated as one
// correctly rounded division; the score is the mean of those maxima over the detected
// communities with at least one member (exact sum rounded once, then one division).
//
// Every non-zero intersection is found from the nodes: a node in C' and in C contributes
// the pair key (C', C) once, so after a radix sort the run length of a key is |C n C'|.
// One thread per run start forms F1 and raises the detected community's maximum (the bit
// patterns of non-negative doubles order like the values); a second pass takes the lowest
// reference id reaching the maximum.
#include "lf_internal.h"

static inline unsigned grid_for(long long n, int block) { return (unsigned)((n + block - 1) / block); }

// pairs contributed by node x: |M'(x)| * |M_ref(x)|
__global__ void k_f1_pairs(const NodeHdr *nh, const long long *roff, long long n, long long *cnt)
{
    const long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (x > n) return;
    cnt[x] = x == n ? 0 : (long long)nh[x].cnt * (roff[x + 1] - roff[x]);
}

__global__ void k_f1_emit(const NodeHdr *nh, const Slot *slot, const long long *roff, const int *rids, long long n,
                          const long long *poff, unsigned long long *keys)
{
    const long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (x >= n) return;
    const NodeHdr hx = nh[x];
    long long p = poff[x];
    for (int t = 0; t < hx.cnt; t++) {
        const unsigned long long hi = (unsigned long long)(unsigned)slot[hx.off + t].comm << 32;
        for (long long a = roff[x]; a < roff[x + 1]; a++) keys[p++] = hi | (unsigned)rids[a];
    }
}

__global__ void k_f1_rsize(const int *rids, long long total, int *rsize)
{
    const long long a = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (a < total) atomicAdd(&rsize[rids[a]], 1);
}

// F1 of the key run starting at i (0 if i does not start a run)
__device__ __forceinline__ bool f1_run(const unsigned long long *k, long long m, long long i, const CommRec *cr,
                                       const int *rsize, int &c, int &r, double &f)
{
    const unsigned long long key = k[i];
    if (i > 0 && k[i - 1] == key) return false;
    long long len = 1;
    while (i + len < m && k[i + len] == key) len++;
    c = (int)(key >> 32);
    r = (int)(unsigned)key;
    f = (double)(2 * len) / (double)((long long)rsize[r] + cr[c].s);
    return true;
}

__global__ void k_f1_max(const unsigned long long *k, long long m, const CommRec *cr, const int *rsize,
                         unsigned long long *best_bits)
{
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= m) return;
    int c, r;
    double f;
    if (f1_run(k, m, i, cr, rsize, c, r, f)) atomicMax(&best_bits[c], (unsigned long long)__double_as_longlong(f));
}

__global__ void k_f1_tie(const unsigned long long *k, long long m, const CommRec *cr, const int *rsize,
                         const unsigned long long *best_bits, int *match)
{
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= m) return;
    int c, r;
    double f;
    if (f1_run(k, m, i, cr, rsize, c, r, f) && (unsigned long long)__double_as_longlong(f) == best_bits[c])
        atomicMin(&match[c], r);
}

__global__ void k_f1_init(int K, int *match)
{
    const long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (c < K) match[c] = 0x7fffffff;
}

__global__ void k_f1_final(const CommRec *cr, int K, const unsigned long long *best_bits, int *match, double *best,
                           unsigned long long *live)
{
    const long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (c >= K) return;
    best[c] = __longlong_as_double((long long)best_bits[c]);
    if (match[c] == 0x7fffffff) match[c] = -1;
    if (cr[c].s > 0) atomicAdd(live, 1ull);
}

extern "C" int lf_cover_f1(lf_handle *h, const int64_t *offsets, const int32_t *ids, int64_t total, uint32_t flags,
                           double *f1, double *best, int32_t *match)
{
    if (!h || !f1) return LF_EINVAL;
    if (h->state < 2) return lf_set_error(h, LF_ESTATE, "no communities yet");
    if (!offsets || total < 0 || (total > 0 && !ids)) return lf_set_error(h, LF_EINVAL, "null cover arrays");
    LF_HIP(h, hipSetDevice(h->device));
    TmpScope tmp_scope(h);
    hipStream_t st = h->stream;
    const int BS = 256;
    const long long n = h->n;
    const int K = h->K;
    const long long *roff = (const long long *)offsets;
    const int *rids = ids;
    if (!(flags & LF_DEVICE_PTR)) {
        long long *o = nullptr;
        int *c = nullptr;
        LF_TRY(lf_tmp_alloc(h, (void **)&o, sizeof(long long) * (n + 1)));
        LF_TRY(lf_tmp_alloc(h, (void **)&c, sizeof(int) * (total > 0 ? total : 1)));
        LF_HIP(h, hipMemcpyAsync(o, offsets, sizeof(long long) * (n + 1), hipMemcpyHostToDevice, st));
        if (total > 0) LF_HIP(h, hipMemcpyAsync(c, ids, sizeof(int) * total, hipMemcpyHostToDevice, st));
        roff = o;
        rids = c;
    }
    int maxid = -1;
    LF_TRY(lf_check_cover(h, roff, rids, total, -1, &maxid));
    const long long R = (long long)maxid + 1;
    long long *pc = nullptr, *poff = nullptr;
    int *rsize = nullptr, *dmatch = nullptr;
    unsigned long long *bbits = nullptr, *live = nullptr;
    double *dbest = nullptr;
    LF_TRY(lf_tmp_alloc(h, (void **)&pc, sizeof(long long) * (n + 1)));
    LF_TRY(lf_tmp_alloc(h, (void **)&poff, sizeof(long long) * (n + 1)));
    LF_TRY(lf_tmp_alloc(h, (void **)&rsize, sizeof(int) * (R > 0 ? R : 1)));
    LF_TRY(lf_tmp_alloc(h, (void **)&dmatch, sizeof(int) * (K > 0 ? K : 1)));
    LF_TRY(lf_tmp_alloc(h, (void **)&bbits, sizeof(unsigned long long) * (K > 0 ? K : 1)));
    LF_TRY(lf_tmp_alloc(h, (void **)&dbest, sizeof(double) * (K > 0 ? K : 1)));
    LF_TRY(lf_tmp_alloc(h, (void **)&live, sizeof(unsigned long long)));
    LF_HIP(h, hipMemsetAsync(rsize, 0, sizeof(int) * (R > 0 ? R : 1), st));
    LF_HIP(h, hipMemsetAsync(bbits, 0, sizeof(unsigned long long) * (K > 0 ? K : 1), st));
    if (K > 0) hipLaunchKernelGGL(k_f1_init, dim3(grid_for(K, BS)), dim3(BS), 0, st, K, dmatch);
    LF_HIP(h, hipMemsetAsync(live, 0, sizeof(unsigned long long), st));
    hipLaunchKernelGGL(k_f1_pairs, dim3(grid_for(n + 1, BS)), dim3(BS), 0, st, h->nh, roff, n, pc);
    LF_TRY(lf_exclusive_scan_i64(h, pc, poff, n + 1));
    long long m = 0;
    LF_HIP(h, hipMemcpyAsync(&m, poff + n, sizeof(long long), hipMemcpyDeviceToHost, st));
    LF_HIP(h, hipStreamSynchronize(st));
    if (m >= (1ll << 31) - 1) return lf_set_error(h, LF_EOVERFLOW, "more than 2^31 - 2 membership pairs");
    if (total > 0) hipLaunchKernelGGL(k_f1_rsize, dim3(grid_for(total, BS)), dim3(BS), 0, st, rids, total, rsize);
    if (m > 0) {
        unsigned long long *keys = nullptr, *alt = nullptr, *sorted = nullptr;
        LF_TRY(lf_tmp_alloc(h, (void **)&keys, sizeof(unsigned long long) * m));
        LF_TRY(lf_tmp_alloc(h, (void **)&alt, sizeof(unsigned long long) * m));
        hipLaunchKernelGGL(k_f1_emit, dim3(grid_for(n, BS)), dim3(BS), 0, st, h->nh, h->slot[h->cur], roff, rids, n,
                           poff, keys);
        LF_TRY(lf_sort_u64(h, keys, alt, m, 64, &sorted));
        hipLaunchKernelGGL(k_f1_max, dim3(grid_for(m, BS)), dim3(BS), 0, st, sorted, m, h->cr, rsize, bbits);
        hipLaunchKernelGGL(k_f1_tie, dim3(grid_for(m, BS)), dim3(BS), 0, st, sorted, m, h->cr, rsize, bbits, dmatch);
    }
    if (K > 0) hipLaunchKernelGGL(k_f1_final, dim3(grid_for(K, BS)), dim3(BS), 0, st, h->cr, K, bbits, dmatch, dbest,
                                  live);
    LF_HIP(h, hipGetLastError());
    double sum = 0.0;
    LF_TRY(lf_exact_sum_dev(h, dbest, K, &sum));
    unsigned long long hl = 0;
    LF_HIP(h, hipMemcpyAsync(&hl, live, sizeof hl, hipMemcpyDeviceToHost, st));
    if (best && K > 0) LF_HIP(h, hipMemcpyAsync(best, dbest, sizeof(double) * K, hipMemcpyDeviceToHost, st));
    if (match && K > 0) LF_HIP(h, hipMemcpyAsync(match, dmatch, sizeof(int) * K, hipMemcpyDeviceToHost, st));
    LF_HIP(h, hipStreamSynchronize(st));
    LF_HIP(h, hipGetLastError());
    *f1 = hl > 0 ? sum / (double)hl : 0.0;
    return LF_OK;
}
