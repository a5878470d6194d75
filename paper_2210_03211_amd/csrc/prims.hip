// prims.hip -- library primitives: device-wide LSD radix sorts and exclusive prefix sums
// written for gfx950 (wave64 ballots, LDS tiles), plus the handle's allocation registry
// and error/profiling helpers.
#include <map>
#include <mutex>
#include <stdarg.h>
#include <utility>

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

// Device blocks of destroyed handles, kept per device and size class for later handles.
// hipFree waits for the whole device, so a serving loop that retires jobs while others
// run would stall the device at every retirement; a block goes back to HIP only when the
// cache is full or the block is large.  Blocks are allocated at their class size (eight
// classes per power of two), so one class serves every request it covers.
namespace {
struct BlockCache {
    std::mutex mu;
    std::map<std::pair<int, size_t>, std::vector<void *>> free;   // device blocks
    std::map<size_t, std::vector<void *>> host;                  // pinned host blocks
    size_t bytes = 0;
};
BlockCache &block_cache()
{
    static BlockCache *c = new BlockCache();   // never destroyed: handles may outlive statics
    return *c;
}
constexpr size_t CACHE_BLOCK_MAX = 256ull << 20;
constexpr size_t CACHE_TOTAL_MAX = 8ull << 30;

size_t size_class(size_t b)
{
    if (b <= 256) return 256;
    const int lg = 63 - __builtin_clzll((unsigned long long)(b - 1));    // 2^lg < b <= 2^(lg+1)
    const size_t step = (size_t)1 << (lg - 3);
    return (b + step - 1) / step * step;
}
}  // namespace

size_t lf_alloc_class(size_t bytes) { return size_class(bytes == 0 ? 256 : bytes); }

// a block whose last use on the device has completed (the caller has synchronised)
void lf_dev_release(int device, void *p, size_t bytes)
{
    if (!p) return;
    BlockCache &c = block_cache();
    if (bytes <= CACHE_BLOCK_MAX && bytes == size_class(bytes)) {
        std::lock_guard<std::mutex> g(c.mu);
        if (c.bytes + bytes <= CACHE_TOTAL_MAX) {
            c.free[{device, bytes}].push_back(p);
            c.bytes += bytes;
            return;
        }
    }
    (void)hipFree(p);
}

// pinned host memory of the same class scheme (hipHostFree may wait for the device too)
int lf_host_alloc(void **p, size_t bytes)
{
    *p = nullptr;
    bytes = lf_alloc_class(bytes);
    {
        BlockCache &c = block_cache();
        std::lock_guard<std::mutex> g(c.mu);
        auto it = c.host.find(bytes);
        if (it != c.host.end() && !it->second.empty()) {
            *p = it->second.back();
            it->second.pop_back();
            return LF_OK;
        }
    }
    if (hipHostMalloc(p, bytes, hipHostMallocDefault) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return LF_ENOMEM;
    }
    return LF_OK;
}

// a pinned block no pending copy writes any more, of the size lf_host_alloc was asked for
void lf_host_release(void *p, size_t bytes)
{
    if (!p) return;
    bytes = lf_alloc_class(bytes);
    if (bytes <= ((size_t)1 << 20)) {
        BlockCache &c = block_cache();
        std::lock_guard<std::mutex> g(c.mu);
        if (c.host[bytes].size() < 4096) {
            c.host[bytes].push_back(p);
            return;
        }
    }
    (void)hipHostFree(p);
}

// zero `bytes` (a multiple of 4) at p with a kernel on the handle's stream: the iteration
// starts and ends, which a batch captures into graphs, clear with kernels only
__global__ void k_zero_words(unsigned *p, long long words)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < words;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = 0u;
}

int lf_zero(lf_handle *h, void *p, size_t bytes)
{
    if (bytes % 4 != 0) return lf_set_error(h, LF_EINTERNAL, "lf_zero of %zu bytes", bytes);
    const long long words = (long long)(bytes / 4);
    if (words == 0) return LF_OK;
    long long g = (words + 255) / 256;
    if (g > 1024) g = 1024;
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)g), dim3(256), 0, h->stream, (unsigned *)p, words);
    LF_HIP(h, hipGetLastError());
    return LF_OK;
}

int lf_dev_alloc(lf_handle *h, void **p, size_t bytes)
{
    *p = nullptr;
    bytes = lf_alloc_class(bytes);
    if (bytes <= CACHE_BLOCK_MAX) {
        BlockCache &c = block_cache();
        std::lock_guard<std::mutex> g(c.mu);
        auto it = c.free.find({h->device, bytes});
        if (it != c.free.end() && !it->second.empty()) {
            *p = it->second.back();
            it->second.pop_back();
            c.bytes -= bytes;
        }
    }
    hipError_t e = *p ? hipSuccess : hipMalloc(p, bytes);
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
    // a batch member's superseded block may still be read by work queued on the shared
    // stream: it stays the handle's until lf_destroy, which waits for the handle's work
    // (no hipFree here, which would wait for the whole device)
    if (h->phase_graphs) return;
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

static bool prof_on(lf_handle *h, int kind) { return kind < LF_K_COUNT && ((h->profiling >> kind) & 1); }

int lf_prof_begin(lf_handle *h, int kind) { return lf_prof_begin_on(h, kind, h->stream); }
int lf_prof_end(lf_handle *h, int kind, int launches) { return lf_prof_end_on(h, kind, launches, h->stream); }

// the per-queue kernel classes, which a stride > 1 samples
static bool per_queue_class(int kind) { return kind >= LF_K_EVAL && kind <= LF_K_REFRESH; }

int lf_prof_begin_on(lf_handle *h, int kind, hipStream_t st)
{
    if (!prof_on(h, kind)) return LF_OK;
    if (per_queue_class(kind) && h->prof_stride > 1 && (h->prof_seq[kind]++ % h->prof_stride) != 0) {
        h->prof_skip |= 1 << kind;
        return LF_OK;
    }
    h->prof_skip &= ~(1 << kind);
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
    if ((h->prof_skip >> kind) & 1) {
        h->prof_skip &= ~(1 << kind);
        return LF_OK;
    }
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

// ------------------------------------------------------------------------------------
// device-wide exclusive prefix sum (64-bit results)
// ------------------------------------------------------------------------------------
// Reduce-then-scan over tiles of SCAN_TILE elements: one pass sums every tile, the tile
// sums are scanned the same way (recursively, a single tile at the top), and a last
// pass scans every tile from its offset.  Each tile is staged through LDS so that the
// global loads and stores are coalesced while every thread scans SCAN_ITEMS
// consecutive elements.  in and out may be the same array.
#define PW 64                     // wavefront width
#define SCAN_BLOCK 256
#define SCAN_ITEMS 16
#define SCAN_TILE (SCAN_BLOCK * SCAN_ITEMS)
#define SCAN_PAD(p) ((p) + ((p) >> 4))   // one spare word per 16: fewer LDS bank conflicts

static inline unsigned grid_of(long long n, long long per) { return (unsigned)((n + per - 1) / per); }

// exclusive prefix of v over the block's threads; *total gets the block's sum
__device__ __forceinline__ long long block_excl_scan(long long v, long long *s_w, long long *total)
{
    const int lane = threadIdx.x & (PW - 1), wv = threadIdx.x / PW;
    long long incl = v;
    for (int o = 1; o < PW; o <<= 1) {
        long long t = __shfl_up(incl, o, PW);
        if (lane >= o) incl += t;
    }
    if (lane == PW - 1) s_w[wv] = incl;
    __syncthreads();
    long long off = 0, tot = 0;
    for (int w = 0; w < SCAN_BLOCK / PW; w++) {
        long long t = s_w[w];
        if (w < wv) off += t;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return off + incl - v;
}

template <typename T>
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_reduce(const T *in, long long n, long long *sums)
{
    __shared__ long long s_w[SCAN_BLOCK / PW];
    const long long base = (long long)blockIdx.x * SCAN_TILE;
    long long acc = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        long long p = base + i * SCAN_BLOCK + threadIdx.x;
        if (p < n) acc += (long long)in[p];
    }
    long long tot;
    (void)block_excl_scan(acc, s_w, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// offs: first value of every tile (nullptr: a single tile starting at 0)
template <typename T>
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_down(const T *in, long long *out, long long n,
                                                          const long long *offs)
{
    __shared__ long long tile[SCAN_PAD(SCAN_TILE)];
    __shared__ long long s_w[SCAN_BLOCK / PW];
    const long long base = (long long)blockIdx.x * SCAN_TILE;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        const int q = i * SCAN_BLOCK + threadIdx.x;
        const long long p = base + q;
        tile[SCAN_PAD(q)] = p < n ? (long long)in[p] : 0;
    }
    __syncthreads();
    const int q0 = threadIdx.x * SCAN_ITEMS;
    long long v = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) v += tile[SCAN_PAD(q0 + i)];
    long long tot;
    long long run = block_excl_scan(v, s_w, &tot) + (offs ? offs[blockIdx.x] : 0);
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        const long long x = tile[SCAN_PAD(q0 + i)];
        tile[SCAN_PAD(q0 + i)] = run;
        run += x;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        const int q = i * SCAN_BLOCK + threadIdx.x;
        const long long p = base + q;
        if (p < n) out[p] = tile[SCAN_PAD(q)];
    }
}

template <typename T>
static int scan_impl(lf_handle *h, const T *in, long long *out, long long n)
{
    if (n <= 0) return LF_OK;
    hipStream_t st = h->stream;
    const long long nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 1) {
        hipLaunchKernelGGL(k_scan_down<T>, dim3(1), dim3(SCAN_BLOCK), 0, st, in, out, n, (const long long *)nullptr);
        LF_HIP(h, hipGetLastError());
        return LF_OK;
    }
    TmpScope tmp_scope(h);
    long long *sums = nullptr, *soff = nullptr;
    LF_TRY(lf_tmp_alloc(h, (void **)&sums, sizeof(long long) * nb));
    LF_TRY(lf_tmp_alloc(h, (void **)&soff, sizeof(long long) * nb));
    hipLaunchKernelGGL(k_scan_reduce<T>, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, st, in, n, sums);
    LF_TRY(scan_impl<long long>(h, sums, soff, nb));
    hipLaunchKernelGGL(k_scan_down<T>, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, st, in, out, n,
                       (const long long *)soff);
    LF_HIP(h, hipGetLastError());
    return LF_OK;
}

int lf_exclusive_scan_i64(lf_handle *h, const long long *in, long long *out, long long n)
{
    return scan_impl<long long>(h, in, out, n);
}

int lf_exclusive_scan_i32_to_i64(lf_handle *h, const int *in, long long *out, long long n)
{
    return scan_impl<int>(h, in, out, n);
}

// ------------------------------------------------------------------------------------
// device-wide LSD radix sort (stable), 8-bit digits
// ------------------------------------------------------------------------------------
// Per pass over digit [shift, shift + nbits):
//   k_radix_hist     every tile of RS_TILE keys counts its digits -> cnt[digit][tile]
//   scan             exclusive scan of cnt, digit-major: the first output position of
//                    (digit, tile) = keys of smaller digits + keys of this digit in
//                    earlier tiles
//   k_radix_scatter  every tile ranks its keys stably and writes them to those positions
// A tile is split into one contiguous range per wave.  A wave ranks 64 keys at a time:
// the lanes holding the same digit are found with nbits ballots, a key's rank is the
// number of those lanes below it plus the wave's running count of the digit (LDS), so
// ranks follow the input order.  The keys are then placed in digit order in LDS and
// written out in runs of equal digit (coalesced).
#define RS_BLOCK 256
#define RS_WAVES (RS_BLOCK / PW)
#define RS_ITEMS 16
#define RS_WTILE (PW * RS_ITEMS)          // keys per wave
#define RS_TILE (RS_BLOCK * RS_ITEMS)     // keys per tile
#define RS_BINS 256

template <typename K>
__device__ __forceinline__ unsigned rs_digit(K k, int shift, unsigned mask)
{
    return (unsigned)(k >> shift) & mask;
}

// lanes of the wave (among those in `valid`) whose digit equals this lane's
__device__ __forceinline__ unsigned long long rs_match(unsigned d, int nbits, unsigned long long valid)
{
    unsigned long long m = valid;
    for (int b = 0; b < nbits; b++) {
        const bool bit = (d >> b) & 1u;
        const unsigned long long bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

template <typename K>
__global__ void __launch_bounds__(RS_BLOCK) k_radix_hist(const K *keys, long long n, int shift, int nbits,
                                                         int *cnt, long long ntiles)
{
    __shared__ int hist[RS_WAVES][RS_BINS];
    const int lane = threadIdx.x & (PW - 1), wv = threadIdx.x / PW;
    for (int t = threadIdx.x; t < RS_WAVES * RS_BINS; t += RS_BLOCK) (&hist[0][0])[t] = 0;
    __syncthreads();
    const unsigned mask = (1u << nbits) - 1u;
    const long long base = (long long)blockIdx.x * RS_TILE + (long long)wv * RS_WTILE;
    K k[RS_ITEMS];
#pragma unroll
    for (int i = 0; i < RS_ITEMS; i++) {
        const long long p = base + i * PW + lane;
        k[i] = p < n ? keys[p] : (K)0;
    }
#pragma unroll
    for (int i = 0; i < RS_ITEMS; i++) {
        const long long p = base + i * PW + lane;
        const unsigned long long valid = __ballot(p < n);
        if (!valid) break;                    // uniform over the wave
        const unsigned d = rs_digit(k[i], shift, mask);
        const unsigned long long m = rs_match(d, nbits, valid);
        if (p < n && __popcll(m & ((1ull << lane) - 1)) == 0) hist[wv][d] += __popcll(m);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < RS_BINS; d += RS_BLOCK) {
        int c = 0;
        for (int w = 0; w < RS_WAVES; w++) c += hist[w][d];
        if (d <= (int)mask) cnt[(long long)d * ntiles + blockIdx.x] = c;
    }
}

template <typename K, bool PAIRS>
__global__ void __launch_bounds__(RS_BLOCK) k_radix_scatter(const K *kin, K *kout, const int *vin, int *vout,
                                                            long long n, int shift, int nbits,
                                                            const long long *goff, long long ntiles)
{
    __shared__ K skey[RS_TILE];
    __shared__ int sval[PAIRS ? RS_TILE : 1];
    __shared__ int wrun[RS_WAVES][RS_BINS];   // per wave: running count, then its offset
    __shared__ int toff[RS_BINS];             // first tile position of each digit
    __shared__ long long gbase[RS_BINS];      // first output position of each digit
    __shared__ long long s_w[RS_BLOCK / PW];
    const int lane = threadIdx.x & (PW - 1), wv = threadIdx.x / PW;
    const unsigned mask = (1u << nbits) - 1u;
    const int nbins = (int)mask + 1;
    for (int t = threadIdx.x; t < RS_WAVES * RS_BINS; t += RS_BLOCK) (&wrun[0][0])[t] = 0;
    for (int d = threadIdx.x; d < RS_BINS; d += RS_BLOCK)
        gbase[d] = d < nbins ? goff[(long long)d * ntiles + blockIdx.x] : 0;
    const long long tbase = (long long)blockIdx.x * RS_TILE;
    const long long base = tbase + (long long)wv * RS_WTILE;
    K k[RS_ITEMS];
    int v[RS_ITEMS];
    int r[RS_ITEMS];
#pragma unroll
    for (int i = 0; i < RS_ITEMS; i++) {
        const long long p = base + i * PW + lane;
        k[i] = p < n ? kin[p] : (K)0;
        v[i] = (PAIRS && p < n) ? vin[p] : 0;
    }
    __syncthreads();
    // ranks within the wave's range, in input order
#pragma unroll
    for (int i = 0; i < RS_ITEMS; i++) {
        const long long p = base + i * PW + lane;
        const unsigned long long valid = __ballot(p < n);
        r[i] = 0;
        if (!valid) continue;                 // uniform over the wave
        const unsigned d = rs_digit(k[i], shift, mask);
        const unsigned long long m = rs_match(d, nbits, valid);
        const int below = __popcll(m & ((1ull << lane) - 1));
        if (p < n) {
            const int prev = wrun[wv][d];     // read by every lane before the leader writes
            r[i] = prev + below;
            if (below == 0) wrun[wv][d] = prev + __popcll(m);
        }
    }
    __syncthreads();
    // per digit: the waves' offsets and the tile's count, then the tile's digit offsets
    int dcount = 0;
    const int d0 = threadIdx.x;               // RS_BLOCK == RS_BINS: one digit per thread
    {
        int run = 0;
        for (int w = 0; w < RS_WAVES; w++) {
            const int c = wrun[w][d0];
            wrun[w][d0] = run;
            run += c;
        }
        dcount = run;
    }
    long long ttot;
    const long long tpos = block_excl_scan((long long)dcount, s_w, &ttot);
    toff[d0] = (int)tpos;
    __syncthreads();
    // keys in digit order in LDS
#pragma unroll
    for (int i = 0; i < RS_ITEMS; i++) {
        const long long p = base + i * PW + lane;
        if (p < n) {
            const unsigned d = rs_digit(k[i], shift, mask);
            const int pos = toff[d] + wrun[wv][d] + r[i];
            skey[pos] = k[i];
            if (PAIRS) sval[pos] = v[i];
        }
    }
    __syncthreads();
    // runs of equal digit go to consecutive output positions
    const long long left = n - tbase;
    const int cnt_tile = left < RS_TILE ? (int)left : RS_TILE;
#pragma unroll
    for (int i = 0; i < RS_ITEMS; i++) {
        const int pos = i * RS_BLOCK + threadIdx.x;
        if (pos < cnt_tile) {
            const K key = skey[pos];
            const unsigned d = rs_digit(key, shift, mask);
            const long long o = gbase[d] + (pos - toff[d]);
            kout[o] = key;
            if (PAIRS) vout[o] = sval[pos];
        }
    }
}

// Sorts keys[0, n) by bits [0, end_bit) (stable; values move with their keys).  The
// passes alternate between the two buffers; *rk / *rv receive the one holding the result.
template <typename K, bool PAIRS>
static int radix_sort(lf_handle *h, K *keys, K *keys_alt, int *vals, int *vals_alt, long long n, int end_bit,
                      K **rk, int **rv)
{
    *rk = keys;
    if (rv) *rv = vals;
    if (n <= 1 || end_bit <= 0) return LF_OK;
    if (n >= (1ll << 31)) return lf_set_error(h, LF_EOVERFLOW, "radix sort of %lld keys exceeds 2^31 - 1", n);
    if (end_bit > (int)(8 * sizeof(K))) end_bit = (int)(8 * sizeof(K));
    TmpScope tmp_scope(h);
    hipStream_t st = h->stream;
    const long long ntiles = (n + RS_TILE - 1) / RS_TILE;
    int *cnt = nullptr;
    long long *goff = nullptr;
    LF_TRY(lf_tmp_alloc(h, (void **)&cnt, sizeof(int) * RS_BINS * ntiles));
    LF_TRY(lf_tmp_alloc(h, (void **)&goff, sizeof(long long) * RS_BINS * ntiles));
    K *ki = keys, *ko = keys_alt;
    int *vi = vals, *vo = vals_alt;
    for (int shift = 0; shift < end_bit; shift += 8) {
        const int nbits = end_bit - shift < 8 ? end_bit - shift : 8;
        hipLaunchKernelGGL(k_radix_hist<K>, dim3((unsigned)ntiles), dim3(RS_BLOCK), 0, st, (const K *)ki, n, shift,
                           nbits, cnt, ntiles);
        LF_TRY(scan_impl<int>(h, cnt, goff, (long long)(1 << nbits) * ntiles));
        hipLaunchKernelGGL((k_radix_scatter<K, PAIRS>), dim3((unsigned)ntiles), dim3(RS_BLOCK), 0, st,
                           (const K *)ki, ko, (const int *)vi, vo, n, shift, nbits, (const long long *)goff, ntiles);
        LF_HIP(h, hipGetLastError());
        K *kt = ki;
        ki = ko;
        ko = kt;
        if (PAIRS) {
            int *vt = vi;
            vi = vo;
            vo = vt;
        }
    }
    *rk = ki;
    if (rv) *rv = vi;
    return LF_OK;
}

int lf_sort_u64(lf_handle *h, unsigned long long *keys, unsigned long long *keys_alt, long long n,
                int end_bit, unsigned long long **result)
{
    return radix_sort<unsigned long long, false>(h, keys, keys_alt, nullptr, nullptr, n, end_bit, result, nullptr);
}

int lf_sort_pairs_u64_i32(lf_handle *h, unsigned long long *keys, unsigned long long *keys_alt,
                          int *vals, int *vals_alt, long long n, int end_bit,
                          unsigned long long **rkeys, int **rvals)
{
    return radix_sort<unsigned long long, true>(h, keys, keys_alt, vals, vals_alt, n, end_bit, rkeys, rvals);
}

int lf_sort_pairs_u32_i32(lf_handle *h, unsigned *keys, unsigned *keys_alt, int *vals,
                          int *vals_alt, long long n, unsigned **rkeys, int **rvals)
{
    return radix_sort<unsigned, true>(h, keys, keys_alt, vals, vals_alt, n, 32, rkeys, rvals);
}

// In-place forms of the sorts and scans above for the diagnostic entry points: the result
// is copied back into the caller's arrays when it ends in the alternate buffers.
int lf_sort_dev_u64(lf_handle *h, unsigned long long *keys, int *vals, long long n, int end_bit)
{
    TmpScope tmp_scope(h);
    hipStream_t st = h->stream;
    unsigned long long *kalt = nullptr, *rk = keys;
    int *valt = nullptr, *rv = vals;
    LF_TRY(lf_tmp_alloc(h, (void **)&kalt, sizeof(unsigned long long) * (n > 0 ? n : 1)));
    if (vals) {
        LF_TRY(lf_tmp_alloc(h, (void **)&valt, sizeof(int) * (n > 0 ? n : 1)));
        LF_TRY(lf_sort_pairs_u64_i32(h, keys, kalt, vals, valt, n, end_bit, &rk, &rv));
    } else {
        LF_TRY(lf_sort_u64(h, keys, kalt, n, end_bit, &rk));
    }
    if (rk != keys) LF_HIP(h, hipMemcpyAsync(keys, rk, sizeof(unsigned long long) * n, hipMemcpyDeviceToDevice, st));
    if (vals && rv != vals) LF_HIP(h, hipMemcpyAsync(vals, rv, sizeof(int) * n, hipMemcpyDeviceToDevice, st));
    LF_HIP(h, hipStreamSynchronize(st));
    LF_HIP(h, hipGetLastError());
    return LF_OK;
}

int lf_sort_dev_u32(lf_handle *h, unsigned *keys, int *vals, long long n)
{
    TmpScope tmp_scope(h);
    hipStream_t st = h->stream;
    unsigned *kalt = nullptr, *rk = keys;
    int *valt = nullptr, *rv = vals;
    LF_TRY(lf_tmp_alloc(h, (void **)&kalt, sizeof(unsigned) * (n > 0 ? n : 1)));
    LF_TRY(lf_tmp_alloc(h, (void **)&valt, sizeof(int) * (n > 0 ? n : 1)));
    LF_TRY(lf_sort_pairs_u32_i32(h, keys, kalt, vals, valt, n, &rk, &rv));
    if (rk != keys) LF_HIP(h, hipMemcpyAsync(keys, rk, sizeof(unsigned) * n, hipMemcpyDeviceToDevice, st));
    if (rv != vals) LF_HIP(h, hipMemcpyAsync(vals, rv, sizeof(int) * n, hipMemcpyDeviceToDevice, st));
    LF_HIP(h, hipStreamSynchronize(st));
    LF_HIP(h, hipGetLastError());
    return LF_OK;
}

int lf_scan_dev(lf_handle *h, const void *in, int in_bytes, long long *out, long long n)
{
    if (in_bytes == 8) LF_TRY(lf_exclusive_scan_i64(h, (const long long *)in, out, n));
    else LF_TRY(lf_exclusive_scan_i32_to_i64(h, (const int *)in, out, n));
    LF_HIP(h, hipStreamSynchronize(h->stream));
    LF_HIP(h, hipGetLastError());
    return LF_OK;
}
