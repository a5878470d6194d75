// graph.hip -- preprocessing and node statistics on the GPU.
//
//   lf_build_graph   multi-edge removal, self-loop removal, dense labels, symmetric CSR with
//                    sorted rows (Methods, "Preprocessing")
//   lf_node_stats    triangles k_i, local clustering coefficient, global cc (mean of local
//                    CCs) and the node order: CC descending, degree descending, id
//                    ascending (Methods, "Node Order"; WCC-hat subsection for cc)
//
// Triangles: every edge is oriented from the endpoint that is smaller in (degree, id)
// order to the larger one, so each triangle {a < b < c} is found exactly once, at a with
// the oriented edges a->b, a->c and b->c.  For a node u, a wave (or a workgroup for long
// out-lists) stages N+(u) in LDS, walks the concatenation of N+(v) over v in N+(u) with
// all its lanes, and binary-searches each w in the staged N+(u).  A hit credits u, v and
// w; the credits of v and w (both in N+(u)) are accumulated in LDS counters and flushed
// to HBM once per (u, position).
#include "lf_internal.h"

#define WAVE 64

static int bits_for(long long n)
{
    int b = 1;
    while ((1ll << b) < n) b++;
    return b;
}

// ------------------------------------------------------------------------------------
// A0: graph build
// ------------------------------------------------------------------------------------
__global__ void k_collect_ids(const long long *src, const long long *dst, long long np,
                              unsigned long long *ids, int *err)
{
    long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= np) return;
    long long a = src[e], b = dst[e];
    if (a < 0 || b < 0) { atomicOr(err, 1); a = b = 0; }
    bool loop = (a == b);
    ids[2 * e] = loop ? ~0ull : (unsigned long long)a;
    ids[2 * e + 1] = loop ? ~0ull : (unsigned long long)b;
}

__global__ void k_unique_flags_u64(const unsigned long long *k, long long n, unsigned long long sentinel,
                                   int *flag)
{
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    unsigned long long v = k[i];
    flag[i] = (v != sentinel) && (i == 0 || k[i - 1] != v);
}

__global__ void k_compact_u64(const unsigned long long *k, const int *flag, const long long *pos,
                              long long n, unsigned long long *out)
{
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (flag[i]) out[pos[i]] = k[i];
}

__device__ __forceinline__ long long find_sorted_u64(const unsigned long long *a, long long n,
                                                     unsigned long long v)
{
    long long lo = 0, hi = n - 1;
    while (lo <= hi) {
        long long mid = lo + ((hi - lo) >> 1);
        unsigned long long x = a[mid];
        if (x == v) return mid;
        if (x < v) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

// canonical (min, max) keys; self-loops -> sentinel; ids checked or remapped
__global__ void k_canon_keys(const long long *src, const long long *dst, long long np, long long n,
                             const unsigned long long *uniq_ids, int B, unsigned long long *keys,
                             int *err)
{
    long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= np) return;
    long long a = src[e], b = dst[e];
    unsigned long long sentinel = (B >= 32) ? ~0ull : ((1ull << (2 * B)) - 1);
    if (a == b) { keys[e] = sentinel; return; }
    if (uniq_ids) {
        a = find_sorted_u64(uniq_ids, n, (unsigned long long)a);
        b = find_sorted_u64(uniq_ids, n, (unsigned long long)b);
    }
    if (a < 0 || b < 0 || a >= n || b >= n) { atomicOr(err, 1); keys[e] = sentinel; return; }
    if (a > b) { long long t = a; a = b; b = t; }
    keys[e] = ((unsigned long long)a << B) | (unsigned long long)b;
}

__global__ void k_degrees(const unsigned long long *uk, long long ne, int B, int *deg)
{
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= ne) return;
    unsigned long long k = uk[i];
    unsigned long long mask = (1ull << B) - 1;
    atomicAdd(&deg[(long long)(k >> B)], 1);
    atomicAdd(&deg[(long long)(k & mask)], 1);
}

__global__ void k_directed_keys(const unsigned long long *uk, long long ne, int B, unsigned long long *dk)
{
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= ne) return;
    unsigned long long k = uk[i];
    unsigned long long mask = (1ull << B) - 1;
    unsigned long long a = k >> B, b = k & mask;
    dk[2 * i] = k;
    dk[2 * i + 1] = (b << B) | a;
}

__global__ void k_col_from_keys(const unsigned long long *dk, long long m, int B, int *col)
{
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= m) return;
    col[i] = (int)(dk[i] & ((1ull << B) - 1));
}

__global__ void k_deg_to_i64(const int *deg, long long n, long long *out, int *maxdeg)
{
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = deg[i];
    atomicMax(maxdeg, deg[i]);
}

__global__ void k_set_last(long long *rowptr, long long n, long long val) { rowptr[n] = val; }

__global__ void k_iota_ids(long long *ids, long long n, const unsigned long long *uniq)
{
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    ids[i] = uniq ? (long long)uniq[i] : i;
}

static inline unsigned grid_for(long long n, int block) { return (unsigned)((n + block - 1) / block); }

int lf_build_graph(lf_handle *h, long long n, long long np, const long long *src,
                   const long long *dst, unsigned flags)
{
    TmpScope tmp_scope(h);
    hipStream_t st = h->stream;
    const int BS = 256;
    long long *dsrc = nullptr, *ddst = nullptr;
    if (flags & LF_DEVICE_PTR) {
        dsrc = (long long *)src;
        ddst = (long long *)dst;
    } else if (np > 0) {
        LF_TRY(lf_tmp_alloc(h, (void **)&dsrc, sizeof(long long) * np));
        LF_TRY(lf_tmp_alloc(h, (void **)&ddst, sizeof(long long) * np));
        LF_HIP(h, hipMemcpyAsync(dsrc, src, sizeof(long long) * np, hipMemcpyHostToDevice, st));
        LF_HIP(h, hipMemcpyAsync(ddst, dst, sizeof(long long) * np, hipMemcpyHostToDevice, st));
    }
    int *derr = nullptr;
    LF_TRY(lf_tmp_alloc(h, (void **)&derr, sizeof(int) * 4));
    LF_HIP(h, hipMemsetAsync(derr, 0, sizeof(int) * 4, st));

    // scratch sized for the largest use: 2 * np 64-bit keys (ids) and 2 * ne directed keys
    long long kcap = 2 * (np > 0 ? np : 1);
    unsigned long long *ka = nullptr, *kb = nullptr;
    int *flag = nullptr;
    long long *pos = nullptr;
    LF_TRY(lf_tmp_alloc(h, (void **)&ka, sizeof(unsigned long long) * kcap));
    LF_TRY(lf_tmp_alloc(h, (void **)&kb, sizeof(unsigned long long) * kcap));
    LF_TRY(lf_tmp_alloc(h, (void **)&flag, sizeof(int) * kcap));
    LF_TRY(lf_tmp_alloc(h, (void **)&pos, sizeof(long long) * (kcap + 1)));

    unsigned long long *uniq_ids = nullptr;
    if (flags & LF_RELABEL) {
        long long m = 2 * np;
        if (np > 0) hipLaunchKernelGGL(k_collect_ids, dim3(grid_for(np, BS)), dim3(BS), 0, st, dsrc, ddst, np, ka, derr);
        unsigned long long *sorted;
        LF_TRY(lf_sort_u64(h, ka, kb, m, 64, &sorted));
        if (m > 0) hipLaunchKernelGGL(k_unique_flags_u64, dim3(grid_for(m, BS)), dim3(BS), 0, st, sorted, m, ~0ull, flag);
        LF_TRY(lf_exclusive_scan_i32_to_i64(h, flag, pos, m + 0));
        long long last_pos = 0;
        int last_flag = 0;
        if (m > 0) {
            LF_HIP(h, hipMemcpyAsync(&last_pos, pos + m - 1, sizeof(long long), hipMemcpyDeviceToHost, st));
            LF_HIP(h, hipMemcpyAsync(&last_flag, flag + m - 1, sizeof(int), hipMemcpyDeviceToHost, st));
        }
        LF_HIP(h, hipStreamSynchronize(st));
        n = (m > 0) ? last_pos + last_flag : 0;
        LF_TRY(lf_tmp_alloc(h, (void **)&uniq_ids, sizeof(unsigned long long) * (n > 0 ? n : 1)));
        if (m > 0) hipLaunchKernelGGL(k_compact_u64, dim3(grid_for(m, BS)), dim3(BS), 0, st, sorted, flag, pos, m, uniq_ids);
    }
    if (n >= (1ll << 31) - 1) {
        return lf_set_error(h, LF_EOVERFLOW, "n = %lld nodes exceeds the supported 2^31 - 2", n);
    }
    int B = bits_for(n > 1 ? n : 2);
    unsigned long long sentinel = (B >= 32) ? ~0ull : ((1ull << (2 * B)) - 1);
    if (np > 0)
        hipLaunchKernelGGL(k_canon_keys, dim3(grid_for(np, BS)), dim3(BS), 0, st, dsrc, ddst, np, n,
                           uniq_ids, B, ka, derr);
    unsigned long long *sorted;
    LF_TRY(lf_sort_u64(h, ka, kb, np, 2 * B, &sorted));
    if (np > 0) hipLaunchKernelGGL(k_unique_flags_u64, dim3(grid_for(np, BS)), dim3(BS), 0, st, sorted, np, sentinel, flag);
    LF_TRY(lf_exclusive_scan_i32_to_i64(h, flag, pos, np));
    long long last_pos = 0;
    int last_flag = 0, herr[4] = {0, 0, 0, 0};
    if (np > 0) {
        LF_HIP(h, hipMemcpyAsync(&last_pos, pos + np - 1, sizeof(long long), hipMemcpyDeviceToHost, st));
        LF_HIP(h, hipMemcpyAsync(&last_flag, flag + np - 1, sizeof(int), hipMemcpyDeviceToHost, st));
    }
    LF_HIP(h, hipMemcpyAsync(herr, derr, sizeof(int) * 4, hipMemcpyDeviceToHost, st));
    LF_HIP(h, hipStreamSynchronize(st));
    if (herr[0]) return lf_set_error(h, LF_EINVAL, "edge list has an id outside [0, n) (n = %lld)", n);
    long long ne = (np > 0) ? last_pos + last_flag : 0;
    if (2 * ne >= (1ll << 31)) return lf_set_error(h, LF_EOVERFLOW, "2|E| = %lld exceeds 2^31 - 1", 2 * ne);
    // unique canonical keys -> kb (or ka) compacted
    unsigned long long *uk = (sorted == ka) ? kb : ka;
    if (np > 0) hipLaunchKernelGGL(k_compact_u64, dim3(grid_for(np, BS)), dim3(BS), 0, st, sorted, flag, pos, np, uk);

    LF_TRY(lf_dev_alloc(h, (void **)&h->deg, sizeof(int) * (n > 0 ? n : 1)));
    LF_TRY(lf_dev_alloc(h, (void **)&h->rowptr, sizeof(long long) * (n + 1)));
    LF_TRY(lf_dev_alloc(h, (void **)&h->col, sizeof(int) * (2 * ne > 0 ? 2 * ne : 1)));
    LF_TRY(lf_dev_alloc(h, (void **)&h->orig_id, sizeof(long long) * (n > 0 ? n : 1)));
    LF_HIP(h, hipMemsetAsync(h->deg, 0, sizeof(int) * (n > 0 ? n : 1), st));
    if (ne > 0) hipLaunchKernelGGL(k_degrees, dim3(grid_for(ne, BS)), dim3(BS), 0, st, uk, ne, B, h->deg);
    // directed keys: the other buffer holds up to 2 np >= 2 ne entries
    unsigned long long *dk = (uk == ka) ? kb : ka;
    unsigned long long *dk_alt = uk;   // unique keys are no longer needed after expansion
    if (ne > 0) hipLaunchKernelGGL(k_directed_keys, dim3(grid_for(ne, BS)), dim3(BS), 0, st, uk, ne, B, dk);
    // uk is about to be overwritten as the sort's alternate buffer: expansion above is
    // stream-ordered before the sort, so this is safe
    LF_TRY(lf_sort_u64(h, dk, dk_alt, 2 * ne, 2 * B, &sorted));
    if (ne > 0) hipLaunchKernelGGL(k_col_from_keys, dim3(grid_for(2 * ne, BS)), dim3(BS), 0, st, sorted, 2 * ne, B, h->col);
    long long *deg64 = pos;     // reuse: n <= kcap? not guaranteed, allocate if needed
    bool own_deg64 = false;
    if (n + 1 > kcap + 1) {
        LF_TRY(lf_tmp_alloc(h, (void **)&deg64, sizeof(long long) * (n + 1)));
        own_deg64 = true;
    }
    LF_HIP(h, hipMemsetAsync(derr, 0, sizeof(int) * 4, st));
    if (n > 0) hipLaunchKernelGGL(k_deg_to_i64, dim3(grid_for(n, BS)), dim3(BS), 0, st, h->deg, n, deg64, derr + 1);
    LF_TRY(lf_exclusive_scan_i64(h, deg64, h->rowptr, n));
    hipLaunchKernelGGL(k_set_last, dim3(1), dim3(1), 0, st, h->rowptr, n, 2 * ne);
    if (n > 0) hipLaunchKernelGGL(k_iota_ids, dim3(grid_for(n, BS)), dim3(BS), 0, st, h->orig_id, n, uniq_ids);
    int maxdeg = 0;
    LF_HIP(h, hipMemcpyAsync(&maxdeg, derr + 1, sizeof(int), hipMemcpyDeviceToHost, st));
    LF_HIP(h, hipStreamSynchronize(st));
    LF_HIP(h, hipGetLastError());
    h->n = n;
    h->ne = ne;
    h->max_deg = maxdeg;
    return LF_OK;
}

// ------------------------------------------------------------------------------------
// A1: triangles
// ------------------------------------------------------------------------------------
__device__ __forceinline__ bool before(int du, int u, int dv, int v)
{
    return du < dv || (du == dv && u < v);
}

// out-degree in the (degree, id) orientation; one wave per node
__global__ void __launch_bounds__(256) k_out_degree(const long long *rowptr, const int *col,
                                                    const int *deg, long long n, int *od)
{
    long long u = (blockIdx.x * (long long)blockDim.x + threadIdx.x) / WAVE;
    int lane = threadIdx.x & (WAVE - 1);
    if (u >= n) return;
    int du = deg[u];
    int c = 0;
    for (long long e = rowptr[u] + lane; e < rowptr[u + 1]; e += WAVE) {
        int v = col[e];
        c += before(du, (int)u, deg[v], v);
    }
    c = wave_sum_int(c);
    if (lane == 0) od[u] = c;
}

// compacted out-lists, kept in ascending id order
__global__ void __launch_bounds__(256) k_out_fill(const long long *rowptr, const int *col,
                                                  const int *deg, long long n, const long long *oro,
                                                  int *orc)
{
    long long u = (blockIdx.x * (long long)blockDim.x + threadIdx.x) / WAVE;
    int lane = threadIdx.x & (WAVE - 1);
    if (u >= n) return;
    int du = deg[u];
    long long w = oro[u];
    for (long long base = rowptr[u]; base < rowptr[u + 1]; base += WAVE) {
        long long e = base + lane;
        bool keep = false;
        int v = 0;
        if (e < rowptr[u + 1]) {
            v = col[e];
            keep = before(du, (int)u, deg[v], v);
        }
        unsigned long long mask = __ballot(keep);
        int rank = __popcll(mask & ((1ull << lane) - 1));
        if (keep) orc[w + rank] = v;
        w += __popcll(mask);
    }
}

__device__ __forceinline__ int lds_find(const int *a, int m, int v)
{
    int lo = 0, hi = m - 1;
    while (lo <= hi) {
        int mid = (lo + hi) >> 1;
        int x = a[mid];
        if (x == v) return mid;
        if (x < v) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

// index j with P[j] <= f < P[j+1] (P exclusive prefix, P[0] = 0)
__device__ __forceinline__ int seg_of(const int *P, int m, int f)
{
    int lo = 0, hi = m - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (P[mid] <= f) lo = mid; else hi = mid - 1;
    }
    return lo;
}

#define TRI_WAVE_CAP 256
#define TRI_WAVES 4

// A triangle {u, v, w} found at u (v = N+(u)[j], w = N+(u)[p]) in the exact-WCC pass:
// the three oriented edges are marked as closing a triangle, and every community that u,
// v and w share gains one triangle at each of them (a walk of their sorted id lists).
__device__ __forceinline__ void wcc_hit(const WccTri &wt, int u, int v, int w, long long e_uv, long long e_uw,
                                        long long e_vw)
{
    wt.eflag[e_uv] = 1;
    wt.eflag[e_uw] = 1;
    wt.eflag[e_vw] = 1;
    long long a = wt.moff[u], b = wt.moff[v], c = wt.moff[w];
    const long long ae = wt.moff[u + 1], be = wt.moff[v + 1], ce = wt.moff[w + 1];
    while (a < ae && b < be && c < ce) {
        const int x = wt.mid[a], y = wt.mid[b], z = wt.mid[c];
        if (x == y && y == z) {
            atomicAdd(&wt.tcm[a], 1);
            atomicAdd(&wt.tcm[b], 1);
            atomicAdd(&wt.tcm[c], 1);
            a++; b++; c++;
        } else {
            const int m = x > y ? (x > z ? x : z) : (y > z ? y : z);
            a += x < m;
            b += y < m;
            c += z < m;
        }
    }
}

// one wave per node with |N+(u)| <= TRI_WAVE_CAP; longer out-lists are deferred.  Every
// wave of the block reaches both barriers (no early exit), inactive waves just idle.
// WCC = false: triangle counts per node into tri; true: wcc_hit per triangle instead.
template <bool WCC>
__global__ void __launch_bounds__(256) k_tri_wave(const long long *oro, const int *orc, long long n,
                                                  unsigned long long *tri, int *defer, int *ndefer, WccTri wt)
{
    __shared__ int s_nbr[TRI_WAVES][TRI_WAVE_CAP];
    __shared__ int s_pre[TRI_WAVES][TRI_WAVE_CAP + 1];
    __shared__ int s_cnt[TRI_WAVES][TRI_WAVE_CAP];
    int wv = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
    long long u = blockIdx.x * (long long)TRI_WAVES + wv;
    long long b = 0;
    int m = 0;
    if (u < n) {
        b = oro[u];
        m = (int)(oro[u + 1] - b);
    }
    if (m > TRI_WAVE_CAP) {
        if (lane == 0) defer[atomicAdd(ndefer, 1)] = (int)u;
        m = 0;
    }
    if (m < 2) m = 0;                      // a triangle needs two out-neighbours of u
    int *nbr = s_nbr[wv], *pre = s_pre[wv], *cnt = s_cnt[wv];
    // stage N+(u), lengths of N+(v), exclusive prefix
    int carry = 0;
    for (int base = 0; base < m; base += WAVE) {
        int j = base + lane;
        int len = 0;
        if (j < m) {
            int v = orc[b + j];
            nbr[j] = v;
            cnt[j] = 0;
            len = (int)(oro[v + 1] - oro[v]);
        }
        int x = len;
        for (int d = 1; d < WAVE; d <<= 1) {
            int y = __shfl_up(x, d, WAVE);
            if (lane >= d) x += y;
        }
        if (j < m) pre[j] = carry + x - len;
        carry += __shfl(x, WAVE - 1, WAVE);
    }
    if (lane == 0) pre[m] = carry;
    __syncthreads();
    int W = carry;
    int total = 0;
    for (int f = lane; f < W; f += WAVE) {
        int j = seg_of(pre, m, f);
        int v = nbr[j];
        long long evw = oro[v] + (f - pre[j]);
        int w = orc[evw];
        int p = lds_find(nbr, m, w);
        if (p >= 0) {
            if constexpr (WCC) {
                wcc_hit(wt, (int)u, v, w, b + j, b + p, evw);
            } else {
                atomicAdd(&cnt[p], 1);
                atomicAdd(&cnt[j], 1);
                total++;
            }
        }
    }
    __syncthreads();
    if constexpr (!WCC) {
        for (int j = lane; j < m; j += WAVE)
            if (cnt[j]) atomicAdd(&tri[nbr[j]], (unsigned long long)cnt[j]);
        total = wave_sum_int(total);
        if (lane == 0 && total) atomicAdd(&tri[u], (unsigned long long)total);
    }
}

// one workgroup per deferred node; out-list, prefix and counters in LDS when they fit,
// otherwise in this workgroup's slice of global scratch
template <bool WCC>
__global__ void __launch_bounds__(1024) k_tri_group(const long long *oro, const int *orc,
                                                    const int *list, int nlist,
                                                    unsigned long long *tri, int lds_cap,
                                                    int *gscratch, long long gslice, WccTri wt)
{
    extern __shared__ int s_dyn[];
    __shared__ int s_total;
    __shared__ int s_carry;
    for (int it = blockIdx.x; it < nlist; it += gridDim.x) {
        int u = list[it];
        long long b = oro[u];
        int m = (int)(oro[u + 1] - b);
        int *nbr, *pre, *cnt;
        bool lds = m <= lds_cap;
        if (lds) {
            nbr = s_dyn;
            pre = s_dyn + lds_cap;
            cnt = s_dyn + 2 * lds_cap + 1;
        } else {
            int *g = gscratch + (long long)blockIdx.x * gslice;
            nbr = g;
            pre = g + m;
            cnt = g + 2 * (long long)m + 1;
        }
        if (threadIdx.x == 0) { s_total = 0; s_carry = 0; }
        __syncthreads();
        for (int j = threadIdx.x; j < m; j += blockDim.x) {
            nbr[j] = orc[b + j];
            cnt[j] = 0;
        }
        __syncthreads();
        // exclusive prefix of |N+(v)| (serial over chunks of blockDim, scan per wave)
        int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
        for (int base = 0; base < m; base += blockDim.x) {
            int j = base + threadIdx.x;
            int len = 0;
            if (j < m) { int v = nbr[j]; len = (int)(oro[v + 1] - oro[v]); }
            int x = len;
            for (int d = 1; d < WAVE; d <<= 1) {
                int y = __shfl_up(x, d, WAVE);
                if (lane >= d) x += y;
            }
            __shared__ int s_wsum[16];
            if (lane == WAVE - 1) s_wsum[wv] = x;
            __syncthreads();
            int off = s_carry;
            for (int k = 0; k < wv; k++) off += s_wsum[k];
            if (j < m) pre[j] = off + x - len;
            __syncthreads();
            if (threadIdx.x == 0) {
                int t = 0;
                for (int k = 0; k < nw; k++) t += s_wsum[k];
                s_carry += t;
            }
            __syncthreads();
        }
        int W = s_carry;
        if (threadIdx.x == 0) pre[m] = W;
        __syncthreads();
        int total = 0;
        for (int f = threadIdx.x; f < W; f += blockDim.x) {
            int j = seg_of(pre, m, f);
            int v = nbr[j];
            long long evw = oro[v] + (f - pre[j]);
            int w = orc[evw];
            int p = lds_find(nbr, m, w);
            if (p >= 0) {
                if constexpr (WCC) {
                    wcc_hit(wt, u, v, w, b + j, b + p, evw);
                } else {
                    atomicAdd(&cnt[p], 1);
                    atomicAdd(&cnt[j], 1);
                    total++;
                }
            }
        }
        if constexpr (!WCC) {
            total = wave_sum_int(total);
            if (lane == 0 && total) atomicAdd(&s_total, total);
        }
        __syncthreads();
        if constexpr (!WCC) {
            for (int j = threadIdx.x; j < m; j += blockDim.x)
                if (cnt[j]) atomicAdd(&tri[nbr[j]], (unsigned long long)cnt[j]);
            if (threadIdx.x == 0 && s_total) atomicAdd(&tri[u], (unsigned long long)s_total);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------
// A2: local CC, global cc, order
// ------------------------------------------------------------------------------------
#define RED_BLOCK 256

// local CC, the exact sum of the CCs (per-block partials) and the triangle sum
__global__ void __launch_bounds__(RED_BLOCK) k_local_cc(const unsigned long long *tri, const int *deg,
                                                        long long n, double *ccl, X192 *partial,
                                                        unsigned long long *tsum, int *err)
{
    __shared__ X192 s_w[RED_BLOCK / WAVE];
    X192 acc = x192_zero();
    unsigned long long t = 0;
    int bad = 0;
    for (long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x; x < n;
         x += (long long)gridDim.x * blockDim.x) {
        long long d = deg[x];
        long long k = (long long)tri[x];
        double c = 0.0;
        if (d > 1) c = (double)k / (double)(d * (d - 1) / 2);
        ccl[x] = c;
        X192 v = x192_from_double(c, bad);
        x192_add(acc, v);
        t += (unsigned long long)k;
    }
    acc = wave_sum_x192(acc);
    t = (unsigned long long)wave_sum_i64((long long)t);
    int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    if (lane == 0) {
        s_w[wv] = acc;
        atomicAdd(tsum, t);
    }
    if (bad) atomicOr(err, LF_DEVERR_INEXACT);
    __syncthreads();
    if (threadIdx.x == 0) {
        X192 s = s_w[0];
        for (int k = 1; k < RED_BLOCK / WAVE; k++) x192_add(s, s_w[k]);
        partial[blockIdx.x] = s;
    }
}

// exact sum of doubles into per-block partials (diagnostic entry point)
__global__ void __launch_bounds__(RED_BLOCK) k_exact_partials(const double *v, long long n, X192 *partial,
                                                              int *err)
{
    __shared__ X192 s_w[RED_BLOCK / WAVE];
    X192 acc = x192_zero();
    int bad = 0;
    for (long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x; x < n;
         x += (long long)gridDim.x * blockDim.x) {
        double a = v[x];
        if (!(fabs(a) <= 1073741824.0)) bad = 1;
        X192 t = x192_from_double(a, bad);
        x192_add(acc, t);
    }
    acc = wave_sum_x192(acc);
    if (bad) atomicOr(err, LF_DEVERR_INEXACT);
    int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    if (lane == 0) s_w[wv] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        X192 s = s_w[0];
        for (int k = 1; k < RED_BLOCK / WAVE; k++) x192_add(s, s_w[k]);
        partial[blockIdx.x] = s;
    }
}

// one wave folds the partials and rounds once; result = R(sum) / divisor (divisor > 0)
__global__ void k_fold_partials(const X192 *partial, int np, double divisor, double *out)
{
    int lane = threadIdx.x;
    X192 acc = x192_zero();
    for (int k = lane; k < np; k += WAVE) x192_add(acc, partial[k]);
    acc = wave_sum_x192(acc);
    if (lane == 0) out[0] = x192_round(acc) / divisor;
}

__global__ void k_order_keys_deg(const int *deg, long long n, int maxdeg, unsigned *key, int *val)
{
    long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (x >= n) return;
    key[x] = (unsigned)(maxdeg - deg[x]);   // degree descending
    val[x] = (int)x;                          // ids ascending (stable sorts keep it)
}

__global__ void k_order_keys_cc(const double *ccl, const int *ids, long long n, unsigned long long *key)
{
    long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (r >= n) return;
    // CC in [0, 1]: its bit pattern orders like the value; subtract to sort descending
    unsigned long long b = (unsigned long long)__double_as_longlong(ccl[ids[r]]);
    key[r] = 0x3FF0000000000000ull - b;
}

__global__ void k_rank(const int *order, long long n, int *rank)
{
    long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (r >= n) return;
    rank[order[r]] = (int)r;
}

// the order position of every adjacency entry's node, so that a pass over a node's
// neighbours reads their positions with its column indices instead of one hop later
__global__ void k_col_rank(const int *col, long long m, const int *rank, int *out)
{
    long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= m) return;
    out[e] = rank[col[e]];
}

__global__ void k_clear_int(int *p) { *p = 0; }

// The exact sum on caller-placed scratch: part (LF_EXACT_PARTIALS X192 entries), err (one
// int) and dout (one double) in device memory; nothing is allocated here.
int lf_exact_sum_run(lf_handle *h, const double *v, long long n, double *out, X192 *part, int *err, double *dout)
{
    hipStream_t st = h->stream;
    int nb = (int)((n + RED_BLOCK - 1) / RED_BLOCK);
    if (nb > LF_EXACT_PARTIALS) nb = LF_EXACT_PARTIALS;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_clear_int, dim3(1), dim3(1), 0, st, err);
    hipLaunchKernelGGL(k_exact_partials, dim3(nb), dim3(RED_BLOCK), 0, st, v, n, part, err);
    hipLaunchKernelGGL(k_fold_partials, dim3(1), dim3(WAVE), 0, st, part, nb, 1.0, dout);
    int herr = 0;
    LF_HIP(h, hipMemcpyAsync(out, dout, sizeof(double), hipMemcpyDeviceToHost, st));
    LF_HIP(h, hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
    LF_HIP(h, hipStreamSynchronize(st));
    LF_HIP(h, hipGetLastError());
    if (herr) return lf_set_error(h, LF_EOVERFLOW, "value outside the exact accumulator's range");
    return LF_OK;
}

int lf_exact_sum_dev(lf_handle *h, const double *v, long long n, double *out)
{
    TmpScope tmp_scope(h);
    X192 *part = nullptr;
    int *err = nullptr;
    double *dout = nullptr;
    LF_TRY(lf_tmp_alloc(h, (void **)&part, sizeof(X192) * LF_EXACT_PARTIALS));
    LF_TRY(lf_tmp_alloc(h, (void **)&err, sizeof(int)));
    LF_TRY(lf_tmp_alloc(h, (void **)&dout, sizeof(double)));
    return lf_exact_sum_run(h, v, n, out, part, err, dout);
}

// Every triangle once, at its lowest endpoint in (degree, id) order: with wt == nullptr
// the per-node counts go to h->tri, otherwise wcc_hit is applied to each triangle.
// Oriented lists (out-offsets oro[n + 1], out-neighbours orc, ascending ids) are built
// into temporaries of the caller's scratch scope and returned if asked for.
int lf_triangle_pass(lf_handle *h, const WccTri *wt, int *launches, long long **oro_out, int **orc_out)
{
    hipStream_t st = h->stream;
    const long long n = h->n;
    const int BS = 256;
    int maxdev = 0;
    LF_HIP(h, hipDeviceGetAttribute(&maxdev, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device));
    int *od = nullptr;
    long long *oro = nullptr;
    int *orc = nullptr;
    int *defer = nullptr;
    int *cnt = nullptr;
    LF_TRY(lf_tmp_alloc(h, (void **)&od, sizeof(int) * (n > 0 ? n : 1)));
    LF_TRY(lf_tmp_alloc(h, (void **)&oro, sizeof(long long) * (n + 1)));
    LF_TRY(lf_tmp_alloc(h, (void **)&orc, sizeof(int) * (h->ne > 0 ? h->ne : 1)));
    LF_TRY(lf_tmp_alloc(h, (void **)&defer, sizeof(int) * (n > 0 ? n : 1)));
    LF_TRY(lf_tmp_alloc(h, (void **)&cnt, sizeof(int) * 4));
    LF_HIP(h, hipMemsetAsync(cnt, 0, sizeof(int) * 4, st));
    WccTri none;
    memset(&none, 0, sizeof none);
    const WccTri w = wt ? *wt : none;
    unsigned gw = grid_for(n * WAVE, BS);
    long long *od64 = nullptr;
    LF_TRY(lf_tmp_alloc(h, (void **)&od64, sizeof(long long) * (n + 1)));
    if (n > 0) {
        hipLaunchKernelGGL(k_out_degree, dim3(gw), dim3(BS), 0, st, h->rowptr, h->col, h->deg, n, od);
        hipLaunchKernelGGL(k_deg_to_i64, dim3(grid_for(n, BS)), dim3(BS), 0, st, od, n, od64, cnt + 2);
    }
    LF_TRY(lf_exclusive_scan_i64(h, od64, oro, n));
    hipLaunchKernelGGL(k_set_last, dim3(1), dim3(1), 0, st, oro, n, h->ne);
    if (n > 0) {
        hipLaunchKernelGGL(k_out_fill, dim3(gw), dim3(BS), 0, st, h->rowptr, h->col, h->deg, n, oro, orc);
        if (wt)
            hipLaunchKernelGGL(k_tri_wave<true>, dim3(grid_for(n, TRI_WAVES)), dim3(TRI_WAVES * WAVE), 0, st,
                               oro, orc, n, h->tri, defer, cnt, w);
        else
            hipLaunchKernelGGL(k_tri_wave<false>, dim3(grid_for(n, TRI_WAVES)), dim3(TRI_WAVES * WAVE), 0, st,
                               oro, orc, n, h->tri, defer, cnt, w);
    }
    int hc[4] = {0, 0, 0, 0};
    LF_HIP(h, hipMemcpyAsync(hc, cnt, sizeof(int) * 4, hipMemcpyDeviceToHost, st));
    LF_HIP(h, hipStreamSynchronize(st));
    int ndefer = hc[0], maxod = hc[2];
    *launches = 5;
    if (ndefer > 0) {
        // LDS: nbr, pre (+1), cnt
        int lds_cap = (maxdev - 1024) / (3 * (int)sizeof(int)) - 1;
        if (lds_cap > 65536) lds_cap = 65536;
        if (h->tri_lds_cap > 0 && h->tri_lds_cap < lds_cap) lds_cap = h->tri_lds_cap;
        int blocks = ndefer < 1024 ? ndefer : 1024;
        int *gs = nullptr;
        long long gslice = 3ll * maxod + 2;
        if (maxod > lds_cap) LF_TRY(lf_tmp_alloc(h, (void **)&gs, sizeof(int) * gslice * blocks));
        size_t shmem = sizeof(int) * (3 * (size_t)lds_cap + 1);
        const void *fn = wt ? (const void *)k_tri_group<true> : (const void *)k_tri_group<false>;
        LF_HIP(h, hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
        if (wt)
            hipLaunchKernelGGL(k_tri_group<true>, dim3(blocks), dim3(1024), shmem, st, oro, orc, defer, ndefer,
                               h->tri, lds_cap, gs, gslice, w);
        else
            hipLaunchKernelGGL(k_tri_group<false>, dim3(blocks), dim3(1024), shmem, st, oro, orc, defer, ndefer,
                               h->tri, lds_cap, gs, gslice, w);
        LF_HIP(h, hipGetLastError());
        LF_HIP(h, hipStreamSynchronize(st));
        *launches = 6;
    }
    LF_HIP(h, hipGetLastError());
    if (oro_out) *oro_out = oro;
    if (orc_out) *orc_out = orc;
    return LF_OK;
}

int lf_node_stats(lf_handle *h)
{
    TmpScope tmp_scope(h);
    hipStream_t st = h->stream;
    long long n = h->n;
    const int BS = 256;

    LF_TRY(lf_prof_begin(h, LF_K_TRIANGLES));
    int *cnt = nullptr;
    LF_TRY(lf_tmp_alloc(h, (void **)&cnt, sizeof(int) * 4));
    LF_TRY(lf_dev_alloc(h, (void **)&h->tri, sizeof(unsigned long long) * (n > 0 ? n : 1)));
    LF_HIP(h, hipMemsetAsync(h->tri, 0, sizeof(unsigned long long) * (n > 0 ? n : 1), st));
    int launches = 0;
    LF_TRY(lf_triangle_pass(h, nullptr, &launches, nullptr, nullptr));
    int hc[4] = {0, 0, 0, 0};
    LF_TRY(lf_prof_end(h, LF_K_TRIANGLES, launches));

    // local CC, cc, T
    LF_TRY(lf_prof_begin(h, LF_K_ORDER));
    LF_TRY(lf_dev_alloc(h, (void **)&h->ccl, sizeof(double) * (n > 0 ? n : 1)));
    int nb = (int)((n + RED_BLOCK - 1) / RED_BLOCK);
    if (nb > 1024) nb = 1024;
    if (nb < 1) nb = 1;
    X192 *part = nullptr;
    unsigned long long *tsum = nullptr;
    double *dcc = nullptr;
    LF_TRY(lf_tmp_alloc(h, (void **)&part, sizeof(X192) * nb));
    LF_TRY(lf_tmp_alloc(h, (void **)&tsum, sizeof(unsigned long long)));
    LF_TRY(lf_tmp_alloc(h, (void **)&dcc, sizeof(double)));
    LF_HIP(h, hipMemsetAsync(tsum, 0, sizeof(unsigned long long), st));
    LF_HIP(h, hipMemsetAsync(cnt, 0, sizeof(int) * 4, st));
    hipLaunchKernelGGL(k_local_cc, dim3(nb), dim3(RED_BLOCK), 0, st, h->tri, h->deg, n, h->ccl, part, tsum, cnt);
    hipLaunchKernelGGL(k_fold_partials, dim3(1), dim3(WAVE), 0, st, part, nb, (double)(n > 0 ? n : 1), dcc);

    // order: stable sort by degree descending, then stable sort by CC descending
    LF_TRY(lf_dev_alloc(h, (void **)&h->order, sizeof(int) * (n > 0 ? n : 1)));
    LF_TRY(lf_dev_alloc(h, (void **)&h->rank, sizeof(int) * (n > 0 ? n : 1)));
    const long long m = 2 * h->ne;
    LF_TRY(lf_dev_alloc(h, (void **)&h->col_rank, sizeof(int) * (m > 0 ? m : 1)));
    unsigned *k1 = nullptr, *k1b = nullptr;
    int *v1 = nullptr, *v1b = nullptr;
    unsigned long long *k2 = nullptr, *k2b = nullptr;
    LF_TRY(lf_tmp_alloc(h, (void **)&k1, sizeof(unsigned) * (n > 0 ? n : 1)));
    LF_TRY(lf_tmp_alloc(h, (void **)&k1b, sizeof(unsigned) * (n > 0 ? n : 1)));
    LF_TRY(lf_tmp_alloc(h, (void **)&v1, sizeof(int) * (n > 0 ? n : 1)));
    LF_TRY(lf_tmp_alloc(h, (void **)&v1b, sizeof(int) * (n > 0 ? n : 1)));
    LF_TRY(lf_tmp_alloc(h, (void **)&k2, sizeof(unsigned long long) * (n > 0 ? n : 1)));
    LF_TRY(lf_tmp_alloc(h, (void **)&k2b, sizeof(unsigned long long) * (n > 0 ? n : 1)));
    unsigned *rk1;
    int *rv1;
    if (n > 0) hipLaunchKernelGGL(k_order_keys_deg, dim3(grid_for(n, BS)), dim3(BS), 0, st, h->deg, n, h->max_deg, k1, v1);
    LF_TRY(lf_sort_pairs_u32_i32(h, k1, k1b, v1, v1b, n, &rk1, &rv1));
    if (n > 0) hipLaunchKernelGGL(k_order_keys_cc, dim3(grid_for(n, BS)), dim3(BS), 0, st, h->ccl, rv1, n, k2);
    int *other = (rv1 == v1) ? v1b : v1;
    unsigned long long *rk2;
    int *rv2;
    LF_TRY(lf_sort_pairs_u64_i32(h, k2, k2b, rv1, other, n, 62, &rk2, &rv2));
    LF_HIP(h, hipMemcpyAsync(h->order, rv2, sizeof(int) * (n > 0 ? n : 1), hipMemcpyDeviceToDevice, st));
    if (n > 0) hipLaunchKernelGGL(k_rank, dim3(grid_for(n, BS)), dim3(BS), 0, st, h->order, n, h->rank);
    if (m > 0) hipLaunchKernelGGL(k_col_rank, dim3(grid_for(m, BS)), dim3(BS), 0, st, h->col, m, h->rank, h->col_rank);
    unsigned long long ht = 0;
    LF_HIP(h, hipMemcpyAsync(&h->cc, dcc, sizeof(double), hipMemcpyDeviceToHost, st));
    LF_HIP(h, hipMemcpyAsync(&ht, tsum, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    LF_HIP(h, hipMemcpyAsync(hc, cnt, sizeof(int) * 4, hipMemcpyDeviceToHost, st));
    LF_HIP(h, hipStreamSynchronize(st));
    LF_HIP(h, hipGetLastError());
    LF_TRY(lf_prof_end(h, LF_K_ORDER, 7));
    LF_TRY(lf_prof_flush(h));
    if (n == 0) h->cc = 0.0;
    h->T = (long long)(ht / 3);
    if (hc[0]) return lf_set_error(h, LF_EINTERNAL, "clustering coefficient not exactly summable");
    if (ht % 3) return lf_set_error(h, LF_EINTERNAL, "triangle credits not divisible by 3");
    return LF_OK;
}
