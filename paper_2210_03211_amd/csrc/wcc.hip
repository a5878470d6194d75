// wcc.hip -- exact WCC of the current partition (Methods, WCC-hat subsection, paragraph
// "WCC"), to set beside the WCC-hat estimate that the iterations optimise.
//
// For a member x of community C, with t(x,S) the triangles of x whose two other nodes lie
// in S and vt(x,S) the nodes of S that close at least one triangle with x:
//   WCC(x,C) = t(x,C) / t(x,V) * vt(x,V) / (|C \ {x}| + vt(x, V \ C)),  0 if t(x,V) = 0,
//   WCC(C) = sum of WCC(x,C) over x in C,  WCC(P) = sum of WCC(C) over the communities.
// A node term is evaluated in FP64 as (t / t_V) * (vt_V / (|C| - 1 + vt_out)) -- three
// IEEE roundings -- and every sum is exact (fixed point), rounded once.  Since
// vt(x,V) <= |C \ {x}| + vt(x, V \ C), every term lies in [0, 1].
//
// Passes (all on the handle's stream):
//   1. compact memberships: each node's community ids, ascending (the order in which
//      lf_get_memberships lists them), with the owning node of each membership;
//   2. the oriented triangle enumeration of the node statistics (every triangle once, at
//      its lowest endpoint in (degree, id) order) marks each oriented edge that closes a
//      triangle and adds one to t(x,C) at all three corners for every community the three
//      nodes share;
//   3. one wave per node: per adjacency position whether the edge closes a triangle, and
//      vt(x,V);
//   4. one wave per membership: vt(x, V \ C), the node term, its digits into the
//      community's carry-save counters;
//   5. community totals folded and rounded; the partition total summed exactly.
#include "lf_internal.h"

#define WAVE 64

static inline unsigned grid_for(long long n, int block) { return (unsigned)((n + block - 1) / block); }

__device__ __forceinline__ bool wcc_before(int du, int u, int dv, int v)
{
    return du < dv || (du == dv && u < v);
}

// position of v in the ascending list a[0, m), -1 if absent
__device__ __forceinline__ long long sorted_find(const int *a, long long m, int v)
{
    long long lo = 0, hi = m - 1;
    while (lo <= hi) {
        long long mid = (lo + hi) >> 1;
        int x = a[mid];
        if (x == v) return mid;
        if (x < v) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

// 1. node x's community ids in ascending order at [moff[x], moff[x + 1]), owner per entry
__global__ void k_wcc_compact(const NodeHdr *nh, const Slot *slot, long long n, const long long *moff, int *mid,
                              int *mnode)
{
    long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (x >= n) return;
    const NodeHdr hx = nh[x];
    const long long o = moff[x];
    for (int t = 0; t < hx.cnt; t++) {          // insertion sort of a handful of entries
        const int c = slot[hx.off + t].comm;
        int b = t;
        while (b > 0 && mid[o + b - 1] > c) {
            mid[o + b] = mid[o + b - 1];
            b--;
        }
        mid[o + b] = c;
        mnode[o + t] = (int)x;
    }
}

__global__ void k_wcc_counts(const NodeHdr *nh, long long n, long long *cnt)
{
    long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (x < n) cnt[x] = nh[x].cnt;
    if (x == n) cnt[n] = 0;
}

// 3. hasf[e] = 1 if the edge at adjacency position e closes a triangle; vt[x] = their
//    number in row x.  The edge x-y is oriented from the endpoint first in (degree, id)
//    order; x's out-neighbours are the row's later-ordered entries in row order.
__global__ void __launch_bounds__(256) k_wcc_closing(const long long *rowptr, const int *col, const int *deg,
                                                     const long long *oro, const int *orc,
                                                     const unsigned char *eflag, long long n,
                                                     unsigned char *hasf, int *vt)
{
    const long long x = (blockIdx.x * (long long)blockDim.x + threadIdx.x) / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    if (x >= n) return;
    const int dx = deg[x];
    const long long r1 = rowptr[x + 1];
    long long wpos = oro[x];
    int cnt = 0;
    for (long long base = rowptr[x]; base < r1; base += WAVE) {
        const long long e = base + lane;
        bool out = false;
        int y = 0;
        if (e < r1) {
            y = col[e];
            out = wcc_before(dx, (int)x, deg[y], y);
        }
        const unsigned long long mask = __ballot(out);
        if (e < r1) {
            long long idx;
            if (out) {
                idx = wpos + __popcll(mask & ((1ull << lane) - 1));
            } else {
                const long long b = oro[y];
                const long long p = sorted_find(orc + b, oro[y + 1] - b, (int)x);   // x-y is an edge
                idx = p >= 0 ? b + p : -1;
            }
            const unsigned char f = idx >= 0 ? eflag[idx] : 0;
            hasf[e] = f;
            cnt += f;
        }
        wpos += __popcll(mask);
    }
    cnt = wave_sum_int(cnt);
    if (lane == 0) vt[x] = cnt;
}

// 4. one wave per membership m = (x, C): vt(x, V \ C), the node term, community digits
__global__ void __launch_bounds__(256) k_wcc_terms(const long long *rowptr, const int *col,
                                                   const unsigned long long *tri, const CommRec *cr,
                                                   const long long *moff, const int *mid, const int *mnode,
                                                   const int *tcm, const unsigned char *hasf, const int *vt,
                                                   long long total, double *wn, int *vto, long long *cdig,
                                                   int *err)
{
    const long long m = (blockIdx.x * (long long)blockDim.x + threadIdx.x) / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    if (m >= total) return;
    const int x = mnode[m], c = mid[m];
    const long long r1 = rowptr[x + 1];
    int out = 0;
    for (long long e = rowptr[x] + lane; e < r1; e += WAVE) {
        if (!hasf[e]) continue;
        const int y = col[e];
        const long long b = moff[y];
        out += sorted_find(mid + b, moff[y + 1] - b, c) < 0;
    }
    out = wave_sum_int(out);
    if (lane != 0) return;
    const unsigned long long kx = tri[x];
    const long long s = cr[c].s;
    double w = 0.0;
    if (kx > 0) {
        const double a = (double)tcm[m] / (double)kx;
        const double b = (double)vt[x] / (double)(s - 1 + out);
        w = a * b;
    }
    wn[m] = w;
    vto[m] = out;
    int bad = 0;
    const X192 v = x192_from_double(w, bad);
    i64 d0, d1, d2, d3;
    x192_digits(v, d0, d1, d2, d3);
    long long *cd = cdig + 4 * (long long)c;
    if (d0) atomicAdd((unsigned long long *)&cd[0], (unsigned long long)d0);
    if (d1) atomicAdd((unsigned long long *)&cd[1], (unsigned long long)d1);
    if (d2) atomicAdd((unsigned long long *)&cd[2], (unsigned long long)d2);
    if (d3) atomicAdd((unsigned long long *)&cd[3], (unsigned long long)d3);
    if (bad) atomicOr(err, 1);
}

// 5. WCC(C) = the community's exact sum, rounded once
__global__ void k_wcc_comm_fold(const long long *cdig, int K, double *wc)
{
    const long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (c >= K) return;
    const long long *d = cdig + 4 * c;
    wc[c] = x192_round(x192_from_digits(d[0], d[1], d[2], d[3]));
}

extern "C" int lf_exact_wcc(lf_handle *h, double *wcc, double *wcc_comm, double *wcc_node, int32_t *t_xc,
                            int32_t *vt_xc, int32_t *vt_x)
{
    if (!h || !wcc) return LF_EINVAL;
    if (h->state < 2) return lf_set_error(h, LF_ESTATE, "no communities yet");
    LF_HIP(h, hipSetDevice(h->device));
    TmpScope tmp_scope(h);
    hipStream_t st = h->stream;
    const int BS = 256;
    const long long n = h->n;
    const int K = h->K;
    // 1. compact memberships
    long long *cnt = nullptr, *moff = nullptr;
    LF_TRY(lf_tmp_alloc(h, (void **)&cnt, sizeof(long long) * (n + 1)));
    LF_TRY(lf_tmp_alloc(h, (void **)&moff, sizeof(long long) * (n + 1)));
    hipLaunchKernelGGL(k_wcc_counts, dim3(grid_for(n + 1, BS)), dim3(BS), 0, st, h->nh, n, cnt);
    LF_TRY(lf_exclusive_scan_i64(h, cnt, moff, n + 1));
    long long total = 0;
    LF_HIP(h, hipMemcpyAsync(&total, moff + n, sizeof(long long), hipMemcpyDeviceToHost, st));
    LF_HIP(h, hipStreamSynchronize(st));
    const size_t tt = (size_t)(total > 0 ? total : 1);
    int *mid = nullptr, *mnode = nullptr, *tcm = nullptr, *vto = nullptr, *vt = nullptr, *err = nullptr;
    double *wn = nullptr, *wc = nullptr;
    long long *cdig = nullptr;
    unsigned char *eflag = nullptr, *hasf = nullptr;
    LF_TRY(lf_tmp_alloc(h, (void **)&mid, sizeof(int) * tt));
    LF_TRY(lf_tmp_alloc(h, (void **)&mnode, sizeof(int) * tt));
    LF_TRY(lf_tmp_alloc(h, (void **)&tcm, sizeof(int) * tt));
    LF_TRY(lf_tmp_alloc(h, (void **)&vto, sizeof(int) * tt));
    LF_TRY(lf_tmp_alloc(h, (void **)&wn, sizeof(double) * tt));
    LF_TRY(lf_tmp_alloc(h, (void **)&vt, sizeof(int) * (n > 0 ? n : 1)));
    LF_TRY(lf_tmp_alloc(h, (void **)&err, sizeof(int)));
    LF_TRY(lf_tmp_alloc(h, (void **)&cdig, sizeof(long long) * 4 * (K > 0 ? K : 1)));
    LF_TRY(lf_tmp_alloc(h, (void **)&wc, sizeof(double) * (K > 0 ? K : 1)));
    LF_TRY(lf_tmp_alloc(h, (void **)&eflag, h->ne > 0 ? h->ne : 1));
    LF_TRY(lf_tmp_alloc(h, (void **)&hasf, 2 * h->ne > 0 ? 2 * h->ne : 1));
    LF_HIP(h, hipMemsetAsync(tcm, 0, sizeof(int) * tt, st));
    LF_HIP(h, hipMemsetAsync(err, 0, sizeof(int), st));
    LF_HIP(h, hipMemsetAsync(cdig, 0, sizeof(long long) * 4 * (K > 0 ? K : 1), st));
    LF_HIP(h, hipMemsetAsync(eflag, 0, h->ne > 0 ? h->ne : 1, st));
    if (n > 0)
        hipLaunchKernelGGL(k_wcc_compact, dim3(grid_for(n, BS)), dim3(BS), 0, st, h->nh, h->slot[h->cur], n, moff,
                           mid, mnode);
    // 2. triangles
    WccTri wt;
    wt.moff = moff;
    wt.mid = mid;
    wt.tcm = tcm;
    wt.eflag = eflag;
    int launches = 0;
    long long *oro = nullptr;
    int *orc = nullptr;
    LF_TRY(lf_triangle_pass(h, &wt, &launches, &oro, &orc));
    // 3. closing edges per adjacency position, vt(x, V)
    if (n > 0)
        hipLaunchKernelGGL(k_wcc_closing, dim3(grid_for(n * WAVE, BS)), dim3(BS), 0, st, h->rowptr, h->col, h->deg,
                           oro, orc, eflag, n, hasf, vt);
    // 4. node terms
    if (total > 0)
        hipLaunchKernelGGL(k_wcc_terms, dim3(grid_for(total * WAVE, BS)), dim3(BS), 0, st, h->rowptr, h->col,
                           h->tri, h->cr, moff, mid, mnode, tcm, hasf, vt, total, wn, vto, cdig, err);
    // 5. totals
    if (K > 0) hipLaunchKernelGGL(k_wcc_comm_fold, dim3(grid_for(K, BS)), dim3(BS), 0, st, cdig, K, wc);
    LF_HIP(h, hipGetLastError());
    int herr = 0;
    LF_HIP(h, hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
    LF_HIP(h, hipStreamSynchronize(st));
    if (herr) return lf_set_error(h, LF_EOVERFLOW, "a WCC term is outside the exact accumulator's range");
    LF_TRY(lf_exact_sum_dev(h, wn, total, wcc));
    if (wcc_comm && K > 0) LF_HIP(h, hipMemcpyAsync(wcc_comm, wc, sizeof(double) * K, hipMemcpyDeviceToHost, st));
    if (wcc_node && total > 0) LF_HIP(h, hipMemcpyAsync(wcc_node, wn, sizeof(double) * total, hipMemcpyDeviceToHost, st));
    if (t_xc && total > 0) LF_HIP(h, hipMemcpyAsync(t_xc, tcm, sizeof(int) * total, hipMemcpyDeviceToHost, st));
    if (vt_xc && total > 0) LF_HIP(h, hipMemcpyAsync(vt_xc, vto, sizeof(int) * total, hipMemcpyDeviceToHost, st));
    if (vt_x && n > 0) LF_HIP(h, hipMemcpyAsync(vt_x, vt, sizeof(int) * n, hipMemcpyDeviceToHost, st));
    LF_HIP(h, hipStreamSynchronize(st));
    LF_HIP(h, hipGetLastError());
    return LF_OK;
}
