// post.hip -- optional post-processing of the final cover (Methods, "Post-processing":
// communities may be duplicated or contained in one another, which some uses do not
// want).
//
// A community A (at least one member) is removed as a duplicate if another community has
// exactly its members and a lower id, and as contained if its members are a strict subset
// of another community's.  Every community that contains A includes A's first member, so
// the candidates are that member's other communities; A is contained in B when every
// member of A lists B.  One wave per community: the lanes test A's members against one
// candidate at a time.  The removal can be applied: the remaining cover then rebuilds the
// state exactly as a warm start does.
#include "lf_internal.h"

#define WAVE 64

static inline unsigned grid_for(long long n, int block) { return (unsigned)((n + block - 1) / block); }

__global__ void __launch_bounds__(256) k_pp_check(const CommRec *cr, const long long *cm_off, const int *cm_len,
                                                  const int *cm_node, const NodeHdr *nh, const Slot *slot, int K,
                                                  unsigned flags, unsigned char *keep, unsigned long long *cnt,
                                                  int *err)
{
    const long long a = (blockIdx.x * (long long)blockDim.x + threadIdx.x) / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    if (a >= K) return;
    const int sa = cr[a].s, la = cm_len[a];
    if (sa != la) {                          // member lists must be current
        if (lane == 0) atomicOr(err, 1);
        return;
    }
    if (sa == 0) {
        if (lane == 0) keep[a] = 0;
        return;
    }
    const long long base = cm_off[a];
    const NodeHdr h0 = nh[cm_node[base]];
    bool dup = false, cont = false;
    for (int t = 0; t < h0.cnt; t++) {       // uniform over the wave
        const int b = slot[h0.off + t].comm;
        if (b == a) continue;
        const int sb = cr[b].s;
        if (sb < sa) continue;
        if (sb == sa && !((flags & LF_PP_DUPLICATES) && b < a)) continue;
        if (sb > sa && !(flags & LF_PP_CONTAINED)) continue;
        bool miss = false;
        for (int i = lane; i < la; i += WAVE) {
            const NodeHdr hy = nh[cm_node[base + i]];
            bool found = false;
            for (int u = 0; u < hy.cnt; u++) found |= slot[hy.off + u].comm == b;
            miss |= !found;
        }
        if (__ballot(miss) == 0) {
            if (sb == sa) dup = true;
            else cont = true;
        }
    }
    if (lane == 0) {
        keep[a] = !(dup || cont);
        if (dup) atomicAdd(&cnt[0], 1ull);
        else if (cont) atomicAdd(&cnt[1], 1ull);
    }
}

// the kept part of the cover as CSR: counts, then ids (slot order)
__global__ void k_pp_counts(const NodeHdr *nh, const Slot *slot, const unsigned char *keep, long long n,
                            long long *cnt)
{
    const long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (x > n) return;
    if (x == n) {
        cnt[n] = 0;
        return;
    }
    const NodeHdr hx = nh[x];
    long long c = 0;
    for (int t = 0; t < hx.cnt; t++) c += keep[slot[hx.off + t].comm];
    cnt[x] = c;
}

__global__ void k_pp_fill(const NodeHdr *nh, const Slot *slot, const unsigned char *keep, long long n,
                          const long long *off, int *ids)
{
    const long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (x >= n) return;
    const NodeHdr hx = nh[x];
    long long p = off[x];
    for (int t = 0; t < hx.cnt; t++) {
        const int c = slot[hx.off + t].comm;
        if (keep[c]) ids[p++] = c;
    }
}

extern "C" int lf_postprocess(lf_handle *h, uint32_t flags, uint8_t *keep, int64_t *removed)
{
    if (!h) return LF_EINVAL;
    if (flags & ~(LF_PP_DUPLICATES | LF_PP_CONTAINED | LF_PP_APPLY)) return lf_set_error(h, LF_EINVAL, "unknown flags");
    if (h->state < 2) return lf_set_error(h, LF_ESTATE, "no communities yet");
    LF_HIP(h, hipSetDevice(h->device));
    TmpScope tmp_scope(h);
    hipStream_t st = h->stream;
    const int BS = 256;
    const long long n = h->n;
    const int K = h->K;
    unsigned char *dkeep = nullptr;
    unsigned long long *cnt = nullptr;
    int *err = nullptr;
    LF_TRY(lf_tmp_alloc(h, (void **)&dkeep, K > 0 ? K : 1));
    LF_TRY(lf_tmp_alloc(h, (void **)&cnt, 2 * sizeof(unsigned long long)));
    LF_TRY(lf_tmp_alloc(h, (void **)&err, sizeof(int)));
    LF_HIP(h, hipMemsetAsync(cnt, 0, 2 * sizeof(unsigned long long), st));
    LF_HIP(h, hipMemsetAsync(err, 0, sizeof(int), st));
    if (K > 0)
        hipLaunchKernelGGL(k_pp_check, dim3(grid_for((long long)K * WAVE, BS)), dim3(BS), 0, st, h->cr, h->cm_off,
                           h->cm_len, h->cm_node, h->nh, h->slot[h->cur], K, flags, dkeep, cnt, err);
    unsigned long long hc[2] = {0, 0};
    int herr = 0;
    LF_HIP(h, hipMemcpyAsync(hc, cnt, sizeof hc, hipMemcpyDeviceToHost, st));
    LF_HIP(h, hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
    if (keep && K > 0) LF_HIP(h, hipMemcpyAsync(keep, dkeep, K, hipMemcpyDeviceToHost, st));
    LF_HIP(h, hipStreamSynchronize(st));
    LF_HIP(h, hipGetLastError());
    if (herr) return lf_set_error(h, LF_EINTERNAL, "member lists out of date");
    if (removed) {
        removed[0] = (int64_t)hc[0];
        removed[1] = (int64_t)hc[1];
    }
    if (flags & LF_PP_APPLY) {
        long long *pc = nullptr, *off = nullptr;
        LF_TRY(lf_tmp_alloc(h, (void **)&pc, sizeof(long long) * (n + 1)));
        LF_TRY(lf_tmp_alloc(h, (void **)&off, sizeof(long long) * (n + 1)));
        hipLaunchKernelGGL(k_pp_counts, dim3(grid_for(n + 1, BS)), dim3(BS), 0, st, h->nh, h->slot[h->cur], dkeep,
                           n, pc);
        LF_TRY(lf_exclusive_scan_i64(h, pc, off, n + 1));
        long long total = 0;
        LF_HIP(h, hipMemcpyAsync(&total, off + n, sizeof(long long), hipMemcpyDeviceToHost, st));
        LF_HIP(h, hipStreamSynchronize(st));
        int *ids = nullptr;
        LF_TRY(lf_tmp_alloc(h, (void **)&ids, sizeof(int) * (total > 0 ? total : 1)));
        if (n > 0)
            hipLaunchKernelGGL(k_pp_fill, dim3(grid_for(n, BS)), dim3(BS), 0, st, h->nh, h->slot[h->cur], dkeep, n,
                               off, ids);
        LF_HIP(h, hipGetLastError());
        LF_TRY(lf_partition_from_cover(h, off, ids, total, K));
    }
    return LF_OK;
}
