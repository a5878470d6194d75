// communities.hip -- initial clustering and LazyFox iterations on the GPU.
//
// Method (Garrels et al., arXiv 2210.03211, Methods):
//  * Initial clustering: in node order, a node without a community opens a new one and its
//    unassigned neighbours join it.  Equivalently, the openers are the lexicographically
//    first maximal independent set in rank order, and every other node joins the
//    lowest-ranked opener among its neighbours; community ids number the openers by rank.
//    The GPU decides openers in rounds (a node is decided once all lower-ranked neighbours
//    are), resuming each node's neighbour scan where it stopped.
//  * WCC-hat (WCC-hat subsection): for a member x of C with d = deg(x,V), i = deg(x,C),
//    s = |C| and community density p, WCC-hat(x,C) = p * g(i,d,s) / cc with
//    g = i(i-1) / ((d-1)(s-1+d-i)) (0 if i < 2 or d < 2).  cc > 0 scales every term alike,
//    so all decisions use the cc-free community score W(C) = fl(p * R(sum_y g)), R = exact
//    sum rounded once.
//  * Node changes (Algorithm 2): for every node x of a queue, on the state at the start of
//    the queue, the change of W(C) when x joins a community C of a neighbour (or leaves one
//    of its own).  With stored exact sums S+ = sum g(i_y, d_y, s+1) and
//    S- = sum g(i_y, d_y, s-1) over C's members, only x's neighbours in C change their in-
//    count, so
//      join:  W' = p(s+1, m+k) * R(S+ + sum_{y in N(x)∩C} [g(i_y+1,..,s+1) - g(i_y,..,s+1)]
//                                     + g(k, d_x, s+1))
//      leave: W' = p(s-1, m-k) * R(S- + sum_{y in N(x)∩C} [g(i_y-1,..,s-1) - g(i_y,..,s-1)]
//                                     - g(k, d_x, s-1))
//    with k = |N(x) ∩ C|.  A move is taken if W' - W(C) > 0, the largest wins, ties go to
//    the lowest community id; the best join and the best leave are both applied.
//  * Bulk apply: membership edits, community sizes, in-counts of the affected neighbours
//    (integer atomics; a node that joined in this queue is counted afresh), then an exact
//    re-sum of every touched community (size changes alter every member's term).
//  * Iteration end: communities with < 2 members are removed, membership slots compacted
//    (+1 free slot per node: a node gains at most one community per iteration), member
//    lists rebuilt and the exact partition score reduced.
//
// Layout in HBM: CSR (rowptr int64, col int32); per node a 16-byte header {slot offset,
// count, degree}; membership slots {community, in-count} (8 bytes); per community SoA
// arrays (size, internal edges, score, S+ and S- as 192-bit fixed point); member lists with
// per-community capacity for the iteration's joiners (overflow goes to a global list).
#include "lf_internal.h"

#define WAVE 64
#define EW 4            // waves per block in the wave evaluation path
#define ECAP 128        // table entries per wave (power of two)
#define MXCAP 32        // memberships of the evaluated node kept in LDS (wave path)

static inline unsigned grid_for(long long n, int block) { return (unsigned)((n + block - 1) / block); }

__device__ __forceinline__ double g_term(long long i, long long d, long long s)
{
    if (d < 2 || i < 2) return 0.0;
    long long num = i * (i - 1);
    long long den = (d - 1) * (s - 1 + d - i);
    return (double)num / (double)den;
}

__device__ __forceinline__ double density(long long s, long long m)
{
    if (s < 2) return 0.0;
    return (double)(2 * m) / (double)(s * (s - 1));
}

#define WAVE_SYNC()                                                                        \
    do {                                                                                   \
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");                             \
        __builtin_amdgcn_wave_barrier();                                                   \
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");                             \
    } while (0)

// ------------------------------------------------------------------------------------
// A3: initial clustering
// ------------------------------------------------------------------------------------
// state: 0 undecided, 1 opener, 2 joins an opener
__global__ void k_lfmis_round(const long long *rowptr, const int *col, const int *rank, long long n,
                              int *state, int *cursor, int *undecided)
{
    int cnt = 0;
    for (long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x; x < n;
         x += (long long)gridDim.x * blockDim.x) {
        if (__atomic_load_n(&state[x], __ATOMIC_RELAXED) != 0) continue;
        int rx = rank[x];
        long long b = rowptr[x], e = rowptr[x + 1];
        long long c = b + cursor[x];
        int mine = 0;
        bool pending = false;
        for (; c < e; c++) {
            int y = col[c];
            if (rank[y] >= rx) continue;
            int sy = __atomic_load_n(&state[y], __ATOMIC_RELAXED);
            if (sy == 1) { mine = 2; break; }
            if (sy == 0) { pending = true; break; }
        }
        cursor[x] = (int)(c - b);
        if (mine == 0 && !pending) mine = 1;
        if (mine) __atomic_store_n(&state[x], mine, __ATOMIC_RELAXED);
        else cnt++;
    }
    cnt = wave_sum_int(cnt);
    if ((threadIdx.x & (WAVE - 1)) == 0 && cnt) atomicAdd(undecided, cnt);
}

__global__ void k_opener_flags(const int *order, const int *state, long long n, int *flag)
{
    long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (r >= n) return;
    flag[r] = state[order[r]] == 1;
}

__global__ void k_opener_ids(const int *order, const int *flag, const long long *pos, long long n, int *comm_of)
{
    long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (r >= n) return;
    if (flag[r]) comm_of[order[r]] = (int)pos[r];
}

// every non-opener joins its lowest-ranked opener neighbour; one wave per node
__global__ void __launch_bounds__(256) k_join_openers(const long long *rowptr, const int *col, const int *rank,
                                                      const int *state, long long n, int *comm_of)
{
    long long x = (blockIdx.x * (long long)blockDim.x + threadIdx.x) / WAVE;
    int lane = threadIdx.x & (WAVE - 1);
    if (x >= n || state[x] != 2) return;
    int best = 0x7fffffff, who = -1;
    for (long long e = rowptr[x] + lane; e < rowptr[x + 1]; e += WAVE) {
        int y = col[e];
        if (state[y] == 1 && rank[y] < best) { best = rank[y]; who = y; }
    }
    for (int m = 32; m >= 1; m >>= 1) {
        int ob = __shfl_xor(best, m, WAVE), ow = __shfl_xor(who, m, WAVE);
        if (ob < best) { best = ob; who = ow; }
    }
    if (lane == 0) comm_of[x] = comm_of[who];
}

// one membership per node plus one free slot; in-count within its community
__global__ void __launch_bounds__(256) k_init_slots(const long long *rowptr, const int *col, const int *deg,
                                                    const int *comm_of, long long n, NodeHdr *nh, Slot *slot,
                                                    int *cs)
{
    long long x = (blockIdx.x * (long long)blockDim.x + threadIdx.x) / WAVE;
    int lane = threadIdx.x & (WAVE - 1);
    if (x > n) return;
    if (x == n) {
        if (lane == 0) { nh[n].off = 2 * n; nh[n].cnt = 0; nh[n].deg = 0; }
        return;
    }
    int c = comm_of[x];
    int in = 0;
    for (long long e = rowptr[x] + lane; e < rowptr[x + 1]; e += WAVE) in += comm_of[col[e]] == c;
    in = wave_sum_int(in);
    if (lane == 0) {
        NodeHdr hd;
        hd.off = 2 * x;
        hd.cnt = 1;
        hd.deg = deg[x];
        nh[x] = hd;
        Slot s0 = {c, in}, s1 = {-1, 0};
        slot[2 * x] = s0;
        slot[2 * x + 1] = s1;
        atomicAdd(&cs[c], 1);
    }
}

// ------------------------------------------------------------------------------------
// member lists (rebuilt at initialisation and at every iteration end)
// ------------------------------------------------------------------------------------
// capacity: current members plus room for joiners (sum of member degrees, at most n)
__global__ void k_member_extra(const NodeHdr *nh, const Slot *slot, long long n, long long *capx)
{
    long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (x >= n) return;
    NodeHdr hd = nh[x];
    for (int t = 0; t < hd.cnt; t++) atomicAdd((unsigned long long *)&capx[slot[hd.off + t].comm], (unsigned long long)hd.deg);
}

__global__ void k_member_cap(long long *capx, const int *cs, int K, long long n)
{
    long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (c >= K) return;
    long long ex = capx[c];
    if (ex > n) ex = n;
    capx[c] = cs[c] + ex;
}

__global__ void k_member_fill(const NodeHdr *nh, const Slot *slot, long long n, const long long *cm_off,
                              int *cm_len, int *cm_node)
{
    long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (x >= n) return;
    NodeHdr hd = nh[x];
    for (int t = 0; t < hd.cnt; t++) {
        int c = slot[hd.off + t].comm;
        int p = atomicAdd(&cm_len[c], 1);
        cm_node[cm_off[c] + p] = (int)x;
    }
}

__global__ void k_iota(int *a, long long n)
{
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i < n) a[i] = (int)i;
}

// ------------------------------------------------------------------------------------
// exact re-sum of touched communities (persistent: each wave takes communities from the
// touched list until it is exhausted)
// ------------------------------------------------------------------------------------
__device__ __forceinline__ int find_slot(const Slot *slot, long long off, int cnt, int c)
{
    for (int t = 0; t < cnt; t++)
        if (slot[off + t].comm == c) return t;
    return -1;
}

__device__ __forceinline__ void member_terms(const Ctx &cx, int y, int C, long long s, X192 &a0, X192 &ap,
                                             X192 &am, long long &sumi, int &bad)
{
    NodeHdr hy = cx.nh[y];
    int t = find_slot(cx.slot, hy.off, hy.cnt, C);
    if (t < 0) return;                       // left C earlier in this iteration
    long long i = cx.slot[hy.off + t].in;
    long long d = hy.deg;
    sumi += i;
    X192 v = x192_from_double(g_term(i, d, s), bad);
    x192_add(a0, v);
    v = x192_from_double(g_term(i, d, s + 1), bad);
    x192_add(ap, v);
    v = x192_from_double(g_term(i, d, s - 1), bad);
    x192_add(am, v);
}

__global__ void __launch_bounds__(256) k_refresh(Ctx cx, int fixed_count)
{
    int lane = threadIdx.x & (WAVE - 1);
    int count = fixed_count >= 0 ? fixed_count : __atomic_load_n(&cx.ctr->tcount, __ATOMIC_RELAXED);
    int bad = 0;
    while (true) {
        int idx = 0;
        if (lane == 0) idx = atomicAdd(&cx.ctr->refresh_next, 1);
        idx = __shfl(idx, 0, WAVE);
        if (idx >= count) break;
        int C = cx.tlist[idx];
        long long s = cx.cs[C];
        long long base = cx.cm_off[C];
        long long cap = cx.cm_off[C + 1] - base;
        long long len = cx.cm_len[C];
        if (len > cap) len = cap;
        X192 a0 = x192_zero(), ap = x192_zero(), am = x192_zero();
        long long sumi = 0;
        for (long long j = lane; j < len; j += WAVE)
            member_terms(cx, cx.cm_node[base + j], C, s, a0, ap, am, sumi, bad);
        if (cx.ovf_flag[C]) {
            int no = __atomic_load_n(&cx.ctr->ovf_cnt, __ATOMIC_RELAXED);
            for (int e = lane; e < no; e += WAVE)
                if (cx.ovf_comm[e] == C) member_terms(cx, cx.ovf_node[e], C, s, a0, ap, am, sumi, bad);
        }
        a0 = wave_sum_x192(a0);
        ap = wave_sum_x192(ap);
        am = wave_sum_x192(am);
        sumi = wave_sum_i64(sumi);
        if (lane == 0) {
            if (sumi & 1) atomicOr(&cx.ctr->error, LF_DEVERR_ODD);
            long long m = sumi / 2;
            cx.cm[C] = m;
            cx.cW[C] = density(s, m) * x192_round(a0);
            cx.cSp[C] = ap;
            cx.cSm[C] = am;
            cx.tflag[C] = 0;
        }
    }
    if (bad) atomicOr(&cx.ctr->error, LF_DEVERR_INEXACT);
}

// ------------------------------------------------------------------------------------
// A4: evaluation
// ------------------------------------------------------------------------------------
__global__ void k_chunk_begin(Ctx cx, int prev_start, int prev_len)
{
    long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (j == 0) {
        cx.ctr->tcount = 0;
        cx.ctr->hub_count = 0;
        cx.ctr->hub_next = 0;
        cx.ctr->refresh_next = 0;
    }
    if (j < prev_len) cx.joined_to[cx.order[prev_start + j]] = -1;
}

__device__ __forceinline__ unsigned hash_tab(int c) { return (unsigned)c * 0x9E3779B1u; }
__device__ __forceinline__ unsigned hash_part(int c) { return ((unsigned)c * 0x85EBCA77u) ^ ((unsigned)c >> 13); }

// candidate-change term of one neighbour membership (y in C with in-count i)
__device__ __forceinline__ X192 visit_term(bool leave, long long i, long long dy, long long s, int &bad)
{
    double gn, go;
    if (leave) { gn = g_term(i - 1, dy, s - 1); go = g_term(i, dy, s - 1); }
    else { gn = g_term(i + 1, dy, s + 1); go = g_term(i, dy, s + 1); }
    X192 t = x192_from_double(gn, bad);
    X192 o = x192_from_double(go, bad);
    x192_sub(t, o);
    return t;
}

// change of C's cc-free score for x joining (leave = false) or leaving C
__device__ __forceinline__ double candidate_delta(const Ctx &cx, int C, bool leave, long long k, long long dx,
                                                  X192 corr, int &bad)
{
    long long s = cx.cs[C];
    long long m = cx.cm[C];
    X192 S;
    double p;
    if (leave) {
        S = cx.cSm[C];
        x192_add(S, corr);
        X192 own = x192_from_double(g_term(k, dx, s - 1), bad);
        x192_sub(S, own);
        p = density(s - 1, m - k);
    } else {
        S = cx.cSp[C];
        x192_add(S, corr);
        X192 own = x192_from_double(g_term(k, dx, s + 1), bad);
        x192_add(S, own);
        p = density(s + 1, m + k);
    }
    double pS = p * x192_round(S);
    return pS - cx.cW[C];
}

__device__ __forceinline__ void better(double d, int c, double &bd, int &bc)
{
    if (!(d > 0.0)) return;
    if (bc < 0 || d > bd || (d == bd && c < bc)) { bd = d; bc = c; }
}

__device__ __forceinline__ void wave_best(double &bd, int &bc)
{
    for (int m = 32; m >= 1; m >>= 1) {
        double od = __shfl_xor(bd, m, WAVE);
        int oc = __shfl_xor(bc, m, WAVE);
        if (oc >= 0 && (bc < 0 || od > bd || (od == bd && oc < bc))) { bd = od; bc = oc; }
    }
}

// one wave per queued node whose candidate table fits ECAP/2 entries; others are deferred
__global__ void __launch_bounds__(EW * WAVE) k_eval(Ctx cx, int cstart, int clen)
{
    __shared__ int s_key[EW][ECAP];
    __shared__ int s_k[EW][ECAP];
    __shared__ unsigned long long s_d[EW][4][ECAP];
    __shared__ int s_mx[EW][MXCAP];
    __shared__ int s_mxin[EW][MXCAP];
    int wv = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
    int j = blockIdx.x * EW + wv;
    if (j >= clen) return;                  // no block barriers in this kernel
    int x = cx.order[cstart + j];
    NodeHdr hx = cx.nh[x];
    long long rb = cx.rowptr[x], re = cx.rowptr[x + 1];
    int V = 0;
    for (long long e = rb + lane; e < re; e += WAVE) V += cx.nh[cx.col[e]].cnt;
    V = wave_sum_int(V);
    int need = V + hx.cnt;
    if (2 * need > ECAP || hx.cnt > MXCAP) {
        if (lane == 0) cx.hub_list[atomicAdd(&cx.ctr->hub_count, 1)] = j;
        return;
    }
    int T = 8;
    while (T < 2 * need) T <<= 1;
    int lg = 31 - __clz(T);
    int *key = s_key[wv], *kk = s_k[wv];
    unsigned long long *d0 = s_d[wv][0], *d1 = s_d[wv][1], *d2 = s_d[wv][2], *d3 = s_d[wv][3];
    for (int t = lane; t < T; t += WAVE) {
        key[t] = -1; kk[t] = 0; d0[t] = 0; d1[t] = 0; d2[t] = 0; d3[t] = 0;
    }
    if (lane < hx.cnt) {
        Slot sl = cx.slot[hx.off + lane];
        s_mx[wv][lane] = sl.comm;
        s_mxin[wv][lane] = sl.in;
    }
    WAVE_SYNC();
    // own communities are leave candidates even without a neighbour in them
    if (lane < hx.cnt) {
        int c = s_mx[wv][lane];
        unsigned hsh = hash_tab(c) >> (32 - lg);
        while (true) {
            int old = atomicCAS(&key[hsh], -1, c);
            if (old == -1 || old == c) break;
            hsh = (hsh + 1) & (T - 1);
        }
    }
    WAVE_SYNC();
    int bad = 0;
    int mcnt = hx.cnt;
    for (long long base = rb; base < re; base += WAVE) {
        long long e = base + lane;
        bool valid = e < re;
        int y = valid ? cx.col[e] : 0;
        NodeHdr hy;
        hy.cnt = 0; hy.off = 0; hy.deg = 0;
        if (valid) hy = cx.nh[y];
        int mc = hy.cnt;
        for (int m = 32; m >= 1; m >>= 1) { int o = __shfl_xor(mc, m, WAVE); mc = o > mc ? o : mc; }
        for (int t = 0; t < mc; t++) {
            if (t < hy.cnt) {
                Slot sl = cx.slot[hy.off + t];
                int C = sl.comm;
                long long s = cx.cs[C];
                bool leave = false;
                for (int a = 0; a < mcnt; a++) leave |= (s_mx[wv][a] == C);
                X192 term = visit_term(leave, sl.in, hy.deg, s, bad);
                i64 t0, t1, t2, t3;
                x192_digits(term, t0, t1, t2, t3);
                unsigned hsh = hash_tab(C) >> (32 - lg);
                while (true) {
                    int old = atomicCAS(&key[hsh], -1, C);
                    if (old == -1 || old == C) break;
                    hsh = (hsh + 1) & (T - 1);
                }
                atomicAdd(&kk[hsh], 1);
                atomicAdd(&d0[hsh], (unsigned long long)t0);
                atomicAdd(&d1[hsh], (unsigned long long)t1);
                atomicAdd(&d2[hsh], (unsigned long long)t2);
                atomicAdd(&d3[hsh], (unsigned long long)t3);
            }
        }
    }
    WAVE_SYNC();
    double bjd = 0.0, bld = 0.0;
    int bj = -1, bl = -1, ncand = 0;
    long long dx = hx.deg;
    for (int t = lane; t < T; t += WAVE) {
        int C = key[t];
        if (C < 0) continue;
        ncand++;
        int k = kk[t];
        int a = -1;
        for (int q = 0; q < mcnt; q++)
            if (s_mx[wv][q] == C) a = q;
        bool leave = a >= 0;
        if (leave && s_mxin[wv][a] != k) atomicOr(&cx.ctr->error, LF_DEVERR_INCOUNT);
        X192 corr = x192_from_digits((i64)d0[t], (i64)d1[t], (i64)d2[t], (i64)d3[t]);
        double dl = candidate_delta(cx, C, leave, k, dx, corr, bad);
        if (leave) better(dl, C, bld, bl);
        else better(dl, C, bjd, bj);
    }
    wave_best(bjd, bj);
    wave_best(bld, bl);
    ncand = wave_sum_int(ncand);
    if (bad) atomicOr(&cx.ctr->error, LF_DEVERR_INEXACT);
    if (lane == 0) {
        cx.dj[j] = bj;
        cx.djd[j] = bj >= 0 ? bjd : 0.0;
        cx.dl[j] = bl;
        cx.dld[j] = bl >= 0 ? bld : 0.0;
        atomicAdd(&cx.ctr->visits, (unsigned long long)V);
        atomicAdd(&cx.ctr->cands, (unsigned long long)ncand);
    }
}

// Workgroup path for deferred nodes: the candidate table lives in dynamic LDS
// (`tab` entries); candidates are split by a hash into P partitions processed one after
// another, P doubling whenever a partition does not fit.  Persistent workgroups take
// deferred nodes until the list is exhausted.
__global__ void __launch_bounds__(256) k_eval_hub(Ctx cx, int cstart, int tab)
{
    extern __shared__ unsigned long long s_dyn[];
    unsigned long long *d0 = s_dyn, *d1 = s_dyn + tab, *d2 = s_dyn + 2 * tab, *d3 = s_dyn + 3 * tab;
    int *key = (int *)(s_dyn + 4 * tab);
    int *kk = key + tab;
    __shared__ int s_item, s_fill, s_ovf;
    __shared__ double s_bd[2][256 / WAVE];
    __shared__ int s_bc[2][256 / WAVE];
    __shared__ int s_nc[256 / WAVE];
    int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    int lg = 31 - __clz(tab);
    int limit = (tab * 3) / 4;
    int count = __atomic_load_n(&cx.ctr->hub_count, __ATOMIC_RELAXED);
    while (true) {
        if (threadIdx.x == 0) s_item = atomicAdd(&cx.ctr->hub_next, 1);
        __syncthreads();
        int item = s_item;
        __syncthreads();
        if (item >= count) break;
        int j = cx.hub_list[item];
        int x = cx.order[cstart + j];
        NodeHdr hx = cx.nh[x];
        long long rb = cx.rowptr[x], re = cx.rowptr[x + 1];
        long long dx = hx.deg;
        int P = 1;
        double bjd = 0.0, bld = 0.0;
        int bj = -1, bl = -1;
        int bad = 0;
        long long nvis = 0, ncand = 0;
        for (int p = 0; p < P; p++) {
            for (int t = threadIdx.x; t < tab; t += blockDim.x) {
                key[t] = -1; kk[t] = 0; d0[t] = 0; d1[t] = 0; d2[t] = 0; d3[t] = 0;
            }
            if (threadIdx.x == 0) { s_fill = 0; s_ovf = 0; }
            __syncthreads();
            // own communities of this partition
            for (int a = threadIdx.x; a < hx.cnt; a += blockDim.x) {
                int c = cx.slot[hx.off + a].comm;
                if ((int)(hash_part(c) & (unsigned)(P - 1)) != p) continue;
                unsigned hsh = hash_tab(c) >> (32 - lg);
                while (true) {
                    int cur = key[hsh];
                    if (cur == c) break;
                    if (cur == -1) {
                        if (atomicAdd(&s_fill, 1) >= limit) { s_ovf = 1; break; }
                        int old = atomicCAS(&key[hsh], -1, c);
                        if (old == -1 || old == c) break;
                    }
                    hsh = (hsh + 1) & (tab - 1);
                }
            }
            __syncthreads();
            for (long long e = rb + threadIdx.x; e < re; e += blockDim.x) {
                int y = cx.col[e];
                NodeHdr hy = cx.nh[y];
                for (int t = 0; t < hy.cnt; t++) {
                    Slot sl = cx.slot[hy.off + t];
                    int C = sl.comm;
                    if ((int)(hash_part(C) & (unsigned)(P - 1)) != p) continue;
                    nvis++;
                    unsigned hsh = hash_tab(C) >> (32 - lg);
                    bool ok = true;
                    while (true) {
                        int cur = key[hsh];
                        if (cur == C) break;
                        if (cur == -1) {
                            if (atomicAdd(&s_fill, 1) >= limit) { s_ovf = 1; ok = false; break; }
                            int old = atomicCAS(&key[hsh], -1, C);
                            if (old == -1 || old == C) break;
                        }
                        hsh = (hsh + 1) & (tab - 1);
                    }
                    if (!ok) break;
                    long long s = cx.cs[C];
                    bool leave = find_slot(cx.slot, hx.off, hx.cnt, C) >= 0;
                    X192 term = visit_term(leave, sl.in, hy.deg, s, bad);
                    i64 t0, t1, t2, t3;
                    x192_digits(term, t0, t1, t2, t3);
                    atomicAdd(&kk[hsh], 1);
                    atomicAdd(&d0[hsh], (unsigned long long)t0);
                    atomicAdd(&d1[hsh], (unsigned long long)t1);
                    atomicAdd(&d2[hsh], (unsigned long long)t2);
                    atomicAdd(&d3[hsh], (unsigned long long)t3);
                }
            }
            __syncthreads();
            if (s_ovf) {
                // partition too large: restart with twice as many partitions
                if (P >= (1 << 20)) {
                    // cannot happen for distinct 32-bit ids (the partition hash is nearly
                    // injective); stop with an error instead of looping
                    if (threadIdx.x == 0) atomicOr(&cx.ctr->error, LF_DEVERR_SLOTS);
                    break;
                }
                P *= 2;
                p = -1;
                bjd = bld = 0.0;
                bj = bl = -1;
                nvis = 0;
                ncand = 0;
                __syncthreads();
                continue;
            }
            for (int t = threadIdx.x; t < tab; t += blockDim.x) {
                int C = key[t];
                if (C < 0) continue;
                ncand++;
                int k = kk[t];
                int a = find_slot(cx.slot, hx.off, hx.cnt, C);
                bool leave = a >= 0;
                if (leave && cx.slot[hx.off + a].in != k) atomicOr(&cx.ctr->error, LF_DEVERR_INCOUNT);
                X192 corr = x192_from_digits((i64)d0[t], (i64)d1[t], (i64)d2[t], (i64)d3[t]);
                double dl = candidate_delta(cx, C, leave, k, dx, corr, bad);
                if (leave) better(dl, C, bld, bl);
                else better(dl, C, bjd, bj);
            }
            __syncthreads();
        }
        // block argmax
        wave_best(bjd, bj);
        wave_best(bld, bl);
        int nc = wave_sum_int((int)ncand);
        int nv = wave_sum_int((int)nvis);
        if (lane == 0) {
            s_bd[0][wv] = bjd; s_bc[0][wv] = bj;
            s_bd[1][wv] = bld; s_bc[1][wv] = bl;
            s_nc[wv] = nc;
        }
        if (lane == 0 && nv) atomicAdd(&cx.ctr->visits, (unsigned long long)nv);
        __syncthreads();
        if (threadIdx.x == 0) {
            double jd = s_bd[0][0], ld = s_bd[1][0];
            int jc = s_bc[0][0], lc = s_bc[1][0];
            int tc = s_nc[0];
            for (int w = 1; w < nw; w++) {
                double od = s_bd[0][w]; int oc = s_bc[0][w];
                if (oc >= 0 && (jc < 0 || od > jd || (od == jd && oc < jc))) { jd = od; jc = oc; }
                od = s_bd[1][w]; oc = s_bc[1][w];
                if (oc >= 0 && (lc < 0 || od > ld || (od == ld && oc < lc))) { ld = od; lc = oc; }
                tc += s_nc[w];
            }
            cx.dj[j] = jc;
            cx.djd[j] = jc >= 0 ? jd : 0.0;
            cx.dl[j] = lc;
            cx.dld[j] = lc >= 0 ? ld : 0.0;
            atomicAdd(&cx.ctr->cands, (unsigned long long)tc);
        }
        if (bad) atomicOr(&cx.ctr->error, LF_DEVERR_INEXACT);
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------
// A5: bulk apply
// ------------------------------------------------------------------------------------
__device__ __forceinline__ void touch(const Ctx &cx, int C)
{
    if (atomicExch(&cx.tflag[C], 1) == 0) cx.tlist[atomicAdd(&cx.ctr->tcount, 1)] = C;
}

// membership edits and sizes; one thread per queued node
__global__ void k_apply_edit(Ctx cx, int cstart, int clen)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= clen) return;
    int J = cx.dj[j], L = cx.dl[j];
    if (J < 0 && L < 0) return;
    int x = cx.order[cstart + j];
    NodeHdr hx = cx.nh[x];
    int cnt = hx.cnt;
    if (L >= 0) {
        int t = find_slot(cx.slot, hx.off, cnt, L);
        cx.slot[hx.off + t] = cx.slot[hx.off + cnt - 1];
        cnt--;
        atomicSub(&cx.cs[L], 1);
        touch(cx, L);
        atomicAdd(&cx.ctr->leaves, 1ull);
    }
    if (J >= 0) {
        long long capx = cx.nh[x + 1].off - hx.off;
        if (cnt >= capx) {
            atomicOr(&cx.ctr->error, LF_DEVERR_SLOTS);
        } else {
            Slot sn = {J, 0};
            cx.slot[hx.off + cnt] = sn;
            cnt++;
            atomicAdd(&cx.cs[J], 1);
            touch(cx, J);
            cx.joined_to[x] = J;
            int p = atomicAdd(&cx.cm_len[J], 1);
            long long cap = cx.cm_off[J + 1] - cx.cm_off[J];
            if (p < cap) {
                cx.cm_node[cx.cm_off[J] + p] = x;
            } else {
                int e = atomicAdd(&cx.ctr->ovf_cnt, 1);
                cx.ovf_node[e] = x;
                cx.ovf_comm[e] = J;
                cx.ovf_flag[J] = 1;
            }
            atomicAdd(&cx.ctr->joins, 1ull);
        }
    }
    cx.nh[x].cnt = cnt;
}

// in-counts: a surviving member y of J (L) gains (loses) one per neighbour that joined
// (left); a node that joined J in this queue gets its in-count counted afresh.  One wave
// per queued node that moved.
__global__ void __launch_bounds__(256) k_apply_in(Ctx cx, int cstart, int clen)
{
    int j = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    int lane = threadIdx.x & (WAVE - 1);
    if (j >= clen) return;
    int J = cx.dj[j], L = cx.dl[j];
    if (J < 0 && L < 0) return;
    int x = cx.order[cstart + j];
    if (J >= 0 && cx.joined_to[x] != J) J = -1;     // join did not fit (error flagged)
    long long rb = cx.rowptr[x], re = cx.rowptr[x + 1];
    int fresh = 0;
    for (long long e = rb + lane; e < re; e += WAVE) {
        int y = cx.col[e];
        NodeHdr hy = cx.nh[y];
        int jy = cx.joined_to[y];
        for (int t = 0; t < hy.cnt; t++) {
            int c = cx.slot[hy.off + t].comm;
            if (c == J && J >= 0) {
                fresh++;
                if (jy != J) atomicAdd(&cx.slot[hy.off + t].in, 1);
            } else if (c == L && L >= 0) {
                if (jy != L) atomicSub(&cx.slot[hy.off + t].in, 1);
            }
        }
    }
    fresh = wave_sum_int(fresh);
    if (lane == 0 && J >= 0) {
        NodeHdr hx = cx.nh[x];
        cx.slot[hx.off + hx.cnt - 1].in = fresh;
    }
}

// ------------------------------------------------------------------------------------
// A6: iteration end
// ------------------------------------------------------------------------------------
// communities with fewer than two members are removed: mark them (tflag = 2), zero their
// statistics, count the live ones
__global__ void k_mark_dead(Ctx cx)
{
    long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (c >= cx.K) return;
    int s = cx.cs[c];
    if (s < 2) {
        if (s == 1) cx.tflag[c] = 2;
        cx.cs[c] = 0;
        cx.cm[c] = 0;
        cx.cW[c] = 0.0;
        cx.cSp[c] = x192_zero();
        cx.cSm[c] = x192_zero();
    } else {
        atomicAdd(&cx.ctr->live, 1);
    }
    cx.cm_len[c] = 0;
    cx.ovf_flag[c] = 0;
}

// drop removed communities from every node's slots; next capacity = count + 1
__global__ void k_drop_dead(Ctx cx, long long *newcap)
{
    long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (x >= cx.n) return;
    NodeHdr hx = cx.nh[x];
    int w = 0;
    for (int t = 0; t < hx.cnt; t++) {
        Slot sl = cx.slot[hx.off + t];
        if (cx.tflag[sl.comm] == 2) continue;
        cx.slot[hx.off + w] = sl;
        w++;
    }
    cx.nh[x].cnt = w;
    newcap[x] = w + 1;
    atomicMax(&cx.ctr->max_mem, w);
}

__global__ void k_clear_dead(Ctx cx)
{
    long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (c >= cx.K) return;
    cx.tflag[c] = 0;
}

__global__ void k_copy_slots(Ctx cx, const long long *noff, Slot *dst, long long total)
{
    long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (x > cx.n) return;
    if (x == cx.n) { cx.nh[x].off = total; return; }
    NodeHdr hx = cx.nh[x];
    long long o = noff[x];
    for (int t = 0; t < hx.cnt; t++) dst[o + t] = cx.slot[hx.off + t];
    Slot e = {-1, 0};
    dst[o + hx.cnt] = e;
    cx.nh[x].off = o;
}

// exact partition score: per-block X256 partials, folded by one wave
__global__ void __launch_bounds__(256) k_score_partials(const double *cW, int K, X256 *part, int *err)
{
    __shared__ X256 s_w[256 / WAVE];
    X256 acc = x256_zero();
    int bad = 0;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < K; c += (long long)gridDim.x * blockDim.x) {
        X256 v = x256_from_double(cW[c], bad);
        x256_add(acc, v);
    }
    acc = wave_sum_x256(acc);
    int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    if (lane == 0) s_w[wv] = acc;
    if (bad) atomicOr(err, LF_DEVERR_INEXACT);
    __syncthreads();
    if (threadIdx.x == 0) {
        X256 s = s_w[0];
        for (int k = 1; k < 256 / WAVE; k++) x256_add(s, s_w[k]);
        part[blockIdx.x] = s;
    }
}

__global__ void k_score_fold(const X256 *part, int np, double *out)
{
    X256 acc = x256_zero();
    for (int k = threadIdx.x; k < np; k += WAVE) x256_add(acc, part[k]);
    acc = wave_sum_x256(acc);
    if (threadIdx.x == 0) out[0] = x256_round(acc);
}

// ------------------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------------------
Ctx lf_ctx(lf_handle *h)
{
    Ctx c;
    c.n = h->n;
    c.K = h->K;
    c.rowptr = h->rowptr;
    c.col = h->col;
    c.deg = h->deg;
    c.order = h->order;
    c.nh = h->nh;
    c.slot = h->slot[h->cur];
    c.cs = h->cs;
    c.cm = h->cm;
    c.cW = h->cW;
    c.cSp = h->cSp;
    c.cSm = h->cSm;
    c.cm_off = h->cm_off;
    c.cm_len = h->cm_len;
    c.cm_node = h->cm_node;
    c.tflag = h->tflag;
    c.tlist = h->tlist;
    c.joined_to = h->joined_to;
    c.ovf_node = h->ovf_node;
    c.ovf_comm = h->ovf_comm;
    c.ovf_flag = h->ovf_flag;
    c.dj = h->dj;
    c.dl = h->dl;
    c.djd = h->djd;
    c.dld = h->dld;
    c.hub_list = h->hub_list;
    c.ctr = h->ctr;
    return c;
}

void lf_free_partition(lf_handle *h)
{
    void **ptrs[] = {(void **)&h->nh, (void **)&h->slot[0], (void **)&h->slot[1], (void **)&h->cs,
                     (void **)&h->cm, (void **)&h->cW, (void **)&h->cSp, (void **)&h->cSm,
                     (void **)&h->cm_off, (void **)&h->cm_len, (void **)&h->cm_node, (void **)&h->tflag,
                     (void **)&h->tlist, (void **)&h->joined_to, (void **)&h->ovf_node,
                     (void **)&h->ovf_comm, (void **)&h->ovf_flag, (void **)&h->dj, (void **)&h->dl,
                     (void **)&h->djd, (void **)&h->dld, (void **)&h->hub_list, (void **)&h->ctr};
    for (void **p : ptrs) {
        lf_dev_free(h, *p);
        *p = nullptr;
    }
    h->K = 0;
    h->slot_capb[0] = h->slot_capb[1] = 0;
    h->cm_cap = 0;
    h->q_cap = 0;
}

// member lists with capacity for joiners; requires sizes and slots to be current
static int rebuild_member_lists(lf_handle *h)
{
    hipStream_t st = h->stream;
    const int BS = 256;
    long long n = h->n;
    int K = h->K;
    long long *capx = nullptr;
    LF_TRY(lf_dev_alloc(h, (void **)&capx, sizeof(long long) * (K + 1)));
    LF_HIP(h, hipMemsetAsync(capx, 0, sizeof(long long) * (K + 1), st));
    Ctx cx = lf_ctx(h);
    if (n > 0) hipLaunchKernelGGL(k_member_extra, dim3(grid_for(n, BS)), dim3(BS), 0, st, h->nh, cx.slot, n, capx);
    if (K > 0) hipLaunchKernelGGL(k_member_cap, dim3(grid_for(K, BS)), dim3(BS), 0, st, capx, h->cs, K, n);
    LF_TRY(lf_exclusive_scan_i64(h, capx, h->cm_off, K + 1));
    long long total = 0;
    LF_HIP(h, hipMemcpyAsync(&total, h->cm_off + K, sizeof(long long), hipMemcpyDeviceToHost, st));
    LF_HIP(h, hipStreamSynchronize(st));
    if (total > h->cm_cap) {
        lf_dev_free(h, h->cm_node);
        h->cm_node = nullptr;
        long long want = total + total / 8 + 1024;
        LF_TRY(lf_dev_alloc(h, (void **)&h->cm_node, sizeof(int) * want));
        h->cm_cap = want;
        cx = lf_ctx(h);
    }
    LF_HIP(h, hipMemsetAsync(h->cm_len, 0, sizeof(int) * (K > 0 ? K : 1), st));
    if (n > 0) hipLaunchKernelGGL(k_member_fill, dim3(grid_for(n, BS)), dim3(BS), 0, st, h->nh, cx.slot, n, h->cm_off, h->cm_len, h->cm_node);
    LF_HIP(h, hipGetLastError());
    LF_HIP(h, hipStreamSynchronize(st));
    lf_dev_free(h, capx);
    return LF_OK;
}

static int partition_score(lf_handle *h, double *out)
{
    hipStream_t st = h->stream;
    int K = h->K;
    int nb = (int)((K + 255) / 256);
    if (nb > 1024) nb = 1024;
    if (nb < 1) nb = 1;
    X256 *part = nullptr;
    double *dw = nullptr;
    LF_TRY(lf_dev_alloc(h, (void **)&part, sizeof(X256) * nb));
    LF_TRY(lf_dev_alloc(h, (void **)&dw, sizeof(double)));
    hipLaunchKernelGGL(k_score_partials, dim3(nb), dim3(256), 0, st, h->cW, K, part, &h->ctr->error);
    hipLaunchKernelGGL(k_score_fold, dim3(1), dim3(WAVE), 0, st, part, nb, dw);
    LF_HIP(h, hipMemcpyAsync(out, dw, sizeof(double), hipMemcpyDeviceToHost, st));
    LF_HIP(h, hipStreamSynchronize(st));
    LF_HIP(h, hipGetLastError());
    lf_dev_free(h, part);
    lf_dev_free(h, dw);
    return LF_OK;
}

static int check_dev_error(lf_handle *h)
{
    int e = 0;
    LF_HIP(h, hipMemcpyAsync(&e, &h->ctr->error, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    LF_HIP(h, hipStreamSynchronize(h->stream));
    if (e & LF_DEVERR_INEXACT) return lf_set_error(h, LF_EOVERFLOW, "a score term left the exact accumulator's range");
    if (e & LF_DEVERR_SLOTS) return lf_set_error(h, LF_EINTERNAL, "membership slot capacity exceeded");
    if (e & LF_DEVERR_INCOUNT) return lf_set_error(h, LF_EINTERNAL, "in-count bookkeeping inconsistent");
    if (e & LF_DEVERR_ODD) return lf_set_error(h, LF_EINTERNAL, "odd internal degree sum");
    return LF_OK;
}

int lf_initial_clustering(lf_handle *h)
{
    hipStream_t st = h->stream;
    const int BS = 256;
    long long n = h->n;
    lf_free_partition(h);
    LF_TRY(lf_dev_alloc(h, (void **)&h->ctr, sizeof(DevCounters)));
    LF_HIP(h, hipMemsetAsync(h->ctr, 0, sizeof(DevCounters), st));
    LF_TRY(lf_prof_begin(h));
    int *state = nullptr, *cursor = nullptr, *comm_of = nullptr, *flag = nullptr, *und = nullptr;
    long long *pos = nullptr;
    size_t nn = (size_t)(n > 0 ? n : 1);
    LF_TRY(lf_dev_alloc(h, (void **)&state, sizeof(int) * nn));
    LF_TRY(lf_dev_alloc(h, (void **)&cursor, sizeof(int) * nn));
    LF_TRY(lf_dev_alloc(h, (void **)&comm_of, sizeof(int) * nn));
    LF_TRY(lf_dev_alloc(h, (void **)&flag, sizeof(int) * nn));
    LF_TRY(lf_dev_alloc(h, (void **)&pos, sizeof(long long) * (nn + 1)));
    const int RB = 8;   // rounds between host checks
    LF_TRY(lf_dev_alloc(h, (void **)&und, sizeof(int) * RB));
    LF_HIP(h, hipMemsetAsync(state, 0, sizeof(int) * nn, st));
    LF_HIP(h, hipMemsetAsync(cursor, 0, sizeof(int) * nn, st));
    int rounds = 0;
    unsigned gr = grid_for(n, BS);
    if (gr > 8192) gr = 8192;
    while (n > 0) {
        LF_HIP(h, hipMemsetAsync(und, 0, sizeof(int) * RB, st));
        for (int r = 0; r < RB; r++)
            hipLaunchKernelGGL(k_lfmis_round, dim3(gr), dim3(BS), 0, st, h->rowptr, h->col, h->rank, n, state,
                               cursor, und + r);
        rounds += RB;
        int hu[RB];
        LF_HIP(h, hipMemcpyAsync(hu, und, sizeof(int) * RB, hipMemcpyDeviceToHost, st));
        LF_HIP(h, hipStreamSynchronize(st));
        if (hu[RB - 1] == 0) break;
        if (rounds > 64 * (n + 8)) return lf_set_error(h, LF_EINTERNAL, "initial clustering did not converge");
    }
    if (n > 0) {
        hipLaunchKernelGGL(k_opener_flags, dim3(grid_for(n, BS)), dim3(BS), 0, st, h->order, state, n, flag);
    }
    LF_TRY(lf_exclusive_scan_i32_to_i64(h, flag, pos, n));
    long long lastp = 0;
    int lastf = 0;
    if (n > 0) {
        hipLaunchKernelGGL(k_opener_ids, dim3(grid_for(n, BS)), dim3(BS), 0, st, h->order, flag, pos, n, comm_of);
        hipLaunchKernelGGL(k_join_openers, dim3(grid_for(n * WAVE, BS)), dim3(BS), 0, st, h->rowptr, h->col, h->rank,
                           state, n, comm_of);
        LF_HIP(h, hipMemcpyAsync(&lastp, pos + n - 1, sizeof(long long), hipMemcpyDeviceToHost, st));
        LF_HIP(h, hipMemcpyAsync(&lastf, flag + n - 1, sizeof(int), hipMemcpyDeviceToHost, st));
    }
    LF_HIP(h, hipStreamSynchronize(st));
    LF_HIP(h, hipGetLastError());
    long long K = lastp + lastf;
    if (K >= (1ll << 31) - 1) return lf_set_error(h, LF_EOVERFLOW, "too many communities");
    h->K = (int)K;
    size_t KK = (size_t)(K > 0 ? K : 1);
    // partition state
    LF_TRY(lf_dev_alloc(h, (void **)&h->nh, sizeof(NodeHdr) * (nn + 1)));
    h->slot_capb[0] = h->slot_capb[1] = 2 * (n > 0 ? n : 1);
    LF_TRY(lf_dev_alloc(h, (void **)&h->slot[0], sizeof(Slot) * h->slot_capb[0]));
    LF_TRY(lf_dev_alloc(h, (void **)&h->slot[1], sizeof(Slot) * h->slot_capb[1]));
    h->cur = 0;
    LF_TRY(lf_dev_alloc(h, (void **)&h->cs, sizeof(int) * KK));
    LF_TRY(lf_dev_alloc(h, (void **)&h->cm, sizeof(long long) * KK));
    LF_TRY(lf_dev_alloc(h, (void **)&h->cW, sizeof(double) * KK));
    LF_TRY(lf_dev_alloc(h, (void **)&h->cSp, sizeof(X192) * KK));
    LF_TRY(lf_dev_alloc(h, (void **)&h->cSm, sizeof(X192) * KK));
    LF_TRY(lf_dev_alloc(h, (void **)&h->cm_off, sizeof(long long) * (KK + 1)));
    LF_TRY(lf_dev_alloc(h, (void **)&h->cm_len, sizeof(int) * KK));
    LF_TRY(lf_dev_alloc(h, (void **)&h->tflag, sizeof(int) * KK));
    LF_TRY(lf_dev_alloc(h, (void **)&h->tlist, sizeof(int) * KK));
    LF_TRY(lf_dev_alloc(h, (void **)&h->ovf_flag, sizeof(int) * KK));
    LF_TRY(lf_dev_alloc(h, (void **)&h->joined_to, sizeof(int) * nn));
    LF_TRY(lf_dev_alloc(h, (void **)&h->ovf_node, sizeof(int) * nn));
    LF_TRY(lf_dev_alloc(h, (void **)&h->ovf_comm, sizeof(int) * nn));
    LF_HIP(h, hipMemsetAsync(h->cs, 0, sizeof(int) * KK, st));
    LF_HIP(h, hipMemsetAsync(h->tflag, 0, sizeof(int) * KK, st));
    LF_HIP(h, hipMemsetAsync(h->ovf_flag, 0, sizeof(int) * KK, st));
    LF_HIP(h, hipMemsetAsync(h->joined_to, 0xff, sizeof(int) * nn, st));
    if (n >= 0)
        hipLaunchKernelGGL(k_init_slots, dim3(grid_for((n + 1) * WAVE, BS)), dim3(BS), 0, st, h->rowptr, h->col,
                           h->deg, comm_of, n, h->nh, h->slot[0], h->cs);
    LF_TRY(rebuild_member_lists(h));
    // every community's statistics
    if (K > 0) hipLaunchKernelGGL(k_iota, dim3(grid_for(K, BS)), dim3(BS), 0, st, h->tlist, K);
    LF_HIP(h, hipMemsetAsync(&h->ctr->refresh_next, 0, sizeof(int), st));
    Ctx cx = lf_ctx(h);
    int rb = (int)((K + 3) / 4);
    if (rb > 4096) rb = 4096;
    if (rb < 1) rb = 1;
    hipLaunchKernelGGL(k_refresh, dim3(rb), dim3(256), 0, st, cx, (int)K);
    LF_HIP(h, hipGetLastError());
    LF_TRY(partition_score(h, &h->Wt));
    LF_TRY(lf_prof_end(h, LF_K_INITCLUST, rounds + 8));
    LF_TRY(check_dev_error(h));
    lf_dev_free(h, state);
    lf_dev_free(h, cursor);
    lf_dev_free(h, comm_of);
    lf_dev_free(h, flag);
    lf_dev_free(h, pos);
    lf_dev_free(h, und);
    return LF_OK;
}

static int ensure_queue_buffers(lf_handle *h, long long q)
{
    if (q <= h->q_cap) return LF_OK;
    void **ptrs[] = {(void **)&h->dj, (void **)&h->dl, (void **)&h->djd, (void **)&h->dld, (void **)&h->hub_list};
    for (void **p : ptrs) {
        lf_dev_free(h, *p);
        *p = nullptr;
    }
    LF_TRY(lf_dev_alloc(h, (void **)&h->dj, sizeof(int) * q));
    LF_TRY(lf_dev_alloc(h, (void **)&h->dl, sizeof(int) * q));
    LF_TRY(lf_dev_alloc(h, (void **)&h->djd, sizeof(double) * q));
    LF_TRY(lf_dev_alloc(h, (void **)&h->dld, sizeof(double) * q));
    LF_TRY(lf_dev_alloc(h, (void **)&h->hub_list, sizeof(int) * q));
    h->q_cap = q;
    return LF_OK;
}

static int iteration_end(lf_handle *h, int last_start, int last_len, long long *joins, long long *leaves,
                         long long *live)
{
    hipStream_t st = h->stream;
    const int BS = 256;
    long long n = h->n;
    int K = h->K;
    Ctx cx = lf_ctx(h);
    hipLaunchKernelGGL(k_chunk_begin, dim3(grid_for(last_len > 0 ? last_len : 1, BS)), dim3(BS), 0, st, cx,
                       last_start, last_len);
    LF_HIP(h, hipMemsetAsync(&h->ctr->live, 0, sizeof(int) * 2, st));   // live, max_mem
    LF_HIP(h, hipMemsetAsync(&h->ctr->ovf_cnt, 0, sizeof(int), st));
    if (K > 0) hipLaunchKernelGGL(k_mark_dead, dim3(grid_for(K, BS)), dim3(BS), 0, st, cx);
    long long *newcap = nullptr, *noff = nullptr;
    LF_TRY(lf_dev_alloc(h, (void **)&newcap, sizeof(long long) * (n + 1)));
    LF_TRY(lf_dev_alloc(h, (void **)&noff, sizeof(long long) * (n + 1)));
    if (n > 0) hipLaunchKernelGGL(k_drop_dead, dim3(grid_for(n, BS)), dim3(BS), 0, st, cx, newcap);
    if (K > 0) hipLaunchKernelGGL(k_clear_dead, dim3(grid_for(K, BS)), dim3(BS), 0, st, cx);
    LF_HIP(h, hipMemsetAsync(newcap + n, 0, sizeof(long long), st));
    LF_TRY(lf_exclusive_scan_i64(h, newcap, noff, n + 1));
    long long total = 0;
    LF_HIP(h, hipMemcpyAsync(&total, noff + n, sizeof(long long), hipMemcpyDeviceToHost, st));
    LF_HIP(h, hipStreamSynchronize(st));
    int other = 1 - h->cur;
    if (total > h->slot_capb[other]) {
        long long want = total + total / 4 + 1024;
        lf_dev_free(h, h->slot[other]);
        h->slot[other] = nullptr;
        LF_TRY(lf_dev_alloc(h, (void **)&h->slot[other], sizeof(Slot) * want));
        h->slot_capb[other] = want;
    }
    hipLaunchKernelGGL(k_copy_slots, dim3(grid_for(n + 1, BS)), dim3(BS), 0, st, cx, noff, h->slot[other], total);
    h->cur = other;
    LF_TRY(rebuild_member_lists(h));
    LF_TRY(partition_score(h, &h->Wt));
    unsigned long long jl[2] = {0, 0};
    int lv[2] = {0, 0};
    LF_HIP(h, hipMemcpyAsync(jl, &h->ctr->joins, sizeof(jl), hipMemcpyDeviceToHost, st));
    LF_HIP(h, hipMemcpyAsync(lv, &h->ctr->live, sizeof(lv), hipMemcpyDeviceToHost, st));
    LF_HIP(h, hipStreamSynchronize(st));
    LF_HIP(h, hipGetLastError());
    lf_dev_free(h, newcap);
    lf_dev_free(h, noff);
    *joins = (long long)jl[0];
    *leaves = (long long)jl[1];
    *live = lv[0];
    return LF_OK;
}

int lf_iterate(lf_handle *h, int q, double theta, int max_iters, lf_run_info *out)
{
    hipStream_t st = h->stream;
    const int BS = 256;
    long long n = h->n;
    lf_run_info dummy;
    memset(&dummy, 0, sizeof dummy);
    if (!out) out = &dummy;
    out->iterations = 0;
    out->converged = 0;
    out->hit_max = 0;
    if (out->wtilde_hist) out->wtilde_hist[0] = h->Wt;
    if (h->cc == 0.0) {
        out->converged = 1;
        out->wtilde = h->Wt;
        out->wcc_hat = 0.0;
        return LF_OK;
    }
    long long qq = q < n ? q : (n > 0 ? n : 1);
    LF_TRY(ensure_queue_buffers(h, qq));
    int maxdev = 0;
    LF_HIP(h, hipDeviceGetAttribute(&maxdev, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device));
    int tab = h->hub_lds_entries;
    while (tab > 64 && (size_t)tab * 40 + 2048 > (size_t)maxdev) tab >>= 1;
    size_t hub_shmem = (size_t)tab * 40;
    LF_HIP(h, hipFuncSetAttribute((const void *)k_eval_hub, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)hub_shmem));
    double prev = h->Wt;
    for (int it = 0; it < max_iters; it++) {
        LF_HIP(h, hipMemsetAsync(&h->ctr->joins, 0, sizeof(unsigned long long) * 2, st));
        int prev_start = 0, prev_len = 0;
        for (long long start = 0; start < n; start += q) {
            int clen = (int)((n - start) < q ? (n - start) : q);
            int cstart = (int)start;
            Ctx cx = lf_ctx(h);
            hipLaunchKernelGGL(k_chunk_begin, dim3(grid_for(prev_len > 0 ? prev_len : 1, BS)), dim3(BS), 0, st, cx,
                               prev_start, prev_len);
            LF_TRY(lf_prof_begin(h));
            hipLaunchKernelGGL(k_eval, dim3(grid_for(clen, EW)), dim3(EW * WAVE), 0, st, cx, cstart, clen);
            LF_TRY(lf_prof_end(h, LF_K_EVAL, 1));
            LF_TRY(lf_prof_begin(h));
            int hb = h->hub_blocks < clen ? h->hub_blocks : clen;
            hipLaunchKernelGGL(k_eval_hub, dim3(hb), dim3(256), hub_shmem, st, cx, cstart, tab);
            LF_TRY(lf_prof_end(h, LF_K_EVAL_HUB, 1));
            LF_TRY(lf_prof_begin(h));
            hipLaunchKernelGGL(k_apply_edit, dim3(grid_for(clen, BS)), dim3(BS), 0, st, cx, cstart, clen);
            hipLaunchKernelGGL(k_apply_in, dim3(grid_for((long long)clen * WAVE, BS)), dim3(BS), 0, st, cx, cstart, clen);
            int rbk = h->refresh_blocks;
            long long need = (2ll * clen + 3) / 4;
            if (need < rbk) rbk = (int)(need > 0 ? need : 1);
            hipLaunchKernelGGL(k_refresh, dim3(rbk), dim3(256), 0, st, cx, -1);
            LF_TRY(lf_prof_end(h, LF_K_APPLY, 3));
            if (h->profiling) {
                h->prof.chunks++;
                h->prof.node_evals += clen;
            }
            prev_start = cstart;
            prev_len = clen;
        }
        LF_HIP(h, hipGetLastError());
        LF_TRY(lf_prof_begin(h));
        long long joins = 0, leaves = 0, live = 0;
        LF_TRY(iteration_end(h, prev_start, prev_len, &joins, &leaves, &live));
        LF_TRY(lf_prof_end(h, LF_K_ITEREND, 8));
        LF_TRY(check_dev_error(h));
        out->iterations = it + 1;
        if (out->wtilde_hist) out->wtilde_hist[it + 1] = h->Wt;
        if (out->joins) out->joins[it] = joins;
        if (out->leaves) out->leaves[it] = leaves;
        if (out->communities) out->communities[it] = live;
        bool stop = (prev == 0.0) || ((h->Wt - prev) / prev < theta);
        prev = h->Wt;
        if (stop) {
            out->converged = 1;
            break;
        }
    }
    if (!out->converged && out->iterations == max_iters) out->hit_max = 1;
    if (h->profiling) {
        unsigned long long vc[2];
        LF_HIP(h, hipMemcpy(vc, &h->ctr->visits, sizeof(vc), hipMemcpyDeviceToHost));
        h->prof.visits = (long long)vc[0];
        h->prof.candidates = (long long)vc[1];
    }
    out->wtilde = h->Wt;
    out->wcc_hat = h->Wt / h->cc;
    return LF_OK;
}

// memberships (sorted per node) and in-counts, copied to host buffers
int lf_fetch_memberships(lf_handle *h, long long *offsets, int *comm_ids, long long capacity,
                         long long *total, int *in_counts)
{
    hipStream_t st = h->stream;
    long long n = h->n;
    std::vector<NodeHdr> hn((size_t)n + 1);
    LF_HIP(h, hipMemcpyAsync(hn.data(), h->nh, sizeof(NodeHdr) * (n + 1), hipMemcpyDeviceToHost, st));
    LF_HIP(h, hipStreamSynchronize(st));
    long long tot = 0;
    for (long long x = 0; x < n; x++) tot += hn[x].cnt;
    *total = tot;
    if (!offsets || (!comm_ids && !in_counts)) return LF_OK;
    if (capacity < tot) return lf_set_error(h, LF_ERANGE, "capacity %lld < %lld memberships", capacity, tot);
    std::vector<Slot> hs((size_t)hn[n].off + 1);
    LF_HIP(h, hipMemcpyAsync(hs.data(), h->slot[h->cur], sizeof(Slot) * hn[n].off, hipMemcpyDeviceToHost, st));
    LF_HIP(h, hipStreamSynchronize(st));
    long long p = 0;
    std::vector<Slot> tmp;
    for (long long x = 0; x < n; x++) {
        offsets[x] = p;
        tmp.assign(hs.begin() + hn[x].off, hs.begin() + hn[x].off + hn[x].cnt);
        // ascending community id (insertion sort: a handful of entries per node)
        for (size_t a = 1; a < tmp.size(); a++) {
            Slot v = tmp[a];
            size_t b = a;
            while (b > 0 && tmp[b - 1].comm > v.comm) { tmp[b] = tmp[b - 1]; b--; }
            tmp[b] = v;
        }
        for (const Slot &s : tmp) {
            if (comm_ids) comm_ids[p] = s.comm;
            if (in_counts) in_counts[p] = s.in;
            p++;
        }
    }
    offsets[n] = p;
    return LF_OK;
}
