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
#include "method.h"

static inline unsigned grid_for(long long n, int block) { return (unsigned)((n + block - 1) / block); }
static inline unsigned min_u(unsigned a, unsigned b) { return a < b ? a : b; }

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
                                                    CommRec *cr)
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
        atomicAdd(&cr[c].s, 1);
    }
}

// warm start: checks of a given cover (waves stride over the nodes): offsets non-decreasing
// within [0, total] (bit 0), ids in [0, K) (bit 1; K < 0: any id >= 0), no id twice per
// node (bit 2); chk[1] = largest id.  One atomic per wave at the end: a single hot
// counter updated per node would serialise millions of atomics.
__global__ void __launch_bounds__(256) k_cover_check(const long long *off, const int *ids, long long n,
                                                     long long total, int K, int *chk)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const long long nw = (long long)gridDim.x * (blockDim.x / WAVE);
    int err = 0, mx = -1;
    for (long long x = (blockIdx.x * (long long)blockDim.x + threadIdx.x) / WAVE; x < n; x += nw) {
        const long long a0 = off[x], a1 = off[x + 1];
        if (a0 < 0 || a1 < a0 || a1 > total) {
            err |= 1;
            continue;
        }
        for (long long a = a0 + lane; a < a1; a += WAVE) {
            const int c = ids[a];
            if (c < 0 || (K >= 0 && c >= K)) err |= 2;
            if (c > mx) mx = c;
            for (long long b = a0; b < a; b++) err |= ids[b] == c ? 4 : 0;
        }
    }
    for (int o = 32; o >= 1; o >>= 1) {
        err |= __shfl_xor(err, o, WAVE);
        const int om = __shfl_xor(mx, o, WAVE);
        mx = om > mx ? om : mx;
    }
    if (lane == 0) {
        if (err) atomicOr(&chk[0], err);
        if (mx >= 0) atomicMax(&chk[1], mx);
    }
}

// warm start: node x's memberships in the given order plus one free slot (slot offset
// off[x] + x); in-count of each = neighbours whose cover lists the community; sizes.
// One wave per node; a pass over the neighbours' lists counts up to COVER_CHUNK of x's
// communities at once (a node's ids are distinct, so each neighbour adds at most one to
// each count), so a node with few memberships gathers its neighbourhood once.
#define COVER_CHUNK 8
__global__ void __launch_bounds__(256) k_cover_slots(const long long *rowptr, const int *col, const int *deg,
                                                     const long long *off, const int *ids, long long n, NodeHdr *nh,
                                                     Slot *slot, CommRec *cr)
{
    long long x = (blockIdx.x * (long long)blockDim.x + threadIdx.x) / WAVE;
    int lane = threadIdx.x & (WAVE - 1);
    if (x > n) return;
    if (x == n) {
        if (lane == 0) { nh[n].off = off[n] + n; nh[n].cnt = 0; nh[n].deg = 0; }
        return;
    }
    const long long a0 = off[x];
    const int cnt = (int)(off[x + 1] - a0);
    const long long base = a0 + x;
    const long long e0 = rowptr[x], e1 = rowptr[x + 1];
    for (int a = 0; a < cnt; a += COVER_CHUNK) {
        const int m = cnt - a < COVER_CHUNK ? cnt - a : COVER_CHUNK;   // uniform over the wave
        int c[COVER_CHUNK], in[COVER_CHUNK];
#pragma unroll
        for (int k = 0; k < COVER_CHUNK; k++) {
            c[k] = k < m ? ids[a0 + a + k] : -1;   // ids are >= 0: -1 matches nothing
            in[k] = 0;
        }
        for (long long e = e0 + lane; e < e1; e += WAVE) {
            const int z = col[e];
            const long long b1 = off[z + 1];
            for (long long b = off[z]; b < b1; b++) {
                const int d = ids[b];
#pragma unroll
                for (int k = 0; k < COVER_CHUNK; k++) in[k] += d == c[k];
            }
        }
#pragma unroll
        for (int k = 0; k < COVER_CHUNK; k++) {
            if (k < m) {
                const int t = wave_sum_int(in[k]);
                if (lane == 0) {
                    Slot sl = {c[k], t};
                    slot[base + a + k] = sl;
                    atomicAdd(&cr[c[k]].s, 1);
                }
            }
        }
    }
    if (lane == 0) {
        NodeHdr hd;
        hd.off = base;
        hd.cnt = cnt;
        hd.deg = deg[x];
        nh[x] = hd;
        Slot free_slot = {-1, 0};
        slot[base + cnt] = free_slot;
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

__global__ void k_member_cap(long long *capx, const CommRec *cr, int K, long long n)
{
    long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (c >= K) return;
    long long ex = capx[c];
    if (ex > n) ex = n;
    capx[c] = cr[c].s + ex;
}

__global__ void k_member_fill(const NodeHdr *nh, const Slot *slot, long long n, int K, const long long *cm_off,
                              int *cm_len, int *cm_node, long long cap)
{
    long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (x >= n || cm_off[K] > cap) return;          // over capacity: the host grows it and refills
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
// exact re-sum of touched communities (persistent: each wave takes REFRESH_CHUNK
// consecutive entries of the touched list at a time until it is exhausted; one returning
// atomic per community on the shared counter would serialise the launch)
// ------------------------------------------------------------------------------------
#define REFRESH_CHUNK 16
__global__ void __launch_bounds__(256) k_refresh_list(Ctx cx, int fixed_count)
{
    int lane = threadIdx.x & (WAVE - 1);
    int count = fixed_count >= 0 ? fixed_count : __atomic_load_n(&cx.ctr->tcount, __ATOMIC_RELAXED);
    int bad = 0;
    // unsigned: the last grabs may pass 2^31 when the list nears the int range
    unsigned idx = 0, end = 0;
    while (true) {
        if (idx == end) {
            if (lane == 0) idx = atomicAdd((unsigned *)&cx.ctr->refresh_next, (unsigned)REFRESH_CHUNK);
            idx = __shfl(idx, 0, WAVE);
            end = idx + REFRESH_CHUNK;
        }
        if (idx >= (unsigned)count) break;
        int C = cx.tlist[idx++];
        long long s = cx.cr[C].s;
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
        if (lane == 0) store_comm(cx, C, s, a0, ap, am, sumi, bad);
    }
    if (bad) atomicOr(&cx.ctr->error, LF_DEVERR_INEXACT);
}

// ------------------------------------------------------------------------------------
// A6: iteration end
// ------------------------------------------------------------------------------------
// The iteration-end kernels fold their shared counters per block (a grid of at most
// END_BLOCKS blocks striding over the range): one atomic per wave on a single address
// would serialise the launch (about 15 ns each).
#define END_BLOCKS 2048

__device__ __forceinline__ int block_fold_int(int v, bool take_max)
{
    __shared__ int s_part[256 / WAVE];
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        const int t = __shfl_xor(v, o, WAVE);
        v = take_max ? (t > v ? t : v) : v + t;
    }
    if ((threadIdx.x & (WAVE - 1)) == 0) s_part[threadIdx.x / WAVE] = v;
    __syncthreads();
    v = s_part[0];
    for (int w = 1; w < (int)blockDim.x / WAVE; w++) v = take_max ? (s_part[w] > v ? s_part[w] : v) : v + s_part[w];
    return v;
}

// communities with fewer than two members are removed: mark them (tflag = 2), zero their
// statistics, count the live ones
__global__ void __launch_bounds__(256) k_mark_dead(Ctx cx)
{
    int live = 0;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < cx.K;
         c += (long long)gridDim.x * blockDim.x) {
        CommRec *r = &cx.cr[c];
        int s = r->s;
        if (s < 2) {
            if (s == 1) cx.tflag[c] = 2;
            r->s = 0;
            r->m = 0;
            r->W = 0.0;
            for (int k = 0; k < 5; k++) { r->Sp[k] = 0; r->Sm[k] = 0; }
        } else {
            live++;
        }
        cx.cm_len[c] = 0;
        cx.ovf_flag[c] = 0;
    }
    live = block_fold_int(live, false);
    if (threadIdx.x == 0 && live) atomicAdd(&cx.ctr->live, live);
}

// drop removed communities from every node's slots (four slots and their flags per round
// trip; a kept slot moves only to a position already read); next capacity = count + 1
__global__ void __launch_bounds__(256) k_drop_dead(Ctx cx, long long *newcap)
{
    int mx = 0;
    for (long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x; x < cx.n;
         x += (long long)gridDim.x * blockDim.x) {
        NodeHdr hx = cx.nh[x];
        Slot *xs = cx.slot + hx.off;
        int w = 0;
        for (int t0 = 0; t0 < hx.cnt; t0 += 4) {
            Slot sl[4];
            bool keep[4];
#pragma unroll
            for (int q = 0; q < 4; q++)
                if (t0 + q < hx.cnt) sl[q] = xs[t0 + q];
#pragma unroll
            for (int q = 0; q < 4; q++) keep[q] = t0 + q < hx.cnt && cx.tflag[sl[q].comm] != 2;
#pragma unroll
            for (int q = 0; q < 4; q++)
                if (keep[q]) xs[w++] = sl[q];
        }
        cx.nh[x].cnt = w;
        newcap[x] = w + 1;
        mx = w > mx ? w : mx;
    }
    mx = block_fold_int(mx, true);
    if (threadIdx.x == 0) atomicMax(&cx.ctr->max_mem, mx);
}

__global__ void k_clear_dead(Ctx cx)
{
    long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (c >= cx.K) return;
    cx.tflag[c] = 0;
}

__global__ void k_copy_slots(Ctx cx, const long long *noff, Slot *dst)
{
    long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (x > cx.n) return;
    if (x == cx.n) { cx.nh[x].off = noff[x]; return; }
    NodeHdr hx = cx.nh[x];
    long long o = noff[x];
    for (int t = 0; t < hx.cnt; t++) dst[o + t] = cx.slot[hx.off + t];
    Slot e = {-1, 0};
    dst[o + hx.cnt] = e;
    cx.nh[x].off = o;
}

// exact partition score: per-block X256 partials, folded by one wave
__global__ void __launch_bounds__(256) k_score_partials(const CommRec *cr, int K, X256 *part, int *err)
{
    __shared__ X256 s_w[256 / WAVE];
    X256 acc = x256_zero();
    int bad = 0;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < K; c += (long long)gridDim.x * blockDim.x) {
        X256 v = x256_from_double(cr[c].W, bad);
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

// everything an iteration end reports to the host, gathered into one record
#define REP_SLOTS 0
#define REP_MEMBERS 1
#define REP_SCORE 2
#define REP_JOINS 3
#define REP_LEAVES 4
#define REP_LIVE 5
#define REP_ERROR 6
__global__ void k_end_report(const DevCounters *c, const long long *slots, const long long *members,
                             const double *score, long long *rep)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    rep[REP_SLOTS] = *slots;
    rep[REP_MEMBERS] = *members;
    rep[REP_SCORE] = __double_as_longlong(*score);
    rep[REP_JOINS] = (long long)c->joins;
    rep[REP_LEAVES] = (long long)c->leaves;
    rep[REP_LIVE] = c->live;
    rep[REP_ERROR] = c->error;
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
    memset(&c, 0, sizeof c);   // padding too: the bytes of a Ctx key captured graphs
    c.n = h->n;
    c.K = h->K;
    c.rowptr = h->rowptr;
    c.col = h->col;
    c.deg = h->deg;
    c.order = h->order;
    c.nh = h->nh;
    c.slot = h->slot[h->cur];
    c.ln = h->lines;
    c.cr = h->cr;
    c.cm_off = h->cm_off;
    c.cm_len = h->cm_len;
    c.cm_node = h->cm_node;
    c.tflag = h->tflag;
    c.tlist = h->tlist;
    c.ovf_node = h->ovf_node;
    c.ovf_comm = h->ovf_comm;
    c.ovf_flag = h->ovf_flag;
    c.dj = h->dj;
    c.dl = h->dl;
    c.djd = h->djd;
    c.dld = h->dld;
    c.dpos = h->dpos;
    c.ctr = h->ctr;
    c.big_idx = h->big_idx;
    for (int k = 0; k < LF_PATH_COUNT; k++) {
        c.plist[k] = h->plist[k];
        c.prec[k] = h->prec[k];
    }
    c.rank = h->rank;
    c.col_rank = h->col_rank;
    c.titem_base = h->titem_base;
    c.titem_node = h->titem_node;
    c.big_bj = h->big_bj;
    c.big_bl = h->big_bl;
    c.big_cj = h->big_cj;
    c.big_cl = h->big_cl;
    c.big_ln = h->big_ln;
    c.gt = h->gt;
    c.occ = h->occ;
    c.occ_key = h->occ_key;
    c.occ_d = h->occ_d;
    c.gmask = h->gT > 0 ? h->gT - 1 : 0;
    c.unit = h->unit;
    c.part_rec = h->part_rec;
    c.part_done = h->part_done;
    c.macc = h->macc;
    c.part_cap = (int)h->part_cap;
    c.mslot_cap = (int)h->mslot_cap;
    c.stats = (h->profiling >> LF_PROF_COUNTERS_BIT) & 1;
    return c;
}

void lf_free_partition(lf_handle *h)
{
    void **ptrs[] = {(void **)&h->nh, (void **)&h->slot[0], (void **)&h->slot[1], (void **)&h->lines, (void **)&h->cr,
                     (void **)&h->cm_off, (void **)&h->cm_len, (void **)&h->cm_node, (void **)&h->tflag,
                     (void **)&h->tlist, (void **)&h->ovf_node,
                     (void **)&h->ovf_comm, (void **)&h->ovf_flag, (void **)&h->ctr,
                     (void **)&h->part_done, (void **)&h->vbound,
                     (void **)&h->cls, (void **)&h->cscan, (void **)&h->plist[0], (void **)&h->plist[1],
                     (void **)&h->plist[2], (void **)&h->plist[3], (void **)&h->prec_all, (void **)&h->pbase};
    for (void **p : ptrs) {
        lf_dev_free(h, *p);
        *p = nullptr;
    }
    h->K = 0;
    h->slot_capb[0] = h->slot_capb[1] = 0;
    h->cm_cap = 0;
    lf_free_iteration_buffers(h);
    h->graph_version++;
}

// member lists with capacity for joiners; requires sizes and slots to be current.  Queued
// on the stream without waiting: if the lists outgrow cm_node nothing is written, and the
// total (cm_off[K]) tells the host to grow it and call this again.
static int rebuild_member_lists_async(lf_handle *h)
{
    TmpScope tmp_scope(h);
    hipStream_t st = h->stream;
    const int BS = 256;
    long long n = h->n;
    int K = h->K;
    long long *capx = nullptr;
    LF_TRY(lf_tmp_alloc(h, (void **)&capx, sizeof(long long) * (K + 1)));
    LF_TRY(lf_zero(h, capx, sizeof(long long) * (K + 1)));
    Ctx cx = lf_ctx(h);
    if (n > 0) hipLaunchKernelGGL(k_member_extra, dim3(grid_for(n, BS)), dim3(BS), 0, st, h->nh, cx.slot, n, capx);
    if (K > 0) hipLaunchKernelGGL(k_member_cap, dim3(grid_for(K, BS)), dim3(BS), 0, st, capx, h->cr, K, n);
    LF_TRY(lf_exclusive_scan_i64(h, capx, h->cm_off, K + 1));
    if (!h->cm_node) {
        long long want = 2 * n + 1024;
        LF_TRY(lf_dev_alloc(h, (void **)&h->cm_node, sizeof(int) * want));
        h->cm_cap = want;
    }
    LF_TRY(lf_zero(h, h->cm_len, sizeof(int) * (K > 0 ? K : 1)));
    if (n > 0)
        hipLaunchKernelGGL(k_member_fill, dim3(grid_for(n, BS)), dim3(BS), 0, st, h->nh, cx.slot, n, K, h->cm_off,
                           h->cm_len, h->cm_node, h->cm_cap);
    LF_HIP(h, hipGetLastError());
    return LF_OK;
}

// grow cm_node to hold `total` member entries and fill the lists again (waits)
static int grow_member_lists(lf_handle *h, long long total)
{
    if (!h->phase_graphs) LF_HIP(h, hipStreamSynchronize(h->stream));   // a batch member keeps the old list
    lf_dev_free(h, h->cm_node);
    h->cm_node = nullptr;
    // grown two-fold (four-fold for a batch member, whose captured iteration starts and
    // ends a moved buffer invalidates), so a growing cover reallocates only a few times
    long long want = (h->phase_graphs ? 4 : 2) * total + 1024;
    LF_TRY(lf_dev_alloc(h, (void **)&h->cm_node, sizeof(int) * want));
    h->cm_cap = want;
    return rebuild_member_lists_async(h);
}

static int rebuild_member_lists(lf_handle *h)
{
    LF_TRY(rebuild_member_lists_async(h));
    long long total = 0;
    LF_HIP(h, hipMemcpyAsync(&total, h->cm_off + h->K, sizeof(long long), hipMemcpyDeviceToHost, h->stream));
    LF_HIP(h, hipStreamSynchronize(h->stream));
    if (total > h->cm_cap) LF_TRY(grow_member_lists(h, total));
    LF_HIP(h, hipStreamSynchronize(h->stream));
    return LF_OK;
}

// exact partition score into the device double *dw (queued, no wait)
static int partition_score_async(lf_handle *h, double *dw)
{
    TmpScope tmp_scope(h);
    hipStream_t st = h->stream;
    int K = h->K;
    int nb = (int)((K + 255) / 256);
    if (nb > 1024) nb = 1024;
    if (nb < 1) nb = 1;
    X256 *part = nullptr;
    LF_TRY(lf_tmp_alloc(h, (void **)&part, sizeof(X256) * nb));
    hipLaunchKernelGGL(k_score_partials, dim3(nb), dim3(256), 0, st, h->cr, K, part, &h->ctr->error);
    hipLaunchKernelGGL(k_score_fold, dim3(1), dim3(WAVE), 0, st, part, nb, dw);
    LF_HIP(h, hipGetLastError());
    return LF_OK;
}

static int partition_score(lf_handle *h, double *out)
{
    TmpScope tmp_scope(h);
    double *dw = nullptr;
    LF_TRY(lf_tmp_alloc(h, (void **)&dw, sizeof(double)));
    LF_TRY(partition_score_async(h, dw));
    LF_HIP(h, hipMemcpyAsync(out, dw, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    LF_HIP(h, hipStreamSynchronize(h->stream));
    LF_HIP(h, hipGetLastError());
    return LF_OK;
}

int lf_check_dev_error(lf_handle *h)
{
    int e = 0;
    LF_HIP(h, hipMemcpyAsync(&e, &h->ctr->error, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    LF_HIP(h, hipStreamSynchronize(h->stream));
    return lf_dev_error_status(h, e);
}

int lf_dev_error_status(lf_handle *h, int e)
{
    if (e & LF_DEVERR_INEXACT) return lf_set_error(h, LF_EOVERFLOW, "a score term left the exact accumulator's range");
    if (e & LF_DEVERR_SLOTS) return lf_set_error(h, LF_EINTERNAL, "membership slot capacity exceeded");
    if (e & LF_DEVERR_INCOUNT) return lf_set_error(h, LF_EINTERNAL, "in-count bookkeeping inconsistent");
    if (e & LF_DEVERR_ODD) return lf_set_error(h, LF_EINTERNAL, "odd internal degree sum");
    if (e & LF_DEVERR_CAP) return lf_set_error(h, LF_EINTERNAL, "a per-queue work buffer was too small");
    return LF_OK;
}

static int alloc_partition_state(lf_handle *h, long long K, long long slots);
static int finish_partition(lf_handle *h);

int lf_initial_clustering(lf_handle *h)
{
    TmpScope tmp_scope(h);
    hipStream_t st = h->stream;
    const int BS = 256;
    long long n = h->n;
    lf_free_partition(h);
    LF_TRY(lf_dev_alloc(h, (void **)&h->ctr, sizeof(DevCounters)));
    LF_HIP(h, hipMemsetAsync(h->ctr, 0, sizeof(DevCounters), st));
    LF_TRY(lf_prof_begin(h, LF_K_INITCLUST));
    int *state = nullptr, *cursor = nullptr, *comm_of = nullptr, *flag = nullptr, *und = nullptr;
    long long *pos = nullptr;
    size_t nn = (size_t)(n > 0 ? n : 1);
    LF_TRY(lf_tmp_alloc(h, (void **)&state, sizeof(int) * nn));
    LF_TRY(lf_tmp_alloc(h, (void **)&cursor, sizeof(int) * nn));
    LF_TRY(lf_tmp_alloc(h, (void **)&comm_of, sizeof(int) * nn));
    LF_TRY(lf_tmp_alloc(h, (void **)&flag, sizeof(int) * nn));
    LF_TRY(lf_tmp_alloc(h, (void **)&pos, sizeof(long long) * (nn + 1)));
    const int RB = 8;   // rounds between host checks
    LF_TRY(lf_tmp_alloc(h, (void **)&und, sizeof(int) * RB));
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
    LF_TRY(alloc_partition_state(h, K, 2 * n));
    if (n >= 0)
        hipLaunchKernelGGL(k_init_slots, dim3(grid_for((n + 1) * WAVE, BS)), dim3(BS), 0, st, h->rowptr, h->col,
                           h->deg, comm_of, n, h->nh, h->slot[0], h->cr);
    LF_TRY(finish_partition(h));
    LF_TRY(lf_prof_end(h, LF_K_INITCLUST, rounds + 8));
    LF_TRY(lf_prof_flush(h));
    LF_TRY(lf_check_dev_error(h));
    return LF_OK;
}

// Partition arrays for K community ids and slot storage for `slots` memberships (at least
// one); community records zeroed, no member lists yet.
static int alloc_partition_state(lf_handle *h, long long K, long long slots)
{
    hipStream_t st = h->stream;
    long long n = h->n;
    size_t nn = (size_t)(n > 0 ? n : 1);
    h->K = (int)K;
    size_t KK = (size_t)(K > 0 ? K : 1);
    LF_TRY(lf_dev_alloc(h, (void **)&h->nh, sizeof(NodeHdr) * (nn + 1)));
    h->slot_capb[0] = h->slot_capb[1] = slots > 0 ? slots : 1;
    h->slot_used = slots;
    LF_TRY(lf_dev_alloc(h, (void **)&h->slot[0], sizeof(Slot) * h->slot_capb[0]));
    LF_TRY(lf_dev_alloc(h, (void **)&h->slot[1], sizeof(Slot) * h->slot_capb[1]));
    h->cur = 0;
    LF_TRY(lf_dev_alloc(h, (void **)&h->cr, sizeof(CommRec) * KK));
    LF_TRY(lf_dev_alloc(h, (void **)&h->cm_off, sizeof(long long) * (KK + 1)));
    LF_TRY(lf_dev_alloc(h, (void **)&h->cm_len, sizeof(int) * KK));
    LF_TRY(lf_dev_alloc(h, (void **)&h->tflag, sizeof(int) * KK));
    LF_TRY(lf_dev_alloc(h, (void **)&h->tlist, sizeof(int) * KK));
    LF_TRY(lf_dev_alloc(h, (void **)&h->ovf_flag, sizeof(int) * KK));
    LF_TRY(lf_dev_alloc(h, (void **)&h->part_done, sizeof(int) * KK));
    LF_TRY(lf_dev_alloc(h, (void **)&h->vbound, sizeof(long long) * (nn + 1)));
    LF_TRY(lf_dev_alloc(h, (void **)&h->cls, sizeof(int) * nn));
    LF_TRY(lf_dev_alloc(h, (void **)&h->cscan, sizeof(long long) * (nn + 1)));
    for (int k = 0; k < LF_PATH_COUNT; k++) LF_TRY(lf_dev_alloc(h, (void **)&h->plist[k], sizeof(int) * nn));
    LF_TRY(lf_dev_alloc(h, (void **)&h->prec_all, sizeof(NodeRec) * nn));
    LF_TRY(lf_dev_alloc(h, (void **)&h->pbase, sizeof(long long) * (LF_PATH_COUNT + 1)));
    for (int k = 0; k < LF_PATH_COUNT; k++) h->prec[k] = h->prec_all;
    LF_TRY(lf_dev_alloc(h, (void **)&h->ovf_node, sizeof(int) * nn));
    LF_TRY(lf_dev_alloc(h, (void **)&h->ovf_comm, sizeof(int) * nn));
    LF_HIP(h, hipMemsetAsync(h->cr, 0, sizeof(CommRec) * KK, st));
    LF_HIP(h, hipMemsetAsync(h->tflag, 0, sizeof(int) * KK, st));
    LF_HIP(h, hipMemsetAsync(h->ovf_flag, 0, sizeof(int) * KK, st));
    h->qtag = 0;
    return LF_OK;
}

// With slots, headers and community sizes written: member lists, every community's
// statistics (internal edges, exact sums, score) and the partition score.
static int finish_partition(lf_handle *h)
{
    hipStream_t st = h->stream;
    const int BS = 256;
    const long long K = h->K;
    LF_TRY(rebuild_member_lists(h));
    if (K > 0) hipLaunchKernelGGL(k_iota, dim3(grid_for(K, BS)), dim3(BS), 0, st, h->tlist, K);
    LF_HIP(h, hipMemsetAsync(&h->ctr->refresh_next, 0, sizeof(int), st));
    Ctx cx = lf_ctx(h);
    int rb = (int)((K + 3) / 4);
    if (rb > 4096) rb = 4096;
    if (rb < 1) rb = 1;
    hipLaunchKernelGGL(k_refresh_list, dim3(rb), dim3(256), 0, st, cx, (int)K);
    LF_HIP(h, hipGetLastError());
    LF_TRY(partition_score(h, &h->Wt));
    return LF_OK;
}

// Warm start from an existing cover (Initial Clustering, last paragraph: an existing
// division can replace the greedy one).  off[n + 1] / ids[total] on the device, each
// node's communities in any order.  Node statistics must exist.
// Checks of a cover on the device (offsets, ids in [0, n_comms) or >= 0 if n_comms < 0, no
// id twice per node); *maxid = the largest id (-1 if none).
int lf_check_cover(lf_handle *h, const long long *off, const int *ids, long long total, int n_comms, int *maxid)
{
    TmpScope tmp_scope(h);
    hipStream_t st = h->stream;
    const int BS = 256;
    const long long n = h->n;
    long long ends[2] = {0, 0};
    LF_HIP(h, hipMemcpyAsync(&ends[0], off, sizeof(long long), hipMemcpyDeviceToHost, st));
    LF_HIP(h, hipMemcpyAsync(&ends[1], off + n, sizeof(long long), hipMemcpyDeviceToHost, st));
    LF_HIP(h, hipStreamSynchronize(st));
    if (ends[0] != 0 || ends[1] != total)
        return lf_set_error(h, LF_EINVAL, "cover offsets must start at 0 and end at total (%lld)", total);
    int *chk = nullptr;                      // [0] error bits, [1] largest id
    LF_TRY(lf_tmp_alloc(h, (void **)&chk, 2 * sizeof(int)));
    const int init[2] = {0, -1};
    LF_HIP(h, hipMemcpyAsync(chk, init, sizeof init, hipMemcpyHostToDevice, st));
    unsigned gc = grid_for(n * WAVE, BS);
    if (gc > 2048) gc = 2048;
    if (n > 0) hipLaunchKernelGGL(k_cover_check, dim3(gc), dim3(BS), 0, st, off, ids, n, total, n_comms, chk);
    int hc[2];
    LF_HIP(h, hipMemcpyAsync(hc, chk, sizeof hc, hipMemcpyDeviceToHost, st));
    LF_HIP(h, hipStreamSynchronize(st));
    LF_HIP(h, hipGetLastError());
    if (hc[0] & 1) return lf_set_error(h, LF_EINVAL, "cover offsets decrease or leave [0, total]");
    if (hc[0] & 2) return lf_set_error(h, LF_EINVAL, "a community id is negative or not below n_comms");
    if (hc[0] & 4) return lf_set_error(h, LF_EINVAL, "a node lists a community twice");
    *maxid = hc[1];
    return LF_OK;
}

int lf_partition_from_cover(lf_handle *h, const long long *off, const int *ids, long long total, int n_comms)
{
    TmpScope tmp_scope(h);
    hipStream_t st = h->stream;
    const int BS = 256;
    const long long n = h->n;
    int maxid = -1;
    LF_TRY(lf_check_cover(h, off, ids, total, n_comms, &maxid));
    const long long K = n_comms >= 0 ? n_comms : (long long)maxid + 1;
    if (K >= (1ll << 31) - 1) return lf_set_error(h, LF_EOVERFLOW, "too many communities");
    h->state = 1;                            // the previous partition is gone from here on
    lf_free_partition(h);
    LF_TRY(lf_dev_alloc(h, (void **)&h->ctr, sizeof(DevCounters)));
    LF_HIP(h, hipMemsetAsync(h->ctr, 0, sizeof(DevCounters), st));
    LF_TRY(lf_prof_begin(h, LF_K_INITCLUST));
    LF_TRY(alloc_partition_state(h, K, total + n));
    hipLaunchKernelGGL(k_cover_slots, dim3(grid_for((n + 1) * WAVE, BS)), dim3(BS), 0, st, h->rowptr, h->col,
                       h->deg, off, ids, n, h->nh, h->slot[0], h->cr);
    LF_TRY(finish_partition(h));
    LF_TRY(lf_prof_end(h, LF_K_INITCLUST, 8));
    LF_TRY(lf_prof_flush(h));
    LF_TRY(lf_check_dev_error(h));
    h->state = 2;
    return LF_OK;
}

// Iteration end, first half (queued): degenerate communities removed, slots compacted,
// member lists rebuilt, score reduced, and one report copied to pinned host memory.
int lf_iteration_end_enqueue(lf_handle *h)
{
    TmpScope tmp_scope(h);
    hipStream_t st = h->stream;
    const int BS = 256;
    long long n = h->n;
    int K = h->K;
    Ctx cx = lf_ctx(h);
    LF_TRY(lf_zero(h, &h->ctr->live, sizeof(int) * 2));   // live, max_mem
    LF_TRY(lf_zero(h, &h->ctr->ovf_cnt, sizeof(int)));
    if (K > 0) hipLaunchKernelGGL(k_mark_dead, dim3(min_u(grid_for(K, BS), END_BLOCKS)), dim3(BS), 0, st, cx);
    long long *newcap = nullptr, *noff = nullptr;
    LF_TRY(lf_tmp_alloc(h, (void **)&newcap, sizeof(long long) * (n + 1)));
    LF_TRY(lf_tmp_alloc(h, (void **)&noff, sizeof(long long) * (n + 1)));
    if (n > 0)
        hipLaunchKernelGGL(k_drop_dead, dim3(min_u(grid_for(n, BS), END_BLOCKS)), dim3(BS), 0, st, cx, newcap);
    if (K > 0) hipLaunchKernelGGL(k_clear_dead, dim3(grid_for(K, BS)), dim3(BS), 0, st, cx);
    LF_TRY(lf_zero(h, newcap + n, sizeof(long long)));
    LF_TRY(lf_exclusive_scan_i64(h, newcap, noff, n + 1));
    // the new layout holds at most the current one's entries plus one per node (a node's
    // count grows only into its free slot), so the copy needs no wait for its size
    int other = 1 - h->cur;
    const long long bound = h->slot_used + n + 1;
    if (bound > h->slot_capb[other]) {
        long long want = (h->phase_graphs ? 3 * bound : bound + bound / 2) + 1024;
        lf_dev_free(h, h->slot[other]);
        h->slot[other] = nullptr;
        LF_TRY(lf_dev_alloc(h, (void **)&h->slot[other], sizeof(Slot) * want));
        h->slot_capb[other] = want;
    }
    hipLaunchKernelGGL(k_copy_slots, dim3(grid_for(n + 1, BS)), dim3(BS), 0, st, cx, noff, h->slot[other]);
    h->cur = other;
    LF_TRY(rebuild_member_lists_async(h));
    double *dw = nullptr;
    LF_TRY(lf_tmp_alloc(h, (void **)&dw, sizeof(double)));
    LF_TRY(partition_score_async(h, dw));
    // the host's one wait of the iteration end: every value it needs in one pinned record
    long long *drep = nullptr;
    LF_TRY(lf_tmp_alloc(h, (void **)&drep, sizeof(long long) * 16));
    hipLaunchKernelGGL(k_end_report, dim3(1), dim3(1), 0, st, (const DevCounters *)h->ctr, noff + n,
                       (const long long *)h->cm_off + K, (const double *)dw, drep);
    LF_HIP(h, hipMemcpyAsync(h->hrep, drep, sizeof(long long) * 16, hipMemcpyDeviceToHost, st));
    LF_HIP(h, hipGetLastError());
    return LF_OK;
}

// second half: read the report (the caller has waited for it), grow the member lists if
// they did not fit
int lf_iteration_end_complete(lf_handle *h, long long *joins, long long *leaves, long long *live)
{
    hipStream_t st = h->stream;
    const long long *r = h->hrep;
    h->slot_used = r[REP_SLOTS];
    if (r[REP_MEMBERS] > h->cm_cap) {        // rare: member lists outgrew their buffer
        LF_TRY(grow_member_lists(h, r[REP_MEMBERS]));
        if (!h->phase_graphs) LF_HIP(h, hipStreamSynchronize(st));
    }
    double wt;
    memcpy(&wt, &r[REP_SCORE], sizeof wt);
    h->Wt = wt;
    unsigned long long jl[2] = {(unsigned long long)r[REP_JOINS], (unsigned long long)r[REP_LEAVES]};
    int lv[2] = {(int)r[REP_LIVE], 0};
    h->last_dev_error = (int)r[REP_ERROR];
    *joins = (long long)jl[0];
    *leaves = (long long)jl[1];
    *live = lv[0];
    return LF_OK;
}

// memberships (community ids ascending per node) and in-counts, gathered on the device
__global__ void k_member_counts(const NodeHdr *nh, long long n, long long *cnt)
{
    long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (x < n) cnt[x] = nh[x].cnt;
    if (x == n) cnt[n] = 0;
}

__global__ void k_member_out(const NodeHdr *nh, const Slot *slot, long long n, const long long *off,
                             int *ids, int *in)
{
    long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (x >= n) return;
    NodeHdr hx = nh[x];
    long long o = off[x];
    // insertion sort of a handful of entries, directly in the output range
    for (int t = 0; t < hx.cnt; t++) {
        Slot v = slot[hx.off + t];
        int b = t;
        while (b > 0 && ids[o + b - 1] > v.comm) {
            ids[o + b] = ids[o + b - 1];
            in[o + b] = in[o + b - 1];
            b--;
        }
        ids[o + b] = v.comm;
        in[o + b] = v.in;
    }
}

int lf_fetch_memberships(lf_handle *h, long long *offsets, int *comm_ids, long long capacity,
                         long long *total, int *in_counts)
{
    TmpScope tmp_scope(h);
    hipStream_t st = h->stream;
    const int BS = 256;
    long long n = h->n;
    long long *cnt = nullptr, *doff = nullptr;
    LF_TRY(lf_tmp_alloc(h, (void **)&cnt, sizeof(long long) * (n + 1)));
    LF_TRY(lf_tmp_alloc(h, (void **)&doff, sizeof(long long) * (n + 1)));
    hipLaunchKernelGGL(k_member_counts, dim3(grid_for(n + 1, BS)), dim3(BS), 0, st, h->nh, n, cnt);
    LF_TRY(lf_exclusive_scan_i64(h, cnt, doff, n + 1));
    long long tot = 0;
    LF_HIP(h, hipMemcpyAsync(&tot, doff + n, sizeof(long long), hipMemcpyDeviceToHost, st));
    LF_HIP(h, hipStreamSynchronize(st));
    *total = tot;
    int rc = LF_OK;
    if (offsets && (comm_ids || in_counts)) {
        if (capacity < tot) {
            rc = lf_set_error(h, LF_ERANGE, "capacity %lld < %lld memberships", capacity, tot);
        } else {
            int *dids = nullptr, *din = nullptr;
            LF_TRY(lf_tmp_alloc(h, (void **)&dids, sizeof(int) * (tot > 0 ? tot : 1)));
            LF_TRY(lf_tmp_alloc(h, (void **)&din, sizeof(int) * (tot > 0 ? tot : 1)));
            if (n > 0)
                hipLaunchKernelGGL(k_member_out, dim3(grid_for(n, BS)), dim3(BS), 0, st, h->nh, h->slot[h->cur], n,
                                   doff, dids, din);
            LF_HIP(h, hipMemcpyAsync(offsets, doff, sizeof(long long) * (n + 1), hipMemcpyDeviceToHost, st));
            if (comm_ids && tot > 0)
                LF_HIP(h, hipMemcpyAsync(comm_ids, dids, sizeof(int) * tot, hipMemcpyDeviceToHost, st));
            if (in_counts && tot > 0)
                LF_HIP(h, hipMemcpyAsync(in_counts, din, sizeof(int) * tot, hipMemcpyDeviceToHost, st));
            LF_HIP(h, hipStreamSynchronize(st));
            LF_HIP(h, hipGetLastError());
        }
    }
    return rc;
}
