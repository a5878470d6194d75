// iterate.hip -- one LazyFox iteration on the GPU: queues of q nodes in node order, each
// evaluated on the state at the start of the queue and then applied together
// (Methods, "Node Changes", Algorithm 2, "Stopping Criteria").
//
// At the start of an iteration every node is given an evaluation path from a bound on
// its visits that holds for the whole iteration (k_node_bounds), and each path gets the
// list of its nodes in order.  Per queue (all launches on the handle's stream, no host
// synchronisation):
//   k_eval           the small path (queues with >= 1024 such nodes): one wave per node
//                    with <= 64 visits; then the medium path: one 256-thread block per
//                    node with <= 256 visits, one visit per thread; each node decided
//                    entirely in an LDS hash table
//   k_eval_big       by block role: the table path's visits (largest nodes): every
//                    neighbour membership (y in C) adds its exact correction to the entry
//                    (node, C) of a global open-addressing table, own memberships add the
//                    leave candidates; the workgroup path (one workgroup per node with
//                    <= 1024 visits, LDS tables); the small path of smaller queues; in
//                    multi-graph steps also the medium path (one wave per node); block 0
//                    of either launch resets the queue's counters
//   k_big_final      every occupied table entry -> change of C's score; per node the
//                    largest positive change (atomicMax on the bits of a positive double)
//   k_big_tie        among the entries equal to that maximum the lowest community id
//   k_apply          the bulk apply: membership edits, sizes, member-list appends and
//                    re-sum planning (a thread per queued node) beside the in-count
//                    changes around the moved nodes (a wave per in-count unit)
//   k_refresh        exact re-sum per part; multi-part communities combine their parts
//                    through carry-save counters and the last part finalises
// k_queue_reset clears the queue counters at the start and the end of an iteration.
//
// Every sum is exact (fixed point), so none of the launch shapes above can change a bit
// of the result.
#include "method.h"

#define EW 4            // waves per block in the wave evaluation path
#define ECAP 128        // table entries per wave (power of two)
#define MXCAP 32        // own memberships kept in LDS (wave path)
#define INB 64          // neighbours per in-count unit (one per lane)
#define HOLE (-2)       // a membership left in the current iteration (removed at its end)
#define PART 128        // members per re-sum part
#define MACC 19         // carry-save counters per multi-part community (3 x 6 digits + in-sum)
#define GEMPTY (~0ull)

static inline unsigned grid_for(long long n, int block) { return (unsigned)((n + block - 1) / block); }

// reset the counters of a queue (at the start and the end of an iteration)
__global__ void k_queue_reset(Ctx cx)
{
    if (threadIdx.x == 0) {
        DevCounters *c = cx.ctr;
        c->occ_cnt = 0;
        c->parts_total = 0;
        c->mslots = 0;
    }
}

// ------------------------------------------------------------------------------------
// evaluation, wave path
// ------------------------------------------------------------------------------------
__device__ __forceinline__ int lds_insert(int *key, int T, int lg, int C)
{
    unsigned hsh = hash_tab(C) >> (32 - lg);
    while (true) {
        int old = atomicCAS(&key[hsh], -1, C);
        if (old == -1 || old == C) return (int)hsh;
        hsh = (hsh + 1) & (T - 1);
    }
}

// LDS of one node evaluation: a candidate hash table of 2*VCAP entries, per candidate
// (compact index, at most VCAP) its size and four correction digits, and per visit its
// degree, table entry and in-count.  The visit-slot list is only needed before the digits
// are cleared and shares their storage.  The last fields exchange values between the
// waves of a workgroup evaluation.
template <int VCAP>
struct NodeLds {
    int key[2 * VCAP];
    int kk[2 * VCAP];
    int ci[2 * VCAP];
    int sz[VCAP];
    int cl[VCAP];
    union {
        unsigned long long d[4][VCAP];
        long long vslot[VCAP];
    };
    int vdeg[VCAP];
    int vhash[VCAP];
    int vin[VCAP];
    int mx[MXCAP];
    int mxin[MXCAP];
    int wtot[4];
    int nc;
    double bjd[4], bld[4];
    int bj[4], bl[4];
};

// big_idx states of a queue index
#define Q_DONE 0        // decided by a wave or workgroup path
#define Q_TABLE 1       // decided by the table path
#define VSMALL 64       // visits of the small wave path
#define VMED 256        // visits of the medium wave path
#define VGRP 1024       // visits of the workgroup path
#define GT 256          // threads of the workgroup path
#define SMALL_OWN_LAUNCH 1024   // small-path nodes from which a queue launches k_eval

// member owning block b of a multi-graph launch (boff: first block of each member, nm + 1
// entries); -1 past the last member's blocks
__device__ __forceinline__ int find_member(const int *boff, int nm, int b)
{
    if (b >= boff[nm]) return -1;
    int lo = 0, hi = nm - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (boff[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// single-graph kernel K(Ctx, QStep) and multi-graph kernel K_multi over Member descriptors,
// both running BODY(cx, qs, block, blocks, lds)
#define QUEUE_KERNELS(K, BOUNDS, LDS_T, BODY)                                                 \
    __global__ void __launch_bounds__(BOUNDS) K(Ctx cx, QStep qs)                             \
    {                                                                                         \
        __shared__ LDS_T lds;                                                                 \
        BODY(cx, qs, (int)blockIdx.x, (int)gridDim.x, lds);                                   \
    }                                                                                         \
    __global__ void __launch_bounds__(BOUNDS) K##_multi(const Member *mem, const int *boff, int nm) \
    {                                                                                         \
        __shared__ LDS_T lds;                                                                 \
        const int m = find_member(boff, nm, (int)blockIdx.x);                                 \
        if (m < 0) return;                                                                    \
        BODY(mem[m].cx, mem[m].qs, (int)blockIdx.x - boff[m], boff[m + 1] - boff[m], lds);    \
    }

struct NoLds {
    int unused;
};

// barrier over the NT threads that evaluate one node (one wave or the whole workgroup)
template <int NT>
__device__ __forceinline__ void node_sync()
{
    if constexpr (NT == WAVE) WAVE_SYNC();
    else __syncthreads();
}

// inclusive prefix sum of v over the NT threads (wave shuffles, then the waves' totals
// through LDS); *total receives the sum over all NT threads
template <int NT, int VCAP>
__device__ __forceinline__ int node_incl_scan(int v, int tid, NodeLds<VCAP> &L, int *total)
{
    const int lane = tid & (WAVE - 1);
    int incl = v;
    for (int o = 1; o < WAVE; o <<= 1) {
        int t = __shfl_up(incl, o, WAVE);
        if (lane >= o) incl += t;
    }
    if constexpr (NT == WAVE) {
        *total = __shfl(incl, WAVE - 1, WAVE);
        return incl;
    } else {
        const int wv = tid / WAVE;
        if (lane == WAVE - 1) L.wtot[wv] = incl;
        __syncthreads();
        int off = 0, tot = 0;
        for (int w = 0; w < NT / WAVE; w++) {
            int t = L.wtot[w];
            if (w < wv) off += t;
            tot += t;
        }
        __syncthreads();
        *total = tot;
        return incl + off;
    }
}

// Evaluate queued node j with NT threads (one wave, or a workgroup of GT threads) if its
// neighbours (<= VCAP), visits and own memberships fit (2 * (visits + own) <= table,
// <= VCAP visits, <= MXCAP own).  Returns false (decision not written) otherwise; the
// decision to return is the same for all NT threads.  Every phase issues all of a
// thread's global gathers (at most VCAP / NT of them) before it uses any, so a node costs
// a handful of memory round trips whatever its size: own slots + column indices,
// neighbour headers, neighbour slots, and one record per candidate.
template <int NT, int VCAP>
__device__ __forceinline__ bool eval_node(const Ctx &cx, int j, const NodeRec nr, int tid, NodeLds<VCAP> &L,
                                          int wcap, int path)
{
    constexpr int NB = VCAP / NT;
    const int lane = tid & (WAVE - 1);
    const int x = nr.x, d = nr.d;
    const long long rb = nr.rb;
    if (d > VCAP) return false;
    // the adjacency gathers need only the node record; the header is fetched beside them
    int yv[NB];
#pragma unroll
    for (int b = 0; b < NB; b++) {
        int e = b * NT + tid;
        yv[b] = e < d ? cx.col[rb + e] : -1;
    }
    // own line: count, placement and (inline) memberships, read beside the adjacency
    const NodeLine *lxp = cx.ln + x;
    const int mcnt = lxp->cnt;
    const long long xoff = lxp->off;
    Slot own = {-1, 0};
    if (tid < LINE_SLOTS) own = lxp->s[tid];
    if (mcnt > MXCAP) return false;
    if (xoff >= 0) own = tid < mcnt ? cx.slot[xoff + tid] : Slot{-1, 0};
    else if (tid >= mcnt) own = Slot{-1, 0};
    // one line per neighbour: its count, degree and memberships in one gather
    NodeLine ly[NB];
#pragma unroll
    for (int b = 0; b < NB; b++) {
        if (yv[b] >= 0) {
            ly[b] = cx.ln[yv[b]];
        } else {
            ly[b].cnt = 0;
            ly[b].deg = 0;
            ly[b].off = -1;
        }
    }
    // neighbour memberships flattened into the visit list: an inline membership is kept
    // as its (community, in-count) pair, one in the slot array as the complement of its
    // slot index (read in phase 1)
    int V = 0;
#pragma unroll
    for (int b = 0; b < NB; b++) {
        if (b * NT < d) {                   // uniform over the NT threads
            int yc = ly[b].cnt, tot;
            int incl = node_incl_scan<NT>(yc, tid, L, &tot);
            int p0 = V + incl - yc;
            V += tot;
            if (V + mcnt > VCAP || 2 * (V + mcnt) > wcap) return false;   // uniform
            if (ly[b].off < 0) {
#pragma unroll
                for (int t = 0; t < LINE_SLOTS; t++)
                    if (t < yc) {
                        L.vslot[p0 + t] = ((long long)ly[b].s[t].in << 32) | (unsigned)ly[b].s[t].comm;
                        L.vdeg[p0 + t] = ly[b].deg;
                    }
            } else {
                for (int t = 0; t < yc; t++) {
                    L.vslot[p0 + t] = ~(ly[b].off + t);
                    L.vdeg[p0 + t] = ly[b].deg;
                }
            }
        }
    }
    int T = 8;
    while (T < 2 * (V + mcnt)) T <<= 1;
    const int lg = 31 - __clz(T);
    for (int t = tid; t < T; t += NT) {
        L.key[t] = -1;
        L.kk[t] = 0;
    }
    if (tid < mcnt) {
        L.mx[tid] = own.comm;
        L.mxin[tid] = own.in;
    }
    if (tid == 0) L.nc = 0;
    node_sync<NT>();
    // 1. candidates and neighbour counts: own communities are leave candidates even without
    //    a neighbour in them; every neighbour membership counts towards its community
    if (tid < mcnt) lds_insert(L.key, T, lg, own.comm);
    Slot sv[NB];
#pragma unroll
    for (int b = 0; b < NB; b++) {
        int v = b * NT + tid;
        sv[b].comm = -1;
        sv[b].in = 0;
        if (v < V) {
            const long long e = L.vslot[v];
            if (e >= 0) {
                sv[b].comm = (int)(unsigned)e;
                sv[b].in = (int)(e >> 32);
            } else {
                sv[b] = cx.slot[~e];
            }
        }
    }
#pragma unroll
    for (int b = 0; b < NB; b++) {
        // lanes of a wave that share the first pending community (a node's own
        // communities often hold most of its neighbours) insert and count it once; a
        // membership its neighbour left earlier in this iteration is no visit
        const int v = b * NT + tid;
        const int C = sv[b].comm;
        bool pend = v < V && C >= 0;
        int h = -1;
        for (int att = 0; att < 2; att++) {
            const unsigned long long pm = __ballot(pend);
            if (!pm) break;
            const int first = __ffsll((long long)pm) - 1;
            const int c0 = __shfl(C, first, WAVE);
            const bool in = pend && C == c0;
            const unsigned long long gm = __ballot(in);
            if (__popcll(gm) < 4) break;    // uniform over the wave
            int h0 = 0;
            if (lane == first) {
                h0 = lds_insert(L.key, T, lg, c0);
                atomicAdd(&L.kk[h0], __popcll(gm));
            }
            h0 = __shfl(h0, first, WAVE);
            if (in) {
                h = h0;
                pend = false;
            }
        }
        if (pend) {
            h = lds_insert(L.key, T, lg, C);
            atomicAdd(&L.kk[h], 1);
        }
        if (v < V) {
            L.vhash[v] = h;                 // -1 for a left membership
            L.vin[v] = sv[b].in;
        }
    }
    node_sync<NT>();
    // compact list of the occupied entries (at most V + mcnt <= VCAP; the order within the
    // list does not matter); the visit slots are consumed, so their storage becomes the
    // candidates' digits
    for (int t0 = 0; t0 < T; t0 += NT) {
        int t = t0 + tid;
        bool occ = t < T && L.key[t] >= 0;
        unsigned long long m = __ballot(occ);
        int base = 0;
        if (lane == 0 && m) base = atomicAdd(&L.nc, __popcll(m));
        base = __shfl(base, 0, WAVE);
        int c = base + __popcll(m & ((1ull << lane) - 1));
        if (occ) {
            L.cl[c] = t;
            L.ci[t] = c;
        }
    }
    node_sync<NT>();
    const int NC = L.nc;
    for (int c = tid; c < NC; c += NT) {
        L.d[0][c] = 0; L.d[1][c] = 0; L.d[2][c] = 0; L.d[3][c] = 0;
    }
    // 2. one community-record gather per candidate; its size feeds the visit terms
    int ct[NB];
    bool lv[NB];
    CandRec rc[NB];
#pragma unroll
    for (int b = 0; b < NB; b++) {
        int c = b * NT + tid;
        ct[b] = c < NC ? L.cl[c] : -1;
        lv[b] = false;
        if (ct[b] >= 0) {
            int C = L.key[ct[b]];
            for (int q = 0; q < mcnt; q++) lv[b] |= (L.mx[q] == C);
            load_cand(cx, C, lv[b], rc[b]);
        }
    }
#pragma unroll
    for (int b = 0; b < NB; b++) {
        int c = b * NT + tid;
        if (ct[b] >= 0) L.sz[c] = rc[b].s;
    }
    node_sync<NT>();
    // 3. exact correction of every visit, summed per candidate; as in phase 1, lanes of a
    //    wave that share the first pending candidate add one wave-summed set of digits
    int bad = 0;
    for (int v0 = 0; v0 < V; v0 += NT) {    // same trip count on every lane of a wave
        const int v = v0 + tid;
        const bool act = v < V && L.vhash[v] >= 0;
        int c = 0;
        i64 t0 = 0, t1 = 0, t2 = 0, t3 = 0;
        if (act) {
            int h = L.vhash[v];
            int C = L.key[h];
            c = L.ci[h];
            bool leave = false;
            for (int a = 0; a < mcnt; a++) leave |= (L.mx[a] == C);
            X192 term = visit_term(leave, L.vin[v], L.vdeg[v], L.sz[c], bad);
            x192_digits(term, t0, t1, t2, t3);
        }
        bool pend = act;
        for (int att = 0; att < 2; att++) {
            const unsigned long long pm = __ballot(pend);
            if (!pm) break;
            const int first = __ffsll((long long)pm) - 1;
            const int c0 = __shfl(c, first, WAVE);
            const bool in = pend && c == c0;
            const unsigned long long gm = __ballot(in);
            if (__popcll(gm) < 4) break;    // uniform over the wave
            const i64 a0 = wave_sum_i64(in ? t0 : 0), a1 = wave_sum_i64(in ? t1 : 0);
            const i64 a2 = wave_sum_i64(in ? t2 : 0), a3 = wave_sum_i64(in ? t3 : 0);
            if (lane == first) {
                atomicAdd(&L.d[0][c0], (unsigned long long)a0);
                atomicAdd(&L.d[1][c0], (unsigned long long)a1);
                atomicAdd(&L.d[2][c0], (unsigned long long)a2);
                atomicAdd(&L.d[3][c0], (unsigned long long)a3);
            }
            if (in) pend = false;
        }
        if (pend) {
            atomicAdd(&L.d[0][c], (unsigned long long)t0);
            atomicAdd(&L.d[1][c], (unsigned long long)t1);
            atomicAdd(&L.d[2][c], (unsigned long long)t2);
            atomicAdd(&L.d[3][c], (unsigned long long)t3);
        }
    }
    node_sync<NT>();
    // 4. change of every candidate's score, best join and best leave
    double bjd = 0.0, bld = 0.0;
    int bj = -1, bl = -1;
#pragma unroll
    for (int b = 0; b < NB; b++) {
        int t = ct[b];
        if (t < 0) continue;
        int c = b * NT + tid;
        int C = L.key[t];
        int k = L.kk[t];
        if (lv[b]) {
            int a = -1;
            for (int q = 0; q < mcnt; q++)
                if (L.mx[q] == C) a = q;
            if (L.mxin[a] != k) atomicOr(&cx.ctr->error, LF_DEVERR_INCOUNT);
        }
        X192 corr = x192_from_digits((i64)L.d[0][c], (i64)L.d[1][c], (i64)L.d[2][c], (i64)L.d[3][c]);
        double dl = cand_delta(rc[b], lv[b], k, d, corr, bad);
        if (lv[b]) better(dl, C, bld, bl);
        else better(dl, C, bjd, bj);
    }
    wave_best(bjd, bj);
    wave_best(bld, bl);
    if constexpr (NT > WAVE) {
        const int wv = tid / WAVE;
        if (lane == 0) {
            L.bjd[wv] = bjd; L.bj[wv] = bj;
            L.bld[wv] = bld; L.bl[wv] = bl;
        }
        __syncthreads();
        if (tid == 0) {
            for (int w = 1; w < NT / WAVE; w++) {
                int oc = L.bj[w];
                double od = L.bjd[w];
                if (oc >= 0 && (bj < 0 || od > bjd || (od == bjd && oc < bj))) { bjd = od; bj = oc; }
                oc = L.bl[w];
                od = L.bld[w];
                if (oc >= 0 && (bl < 0 || od > bld || (od == bld && oc < bl))) { bld = od; bl = oc; }
            }
        }
    }
    if (bad) atomicOr(&cx.ctr->error, LF_DEVERR_INEXACT);
    if (tid == 0) {
        cx.dj[j] = bj;
        cx.djd[j] = bj >= 0 ? bjd : 0.0;
        cx.dl[j] = bl;
        cx.dld[j] = bl >= 0 ? bld : 0.0;
        cx.dpos[j] = mcnt;
        cx.big_idx[j] = Q_DONE;
        if (cx.stats) {
            unsigned long long *w = cx.ctr->work[path];
            atomicAdd(&w[0], 1ull);
            atomicAdd(&w[1], (unsigned long long)d);
            atomicAdd(&w[2], (unsigned long long)V);
            atomicAdd(&w[3], (unsigned long long)NC);
            atomicAdd(&w[4], (unsigned long long)mcnt);
        }
    }
    return true;
}

__device__ __forceinline__ void mark_table(const Ctx &cx, int j, int deg, int own, const NodeLine &line)
{
    cx.big_ln[j] = line;                    // k_big_final reads it beside each entry's record
    if (cx.stats) {
        atomicAdd(&cx.ctr->work[LF_PATH_TABLE][0], 1ull);
        atomicAdd(&cx.ctr->work[LF_PATH_TABLE][1], (unsigned long long)deg);
        atomicAdd(&cx.ctr->work[LF_PATH_TABLE][4], (unsigned long long)own);
    }
    cx.big_idx[j] = Q_TABLE;
    cx.dpos[j] = own;
    cx.big_bj[j] = 0;
    cx.big_bl[j] = 0;
    cx.big_cj[j] = 0x7fffffff;
    cx.big_cl[j] = 0x7fffffff;
}


// The in-LDS evaluation paths take their queue's nodes from their path lists; the path
// was chosen so that the node fits, and a node that does not is an internal error.

// The small and medium paths of a single graph's queue in one launch of 256-thread
// blocks with 21 KB of LDS (seven blocks per CU): the first es blocks evaluate small-path
// nodes, one wave each (queues with many of them; otherwise they are a block role of
// k_eval_big), the next em blocks one medium-path node each, one visit per thread.
// Block 0 also resets the queue's apply counters.
union EvalLds {
    NodeLds<VSMALL> w[EW];
    NodeLds<VMED> m;
};

__device__ __forceinline__ void body_eval(const Ctx &cx, const QStep &qs, int blk, int nblk, EvalLds &L)
{
    (void)nblk;
    const int wv = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
    if (blk == 0 && threadIdx.x == 0) {
        DevCounters *c = cx.ctr;
        c->parts_total = 0;
        c->mslots = 0;
    }
    if (blk < qs.es) {
        const int p = blk * EW + wv;
        if (p >= qs.ln) return;             // small blocks have no block barriers
        const int j = cx.plist[LF_PATH_SMALL][qs.ls + p] - qs.cstart;
        const NodeRec nr = cx.prec[LF_PATH_SMALL][qs.ls + p];
        if (!eval_node<WAVE, VSMALL>(cx, j, nr, lane, L.w[wv], qs.wcap, LF_PATH_SMALL) && lane == 0)
            atomicOr(&cx.ctr->error, LF_DEVERR_CAP);
        return;
    }
    const int m = blk - qs.es;              // a medium block: every thread takes part
    if (m >= qs.em) return;
    const int j = cx.plist[LF_PATH_MED][qs.br.lm + m] - qs.cstart;
    const NodeRec nr = cx.prec[LF_PATH_MED][qs.br.lm + m];
    if (!eval_node<EW * WAVE, VMED>(cx, j, nr, threadIdx.x, L.m, qs.mcap, LF_PATH_MED) && threadIdx.x == 0)
        atomicOr(&cx.ctr->error, LF_DEVERR_CAP);
}

__global__ void __launch_bounds__(EW * WAVE) k_eval(Ctx cx, QStep qs)
{
    __shared__ EvalLds lds;
    body_eval(cx, qs, (int)blockIdx.x, (int)gridDim.x, lds);
}

// ------------------------------------------------------------------------------------
// evaluation, table path
// ------------------------------------------------------------------------------------
// slot of key (b, C) in the global table, claimed if absent (claimed = true then)
__device__ __forceinline__ long long gfind(const Ctx &cx, int b, int C, bool &claimed)
{
    unsigned long long key = ((unsigned long long)(unsigned)b << 32) | (unsigned)C;
    long long h = (long long)(hash64(key) & (unsigned long long)cx.gmask);
    claimed = false;
    for (long long probe = 0; probe <= cx.gmask; probe++) {
        unsigned long long cur = __atomic_load_n(&cx.gt[h].key, __ATOMIC_RELAXED);
        if (cur == key) return h;
        if (cur == GEMPTY) {
            unsigned long long old = atomicCAS(&cx.gt[h].key, GEMPTY, key);
            if (old == GEMPTY) {
                claimed = true;
                return h;
            }
            if (old == key) return h;
        }
        h = (h + 1) & cx.gmask;
    }
    return -1;
}

// The occupied list: a wave reserves one slot per visit of its 64 work items with a single
// atomic (a returning atomic on one shared counter costs ~10-20 ns, serialised, so one per
// 64-visit step would be the table path's bottleneck); each visit then writes the entry it
// claimed, or -1, into its own slot.

#define EWB 4           // waves per block in the table-path kernels

// Table path, one wave per 64 consecutive work items (neighbours, then own memberships,
// of the table-path nodes of this queue).  The wave flattens its items' neighbour
// memberships and walks them 64 at a time with every lane converged.  The lane that
// claims a key records its visit inline (no community gather, one atomic in total); every
// other visit adds its exact correction, with lanes of one wave that hit the same entry
// summed first so that a hot entry gets one set of atomics per wave.
struct TabLds {
    int vw[EWB];             // visits of each wave's chunk (block-wide slot reservation)
    long long obase;         // first occupied-list slot of the block's chunk
    long long sbase[EWB][WAVE];
    long long xoff[EWB][WAVE];
    int start[EWB][WAVE];
    int dy[EWB][WAVE];
    int j[EWB][WAVE];
    int xcnt[EWB][WAVE];
    int own[EWB][WAVE];
};

// blocks blk of nblk (EWB waves each) walk the work items of the queue's table-path
// nodes (list positions [ls, ls + ln))
__device__ __forceinline__ void table_visits(const Ctx &cx, int cstart, int ls, int ln, int blk, int nblk,
                                             TabLds &S)
{
    auto &s_sbase = S.sbase;
    auto &s_xoff = S.xoff;
    auto &s_start = S.start;
    auto &s_dy = S.dy;
    auto &s_j = S.j;
    auto &s_xcnt = S.xcnt;
    auto &s_own = S.own;
    const int wv = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
    const long long ib0 = cx.titem_base[ls];
    const long long count = cx.titem_base[ls + ln] - ib0;
    const long long bstride = (long long)nblk * EWB * WAVE;
    int bad = 0, capfail = 0;
    unsigned long long nvis = 0;
    // the block walks its chunks of EWB * 64 items in lockstep (same trip count for every
    // wave), so its waves can reserve their occupied-list slots with one atomic
    for (long long bbase = (long long)blk * EWB * WAVE; bbase < count; bbase += bstride) {
        const long long base = bbase + (long long)wv * WAVE;
        long long f = base + lane;
        int vc = 0, dy = 0, jj = -1, own = 0, xcnt = 0;
        long long sb = 0, xoff = 0;
        if (f < count) {
            int p = cx.titem_node[ib0 + f];
            int r = cx.plist[LF_PATH_TABLE][p];
            int j = r - cstart;
            {
                const NodeRec nr = cx.prec[LF_PATH_TABLE][p];
                const int x = nr.x;
                long long e = ib0 + f - cx.titem_base[p];
                int y = -1;
                if (e < nr.d) y = cx.col[nr.rb + e];  // issued beside the node's header
                const NodeLine *lxp = cx.ln + x;
                const int xdeg = lxp->deg, xc0 = lxp->cnt;
                const long long xo0 = lxp->off;
                Slot *xs = xo0 < 0 ? (Slot *)lxp->s : cx.slot + xo0;
                if (e == 0) mark_table(cx, j, xdeg, xc0, *lxp);   // k_big_final reads it after this launch
                if (e < xdeg) {
                    const NodeLine *lyp = cx.ln + y;
                    vc = lyp->cnt;
                    dy = lyp->deg;
                    const long long yo = lyp->off;
                    sb = (long long)(yo < 0 ? (Slot *)lyp->s : cx.slot + yo);
                } else if (e < (long long)xdeg + xc0) {
                    vc = 1;
                    sb = (long long)(xs + (e - xdeg));
                    own = 1;
                }
                jj = j;
                xoff = (long long)xs;
                xcnt = xc0;
            }
        }
        int incl = vc;
        for (int o = 1; o < WAVE; o <<= 1) {
            int t = __shfl_up(incl, o, WAVE);
            if (lane >= o) incl += t;
        }
        const int Vw = __shfl(incl, WAVE - 1, WAVE);
        // this wave's occupied-list slots [obase, obase + Vw): one atomic for the block
        if (lane == 0) S.vw[wv] = Vw;
        __syncthreads();
        if (threadIdx.x == 0) {
            int tot = 0;
            for (int w = 0; w < EWB; w++) tot += S.vw[w];
            S.obase = tot > 0 ? (long long)atomicAdd(&cx.ctr->occ_cnt, tot) : 0;
        }
        __syncthreads();
        long long obase = S.obase;
        for (int w = 0; w < wv; w++) obase += S.vw[w];
        s_start[wv][lane] = incl - vc;
        s_sbase[wv][lane] = sb;
        s_dy[wv][lane] = dy;
        s_j[wv][lane] = jj;
        s_xoff[wv][lane] = xoff;
        s_xcnt[wv][lane] = xcnt;
        s_own[wv][lane] = own;
        WAVE_SYNC();
        for (int v0 = 0; v0 < Vw; v0 += WAVE) {
            const int v = v0 + lane;
            const bool act = v < Vw;
            int C = 0, iv = 0, dyv = 0, xc = 0;
            long long hh = -1, xo = 0;
            bool claimed = false, ownv = false;
            if (act) {
                int lo = 0, hi = WAVE - 1;          // owner: last lane whose range starts <= v
                while (lo < hi) {
                    int mid = (lo + hi + 1) >> 1;
                    if (s_start[wv][mid] <= v) lo = mid; else hi = mid - 1;
                }
                int j = s_j[wv][lo];
                ownv = s_own[wv][lo] != 0;
                dyv = s_dy[wv][lo];
                xo = s_xoff[wv][lo];
                xc = s_xcnt[wv][lo];
                Slot sl = ((const Slot *)s_sbase[wv][lo])[v - s_start[wv][lo]];
                C = sl.comm;
                iv = sl.in;
                if (C >= 0) {                   // not a membership left in this iteration
                    hh = gfind(cx, j, C, claimed);
                    if (hh < 0) capfail = 1;
                }
            }
            if (act) cx.occ[obase + v] = claimed ? (int)hh : -1;
            const bool vis = act && hh >= 0 && !ownv;
            if (vis && claimed) {
                cx.gt[hh].ii = iv;
                cx.gt[hh].idy = dyv;
            }
            const bool extra = vis && !claimed;
            i64 t0 = 0, t1 = 0, t2 = 0, t3 = 0;
            if (extra) {
                long long s = cx.cr[C].s;
                bool leave = find_slot((const Slot *)xo, 0, xc, C) >= 0;
                X192 term = visit_term(leave, iv, dyv, s, bad);
                x192_digits(term, t0, t1, t2, t3);
            }
            bool pending = extra;
            for (int attempt = 0; attempt < 3; attempt++) {
                unsigned long long pm = __ballot(pending);
                if (!pm) break;
                int first = __ffsll((long long)pm) - 1;
                long long h0 = __shfl(hh, first, WAVE);
                bool in = pending && hh == h0;
                unsigned long long gm = __ballot(in);
                if (__popcll(gm) >= 4) {
                    i64 a0 = wave_sum_i64(in ? t0 : 0), a1 = wave_sum_i64(in ? t1 : 0);
                    i64 a2 = wave_sum_i64(in ? t2 : 0), a3 = wave_sum_i64(in ? t3 : 0);
                    if (lane == first) {
                        GEntry *g = &cx.gt[h0];
                        atomicAdd(&g->cnt, __popcll(gm));
                        atomicAdd((unsigned long long *)&g->d[0], (unsigned long long)a0);
                        atomicAdd((unsigned long long *)&g->d[1], (unsigned long long)a1);
                        atomicAdd((unsigned long long *)&g->d[2], (unsigned long long)a2);
                        atomicAdd((unsigned long long *)&g->d[3], (unsigned long long)a3);
                    }
                    if (in) pending = false;
                } else if (in) {
                    GEntry *g = &cx.gt[hh];
                    atomicAdd(&g->cnt, 1);
                    atomicAdd((unsigned long long *)&g->d[0], (unsigned long long)t0);
                    atomicAdd((unsigned long long *)&g->d[1], (unsigned long long)t1);
                    atomicAdd((unsigned long long *)&g->d[2], (unsigned long long)t2);
                    atomicAdd((unsigned long long *)&g->d[3], (unsigned long long)t3);
                    pending = false;
                }
            }
            if (pending) {
                GEntry *g = &cx.gt[hh];
                atomicAdd(&g->cnt, 1);
                atomicAdd((unsigned long long *)&g->d[0], (unsigned long long)t0);
                atomicAdd((unsigned long long *)&g->d[1], (unsigned long long)t1);
                atomicAdd((unsigned long long *)&g->d[2], (unsigned long long)t2);
                atomicAdd((unsigned long long *)&g->d[3], (unsigned long long)t3);
            }
            nvis += vis ? 1 : 0;
        }
        __syncthreads();                      // the chunk's LDS (and the reservation) is reused
    }
    if (cx.stats) {
        nvis = (unsigned long long)wave_sum_i64((long long)nvis);
        if (lane == 0 && nvis) atomicAdd(&cx.ctr->work[LF_PATH_TABLE][2], nvis);
    }
    if (bad) atomicOr(&cx.ctr->error, LF_DEVERR_INEXACT);
    if (capfail) atomicOr(&cx.ctr->error, LF_DEVERR_CAP);
}

// The larger nodes of a queue in one launch, by block role (BigRoles).  All read the state
// at the queue's start, so the roles are independent.

union BigLds {
    TabLds t;
    NodeLds<VGRP> g;
    NodeLds<VMED> m[GT / WAVE];
    NodeLds<VSMALL> s[GT / WAVE];
};

__device__ __forceinline__ void body_eval_big(const Ctx &cx, const QStep &qs, int blk, int nblk, BigLds &L)
{
    (void)nblk;
    const BigRoles &r = qs.br;
    const int cstart = qs.cstart;
    if (blk == 0 && threadIdx.x == 0) {     // the queue's apply counters (no role uses them)
        DevCounters *c = cx.ctr;
        c->parts_total = 0;
        c->mslots = 0;
    }
    int b = blk;
    if (b < r.bt) {
        table_visits(cx, cstart, r.lt, r.nt, b, r.bt, L.t);
        return;
    }
    b -= r.bt;
    if (b < r.bg) {
        for (int p = b; p < r.ng; p += r.bg) {
            const int j = cx.plist[LF_PATH_GROUP][r.lg + p] - cstart;
            const NodeRec nr = cx.prec[LF_PATH_GROUP][r.lg + p];
            if (!eval_node<GT, VGRP>(cx, j, nr, threadIdx.x, L.g, qs.gcap, LF_PATH_GROUP) && threadIdx.x == 0)
                atomicOr(&cx.ctr->error, LF_DEVERR_CAP);
            __syncthreads();                // the next node reuses the LDS
        }
        return;
    }
    b -= r.bg;
    const int wv = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
    if (b < r.bm) {
        for (int p = b * (GT / WAVE) + wv; p < r.nm; p += r.bm * (GT / WAVE)) {   // no block barriers
            const int j = cx.plist[LF_PATH_MED][r.lm + p] - cstart;
            const NodeRec nr = cx.prec[LF_PATH_MED][r.lm + p];
            if (!eval_node<WAVE, VMED>(cx, j, nr, lane, L.m[wv], qs.mcap, LF_PATH_MED) && lane == 0)
                atomicOr(&cx.ctr->error, LF_DEVERR_CAP);
        }
        return;
    }
    b -= r.bm;
    for (int p = b * (GT / WAVE) + wv; p < r.ns; p += r.bs * (GT / WAVE)) {    // small path, one wave per node
        const int j = cx.plist[LF_PATH_SMALL][qs.ls + p] - cstart;
        const NodeRec nr = cx.prec[LF_PATH_SMALL][qs.ls + p];
        if (!eval_node<WAVE, VSMALL>(cx, j, nr, lane, L.s[wv], qs.wcap, LF_PATH_SMALL) && lane == 0)
            atomicOr(&cx.ctr->error, LF_DEVERR_CAP);
    }
}
QUEUE_KERNELS(k_eval_big, GT, BigLds, body_eval_big)

__device__ __forceinline__ void body_big_final(const Ctx &cx, const QStep &qs, int blk, int nblk, NoLds &)
{
    const int cstart = qs.cstart, clen = qs.clen;
    int count = __atomic_load_n(&cx.ctr->occ_cnt, __ATOMIC_RELAXED);
    int bad = 0;
    unsigned long long ncand = 0;
    long long stride = (long long)nblk * blockDim.x;
    // every lane of a wave runs the same number of trips (invalid lanes idle), so the
    // per-wave reduction below sees all 64 lanes
    for (long long base = blk * (long long)blockDim.x; base < count; base += stride) {
        long long e = base + threadIdx.x;
        const bool inrange = e < count;
        long long h = inrange ? cx.occ[e] : -1;   // -1: a visit that claimed no entry
        bool valid = h >= 0;
        GEntry ge;
        ge.key = GEMPTY;
        if (valid) ge = cx.gt[h];
        unsigned long long key = ge.key;
        int b = valid ? (int)(key >> 32) : -1, C = (int)(unsigned)key;
        if (b >= clen) b = -1;
        double dlt = 0.0;
        bool leave = false;
        if (b >= 0) {
            // the node's line (copied at its marking) and the whole community record are
            // gathered side by side; the leave test then picks the record's half
            const NodeLine hx = cx.big_ln[b];
            const CommRec rec = cx.cr[C];
            int k = ge.cnt + (ge.idy > 0 ? 1 : 0);
            X192 corr = x192_from_digits(ge.d[0], ge.d[1], ge.d[2], ge.d[3]);
            int own_in = 0;
            int a = line_find(cx, hx, C, &own_in);
            leave = a >= 0;
            if (ge.idy > 0) {
                X192 t = visit_term(leave, ge.ii, ge.idy, rec.s, bad);
                x192_add(corr, t);
            }
            if (leave && own_in != k) atomicOr(&cx.ctr->error, LF_DEVERR_INCOUNT);
            CandRec r;
            r.s = rec.s;
            r.m = rec.m;
            r.W = rec.W;
#pragma unroll
            for (int q = 0; q < 5; q++) r.S[q] = leave ? rec.Sm[q] : rec.Sp[q];
            dlt = cand_delta(r, leave, k, hx.deg, corr, bad);
            ncand++;
        }
        // per-node maximum of the positive changes; one atomic per wave when every active
        // lane works on the same node (the common case: a node's entries are contiguous)
        {
            unsigned long long bits = dlt > 0.0 ? (unsigned long long)__double_as_longlong(dlt) : 0ull;
            unsigned long long jb = leave ? 0ull : bits, lb = leave ? bits : 0ull;
            int lane = threadIdx.x & (WAVE - 1);
            int b0 = __shfl(b, 0, WAVE);
            bool uni = __ballot(b != b0) == 0 && b0 >= 0;
            if (uni) {
                for (int o = 32; o >= 1; o >>= 1) {
                    unsigned long long oj = (unsigned long long)__shfl_xor((long long)jb, o, WAVE);
                    unsigned long long ol = (unsigned long long)__shfl_xor((long long)lb, o, WAVE);
                    if (oj > jb) jb = oj;
                    if (ol > lb) lb = ol;
                }
                if (lane == 0) {
                    if (jb) atomicMax(&cx.big_bj[b0], jb);
                    if (lb) atomicMax(&cx.big_bl[b0], lb);
                }
            } else if (b >= 0) {
                if (jb) atomicMax(&cx.big_bj[b], jb);
                if (lb) atomicMax(&cx.big_bl[b], lb);
            }
        }
        if (inrange && !valid) cx.occ_d[e] = 0.0;   // k_big_tie skips it
        if (valid) {
            cx.occ_key[e] = key | (leave ? (1ull << 63) : 0ull);
            cx.occ_d[e] = dlt;
            // leave the entry empty for the next queue
            GEntry *gp = &cx.gt[h];
            gp->key = GEMPTY;
            gp->cnt = 0;
            gp->ii = 0;
            gp->idy = 0;
            gp->d[0] = 0; gp->d[1] = 0; gp->d[2] = 0; gp->d[3] = 0;
        }
    }
    if (cx.stats) {
        ncand = (unsigned long long)wave_sum_i64((long long)ncand);
        if ((threadIdx.x & (WAVE - 1)) == 0 && ncand) atomicAdd(&cx.ctr->work[LF_PATH_TABLE][3], ncand);
    }
    if (bad) atomicOr(&cx.ctr->error, LF_DEVERR_INEXACT);
}

QUEUE_KERNELS(k_big_final, 256, NoLds, body_big_final)

__device__ __forceinline__ void body_big_tie(const Ctx &cx, const QStep &qs, int blk, int nblk, NoLds &)
{
    (void)qs;
    int count = __atomic_load_n(&cx.ctr->occ_cnt, __ATOMIC_RELAXED);
    long long stride = (long long)nblk * blockDim.x;
    for (long long e = blk * (long long)blockDim.x + threadIdx.x; e < count; e += stride) {
        double dlt = cx.occ_d[e];
        if (!(dlt > 0.0)) continue;
        unsigned long long key = cx.occ_key[e];
        bool leave = (key >> 63) != 0;
        int b = (int)((key >> 32) & 0x7fffffffull), C = (int)(unsigned)key;
        unsigned long long best = leave ? cx.big_bl[b] : cx.big_bj[b];
        if ((unsigned long long)__double_as_longlong(dlt) == best) atomicMin(leave ? &cx.big_cl[b] : &cx.big_cj[b], C);
    }
}
QUEUE_KERNELS(k_big_tie, 256, NoLds, body_big_tie)

// ------------------------------------------------------------------------------------
// bulk apply
// ------------------------------------------------------------------------------------

// A queue's decisions are applied by one launch: the membership edits (one thread per
// queued node) and the in-count changes around the moved nodes (one wave per in-count
// unit of the queue) run side by side.  Slot positions stay put within an iteration: a
// leave turns its slot's community into HOLE, a join writes its community into the
// node's free slot (position dpos, in-count 0 from the iteration start).  So the in-count
// updates can target slots while the edits run, and they take each neighbour's
// membership after the queue from the neighbour's own decision rather than from its
// slots: the result is a from-scratch recount of every in-count on the new partition.

// decision of the node at queue position j: community joined J and left L (-1: none)
__device__ __forceinline__ void queue_decision(const Ctx &cx, int j, int &J, int &L, unsigned long long *bjp,
                                               unsigned long long *blp)
{
    const int bi = cx.big_idx[j];
    const int dj = cx.dj[j], dl = cx.dl[j];
    const unsigned long long bj = cx.big_bj[j], bl = cx.big_bl[j];
    const int cj = cx.big_cj[j], cl = cx.big_cl[j];
    if (bi == Q_TABLE) {
        J = bj ? cj : -1;
        L = bl ? cl : -1;
    } else {
        J = dj;
        L = dl;
    }
    if (bjp) *bjp = bi == Q_TABLE ? bj : 0;
    if (blp) *blp = bi == Q_TABLE ? bl : 0;
}

// Re-sum parts of community C at its first touch in the queue, planned from its
// member-list capacity (fixed within an iteration).  Every lane of the wave calls this
// (want = false: it only takes part in the wave's reservation).
__device__ __forceinline__ void plan_parts(const Ctx &cx, bool want, int C, long long base, long long cap)
{
    int parts = (int)((cap + PART - 1) / PART);
    if (parts < 1) parts = 1;
    int p0 = wave_reserve(&cx.ctr->parts_total, want && parts == 1);
    if (!want) return;
    if (parts > 1) p0 = atomicAdd(&cx.ctr->parts_total, parts);
    PartRec pr;
    pr.base = base;
    pr.C = C;
    pr.parts = parts;
    pr.cap = (int)cap;
    pr.ms = -1;
    pr.pad = 0;
    if (p0 + parts > cx.part_cap) {
        atomicOr(&cx.ctr->error, LF_DEVERR_CAP);     // the run fails with this error
        pr.C = -1;                                    // the records that exist stay empty
    } else if (parts > 1) {
        cx.part_done[C] = 0;
        int ms = atomicAdd(&cx.ctr->mslots, 1);
        if (ms >= cx.mslot_cap) {
            atomicOr(&cx.ctr->error, LF_DEVERR_CAP);
            ms = 0;
        }
        pr.ms = ms;
        for (int k = 0; k < MACC; k++) cx.macc[(long long)ms * MACC + k] = 0;
    }
    for (int k = 0; k < parts && p0 + k < cx.part_cap; k++) {
        pr.k = k;
        cx.part_rec[p0 + k] = pr;
    }
}

// membership edits of queue position j (threads past the queue only take part in the
// wave-wide counting and reservations)
__device__ __forceinline__ void apply_edit(const Ctx &cx, const QStep &qs, int j)
{
    const int cstart = qs.cstart, clen = qs.clen;
    const int lane = threadIdx.x & (WAVE - 1);
    if (j == 0) cx.ctr->occ_cnt = 0;        // the table path of this queue is done
    const bool inq = j < clen;
    int J = -1, L = -1, x = -1;
    if (inq) {
        unsigned long long bj = 0, bl = 0;
        queue_decision(cx, j, J, L, &bj, &bl);
        x = cx.order[cstart + j];
        if (bj || bl || cx.big_idx[j] == Q_TABLE) {
            cx.dj[j] = J;
            cx.dl[j] = L;
            cx.djd[j] = __longlong_as_double((long long)bj);
            cx.dld[j] = __longlong_as_double((long long)bl);
        }
    }
    unsigned long long ml = __ballot(L >= 0);
    if (lane == 0 && ml) atomicAdd(&cx.ctr->leaves, (unsigned long long)__popcll(ml));
    const bool act = inq && (J >= 0 || L >= 0);
    bool firstL = false, firstJ = false, joined = false;
    long long cmoL = 0, cmeL = 0, cmoJ = 0, cmeJ = 0;
    int own_scanned = 0;
    if (act) {
        // the node's line and slot capacity and both member-list ranges in one round trip
        const NodeLine hx = cx.ln[x];
        const long long nxt = cx.nh[x + 1].off;
        if (L >= 0) {
            cmoL = cx.cm_off[L];
            cmeL = cx.cm_off[L + 1];
        }
        if (J >= 0) {
            cmoJ = cx.cm_off[J];
            cmeJ = cx.cm_off[J + 1];
        }
        // a node's slots change only in its own queue, so they hold no hole yet and its
        // free slot is at cnt
        const int cnt = hx.cnt;
        const long long capx = hx.off < 0 ? LINE_SLOTS : nxt - hx.off;
        Slot *xs = hx.off < 0 ? cx.ln[x].s : cx.slot + hx.off;
        const bool jfits = J >= 0 && cnt < capx;
        if (J >= 0 && !jfits) atomicOr(&cx.ctr->error, LF_DEVERR_SLOTS);
        own_scanned = L >= 0 ? cnt : 0;
        int oldL = 1, oldJ = 1, p = 0;
        if (L >= 0) {
            atomicSub(&cx.cr[L].s, 1);
            oldL = atomicExch(&cx.tflag[L], 1);
        }
        if (jfits) {
            atomicAdd(&cx.cr[J].s, 1);
            p = atomicAdd(&cx.cm_len[J], 1);
            oldJ = atomicExch(&cx.tflag[J], 1);
        }
        if (L >= 0) {
            int tin = 0;
            const int t = line_find(cx, hx, L, &tin);
            if (t >= 0) xs[t].comm = HOLE;  // only the community word: in-counts are updated beside
            firstL = oldL == 0;             // first touch of L in this queue
        }
        if (jfits) {
            xs[cnt].comm = J;               // the free slot; its in-count is counted by the units
            cx.ln[x].cnt = cnt + 1;
            joined = true;
            if (p < cmeJ - cmoJ) {
                cx.cm_node[cmoJ + p] = x;
            } else {
                int e = atomicAdd(&cx.ctr->ovf_cnt, 1);
                cx.ovf_node[e] = x;
                cx.ovf_comm[e] = J;
                cx.ovf_flag[J] = 1;
            }
            firstJ = oldJ == 0;
        }
    }
    unsigned long long mj = __ballot(joined);
    if (mj && lane == __ffsll((long long)mj) - 1) atomicAdd(&cx.ctr->joins, (unsigned long long)__popcll(mj));
    if (cx.stats) {
        const long long mv = wave_sum_i64(act ? 1 : 0), os = wave_sum_i64(own_scanned);
        if (lane == 0 && mv) {
            atomicAdd(&cx.ctr->apply[LF_APPLY_MOVES], (unsigned long long)mv);
            atomicAdd(&cx.ctr->apply[LF_APPLY_OWN_SLOTS], (unsigned long long)os);
        }
    }
    plan_parts(cx, firstL, L, cmoL, cmeL - cmoL);
    plan_parts(cx, firstJ, J, cmoJ, cmeJ - cmoJ);
}

// in-count changes of the neighbours in unit u (one wave): a neighbour y that holds J
// (L) from before this queue and keeps it gains (loses) one; the node's new J slot counts
// its neighbours in J after the queue (those that keep J and those that join it)
__device__ __forceinline__ void apply_unit(const Ctx &cx, const QStep &qs, long long u)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const UnitRec ur = cx.unit[u];
    const int j = ur.r - qs.cstart;
    // the unit's neighbours, the node's decision, join position and line placement
    const int y = lane < ur.cnt ? cx.col[ur.rb + lane] : -1;
    const int ry = lane < ur.cnt ? cx.col_rank[ur.rb + lane] : -1;
    int J, L;
    queue_decision(cx, j, J, L, nullptr, nullptr);
    const int pos = cx.dpos[j];
    const long long xoff = cx.ln[ur.x].off;
    if (J < 0 && L < 0) return;             // uniform over the wave
    NodeLine ly;
    ly.cnt = 0;
    ly.off = -1;
    int Jy = -1, Ly = -1;
    if (y >= 0) {
        ly = cx.ln[y];
        const int jy = ry - qs.cstart;
        if (jy >= 0 && jy < qs.clen) queue_decision(cx, jy, Jy, Ly, nullptr, nullptr);
    }
    bool inJ = false;
    if (y >= 0) {
        if (ly.off < 0) {
#pragma unroll
            for (int t = 0; t < LINE_SLOTS; t++) {
                const int c = t < ly.cnt ? ly.s[t].comm : -1;
                if (J >= 0 && c == J) {
                    inJ = true;
                    if (Jy != J && Ly != J) atomicAdd(&cx.ln[y].s[t].in, 1);
                } else if (L >= 0 && c == L) {
                    if (Ly != L && Jy != L) atomicSub(&cx.ln[y].s[t].in, 1);
                }
            }
        } else {
            Slot *ys = cx.slot + ly.off;
            for (int t0 = 0; t0 < ly.cnt; t0 += 4) {   // four slot loads per round trip
                int cc[4];
#pragma unroll
                for (int q = 0; q < 4; q++) cc[q] = t0 + q < ly.cnt ? ys[t0 + q].comm : -1;
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const int c = cc[q];
                    if (J >= 0 && c == J) {
                        inJ = true;
                        if (Jy != J && Ly != J) atomicAdd(&ys[t0 + q].in, 1);
                    } else if (L >= 0 && c == L) {
                        if (Ly != L && Jy != L) atomicSub(&ys[t0 + q].in, 1);
                    }
                }
            }
        }
    }
    int fresh = (J >= 0 && y >= 0 && (Jy == J || (inJ && Ly != J))) ? 1 : 0;
    fresh = wave_sum_int(fresh);
    if (lane == 0 && J >= 0 && fresh) {
        Slot *xs = xoff < 0 ? cx.ln[ur.x].s : cx.slot + xoff;
        if (xoff >= 0 || pos < LINE_SLOTS) atomicAdd(&xs[pos].in, fresh);
    }
    if (cx.stats) {
        const long long sc = wave_sum_i64(y >= 0 ? ly.cnt : 0);
        if (lane == 0) {
            atomicAdd(&cx.ctr->apply[LF_APPLY_IN_ITEMS], 1ull);
            atomicAdd(&cx.ctr->apply[LF_APPLY_IN_NEIGHBOURS], (unsigned long long)ur.cnt);
            atomicAdd(&cx.ctr->apply[LF_APPLY_IN_SLOTS], (unsigned long long)sc);
        }
    }
}

// blocks [0, eb) edit (a thread per queued node), the rest take one in-count unit per wave
__device__ __forceinline__ void body_apply(const Ctx &cx, const QStep &qs, int blk, int nblk, NoLds &)
{
    (void)nblk;
    const int eb = (qs.clen + 255) / 256;
    if (blk < eb) {
        apply_edit(cx, qs, blk * 256 + threadIdx.x);
        return;
    }
    const long long w = (long long)(blk - eb) * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    if (w < qs.un) apply_unit(cx, qs, qs.ub + w);
}
QUEUE_KERNELS(k_apply, 256, NoLds, body_apply)

// ------------------------------------------------------------------------------------
// exact re-sum of the touched communities
// ------------------------------------------------------------------------------------
__device__ __forceinline__ void x192_to_digits6(const X192 &v, long long *dg)
{
    dg[0] = (long long)(v.w0 & 0xffffffffull);
    dg[1] = (long long)(v.w0 >> 32);
    dg[2] = (long long)(v.w1 & 0xffffffffull);
    dg[3] = (long long)(v.w1 >> 32);
    dg[4] = (long long)(v.w2 & 0xffffffffull);
    dg[5] = (long long)(int)(unsigned)(v.w2 >> 32);
}

// sum_k D_k 2^(32k) for six signed 64-bit counters
__device__ __forceinline__ X192 x192_from_digits6(const long long *D)
{
    X192 r = x192_zero();
#pragma unroll
    for (int k = 0; k < 6; k++) {
        long long v = D[k];
        u64 sgn = v < 0 ? ~0ull : 0ull;
        // v * 2^(32k) as a 192-bit two's complement value
        u64 w[3] = {0, 0, 0};
        int sh = 32 * k;
        int li = sh >> 6, bi = sh & 63;
        u64 lo = (u64)v << bi;
        u64 hi = bi ? (((u64)v >> (64 - bi)) | (sgn << bi)) : sgn;
        w[li] = lo;
        if (li + 1 < 3) w[li + 1] = hi;
        for (int q = li + 2; q < 3; q++) w[q] = sgn;
        X192 t = {w[0], w[1], w[2]};
        x192_add(r, t);
    }
    return r;
}

__device__ __forceinline__ void body_refresh(const Ctx &cx, const QStep &qs, int blk, int nblk, NoLds &)
{
    (void)qs;
    int lane = threadIdx.x & (WAVE - 1);
    long long nw = (long long)nblk * (blockDim.x / WAVE);
    int bad = 0;
    long long p = (blk * (long long)blockDim.x + threadIdx.x) / WAVE;
    // the wave's first part is read beside the count (the buffer holds part_cap records)
    PartRec first;
    if (p < cx.part_cap) first = cx.part_rec[p];
    int count = __atomic_load_n(&cx.ctr->parts_total, __ATOMIC_RELAXED);
    if (count > cx.part_cap) count = cx.part_cap;
    for (bool at_first = true; p < count; p += nw, at_first = false) {
        const PartRec pr = at_first ? first : cx.part_rec[p];
        const int C = pr.C;
        if (C < 0 || C >= cx.K) continue;          // only after a flagged overflow
        const int k = pr.k;
        const long long base = pr.base, cap = pr.cap;
        // size, list length and overflow after the edits, read beside the part's entries
        const long long s = cx.cr[C].s;
        long long len = cx.cm_len[C];
        const int ovf = cx.ovf_flag[C];
        const long long lo = (long long)k * PART;
        int mem[PART / WAVE];
#pragma unroll
        for (int i = 0; i < PART / WAVE; i++) {
            const long long q = lo + i * WAVE + lane;
            mem[i] = q < cap ? cx.cm_node[base + q] : -1;
        }
        if (len > cap) len = cap;
        // the plan covers the list's capacity; the parts that hold members after the edits
        // (the same count for every part of C: the length is final here) do the re-sum
        int parts = (int)((len + PART - 1) / PART);
        if (parts < 1) parts = 1;
        if (k >= parts) continue;
        const long long hi = lo + PART < len ? lo + PART : len;
        X192 a0 = x192_zero(), ap = x192_zero(), am = x192_zero();
        long long sumi = 0;
#pragma unroll
        for (int i = 0; i < PART / WAVE; i++)
            if (lo + i * WAVE + lane < hi) member_terms_line(cx, mem[i], C, s, a0, ap, am, sumi, bad);
        if (cx.stats) {
            long long mslots = 0;
            for (int i = 0; i < PART / WAVE; i++)
                if (lo + i * WAVE + lane < hi) mslots += cx.ln[mem[i]].cnt;
            mslots = wave_sum_i64(mslots);
            if (lane == 0) {
                atomicAdd(&cx.ctr->apply[LF_APPLY_PARTS], 1ull);
                if (k == 0) atomicAdd(&cx.ctr->apply[LF_APPLY_TOUCHED], 1ull);
                atomicAdd(&cx.ctr->apply[LF_APPLY_MEMBERS], (unsigned long long)(hi > lo ? hi - lo : 0));
                atomicAdd(&cx.ctr->apply[LF_APPLY_MEMBER_SLOTS], (unsigned long long)mslots);
            }
        }
        if (k == 0 && ovf) {
            int no = __atomic_load_n(&cx.ctr->ovf_cnt, __ATOMIC_RELAXED);
            for (int e = lane; e < no; e += WAVE)
                if (cx.ovf_comm[e] == C) member_terms_line(cx, cx.ovf_node[e], C, s, a0, ap, am, sumi, bad);
        }
        a0 = wave_sum_x192(a0);
        ap = wave_sum_x192(ap);
        am = wave_sum_x192(am);
        sumi = wave_sum_i64(sumi);
        if (lane != 0) continue;
        if (parts == 1) {
            store_comm(cx, C, s, a0, ap, am, sumi, bad);
            continue;
        }
        unsigned long long *acc = (unsigned long long *)&cx.macc[(long long)pr.ms * MACC];
        long long dg[6];
        x192_to_digits6(a0, dg);
        for (int q = 0; q < 6; q++) atomicAdd(acc + q, (unsigned long long)dg[q]);
        x192_to_digits6(ap, dg);
        for (int q = 0; q < 6; q++) atomicAdd(acc + 6 + q, (unsigned long long)dg[q]);
        x192_to_digits6(am, dg);
        for (int q = 0; q < 6; q++) atomicAdd(acc + 12 + q, (unsigned long long)dg[q]);
        atomicAdd(acc + 18, (unsigned long long)sumi);
        __threadfence();
        if (atomicAdd(&cx.part_done[C], 1) == parts - 1) {
            // last part: every other part's counters are in (they fenced before counting)
            __threadfence();
            long long D[MACC];
            for (int q = 0; q < MACC; q++) D[q] = (long long)__atomic_load_n(acc + q, __ATOMIC_RELAXED);
            store_comm(cx, C, s, x192_from_digits6(D), x192_from_digits6(D + 6), x192_from_digits6(D + 12), D[18],
                       bad);
        }
    }
    if (bad) atomicOr(&cx.ctr->error, LF_DEVERR_INEXACT);
}
QUEUE_KERNELS(k_refresh, 256, NoLds, body_refresh)

// ------------------------------------------------------------------------------------
// per-iteration sizing of the queue buffers
// ------------------------------------------------------------------------------------
// Evaluation path of every node for this iteration.  A node's own memberships do not
// change before it is evaluated, and each neighbour gains at most one membership per
// iteration, only if it is evaluated earlier (a smaller order position: the neighbours
// in the same queue are read at the queue's start).  So visits at evaluation <=
// B = visits at the iteration start + neighbours earlier in the order, and the path
// chosen from B always fits.  vbound[x] = B + own + 1 bounds x's distinct table keys.
// NB_NODES consecutive nodes per wave: their neighbour ranges are walked as one flattened
// range (most nodes have far fewer than 64 neighbours), each lane finding its node in the
// wave's range starts, and the per-node sums collect in LDS.
#define NB_NODES 16
__global__ void __launch_bounds__(256) k_node_bounds(Ctx cx, long long *vbound, int *cls, int wcap, int mcap,
                                                     int gcap)
{
    __shared__ long long s_start[256 / WAVE][NB_NODES + 1];
    __shared__ long long s_rb[256 / WAVE][NB_NODES];
    __shared__ unsigned long long s_v[256 / WAVE][NB_NODES];
    __shared__ unsigned s_pre[256 / WAVE][NB_NODES];
    __shared__ int s_rx[256 / WAVE][NB_NODES];
    const int wv = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
    const long long x0 = (blockIdx.x * (long long)(blockDim.x / WAVE) + wv) * NB_NODES;
    if (x0 >= cx.n) return;                 // uniform over the wave; only wave-level syncs below
    const int nn = cx.n - x0 < NB_NODES ? (int)(cx.n - x0) : NB_NODES;
    long long rb = 0, d = 0;
    int rx = 0;
    if (lane < nn) {
        rb = cx.rowptr[x0 + lane];
        d = cx.rowptr[x0 + lane + 1] - rb;
        rx = cx.rank[x0 + lane];
    }
    long long incl = d;                     // lanes >= nn add nothing
    for (int o = 1; o < NB_NODES; o <<= 1) {
        const long long t = __shfl_up(incl, o, WAVE);
        if (lane >= o) incl += t;
    }
    const long long D = __shfl(incl, NB_NODES - 1, WAVE);
    if (lane < NB_NODES) {
        s_start[wv][lane + 1] = incl;
        s_rb[wv][lane] = rb;
        s_rx[wv][lane] = rx;
        s_v[wv][lane] = 0;
        s_pre[wv][lane] = 0;
    }
    if (lane == 0) s_start[wv][0] = 0;
    WAVE_SYNC();
    for (long long f = lane; f < D; f += WAVE) {
        int lo = 0, hi = nn - 1;            // the last node whose range starts at or before f
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_start[wv][mid] <= f) lo = mid; else hi = mid - 1;
        }
        const long long e = s_rb[wv][lo] + (f - s_start[wv][lo]);
        const int y = cx.col[e];
        const int ry = cx.col_rank[e];
        atomicAdd(&s_v[wv][lo], (unsigned long long)cx.nh[y].cnt);
        if (ry < s_rx[wv][lo]) atomicAdd(&s_pre[wv][lo], 1u);
    }
    WAVE_SYNC();
    if (lane < nn) {
        const long long x = x0 + lane;
        NodeHdr hx = cx.nh[x];
        const long long B = (long long)s_v[wv][lane] + s_pre[wv][lane], M = hx.cnt, dd = hx.deg;
        vbound[x] = B + M + 1;
        int c = LF_PATH_TABLE;
        if (M <= MXCAP) {
            if (dd <= VSMALL && B + M <= VSMALL && 2 * (B + M) <= wcap) c = LF_PATH_SMALL;
            else if (dd <= VMED && B + M <= VMED && 2 * (B + M) <= mcap) c = LF_PATH_MED;
            else if (dd <= VGRP && B + M <= VGRP && 2 * (B + M) <= gcap) c = LF_PATH_GROUP;
        }
        cls[rx] = c;
    }
}

// per queue: work items and table keys of its table-path nodes, and in-count items of
// all its nodes; the maxima over queues go to out[0..2]
__global__ void __launch_bounds__(256) k_chunk_bounds(Ctx cx, const long long *vbound, const int *cls, int q,
                                                      unsigned long long *out)
{
    __shared__ long long s_a[256 / WAVE], s_b[256 / WAVE], s_c[256 / WAVE];
    long long start = (long long)blockIdx.x * q;
    long long end = start + q < cx.n ? start + q : cx.n;
    long long a = 0, b = 0, c = 0;
    for (long long r = start + threadIdx.x; r < end; r += blockDim.x) {
        int x = cx.order[r];
        NodeHdr hx = cx.nh[x];
        if (cls[r] == LF_PATH_TABLE) {
            a += hx.deg + hx.cnt + 1;
            b += vbound[x];
        }
        c += (hx.deg + INB - 1) / INB;
    }
    a = wave_sum_i64(a);
    b = wave_sum_i64(b);
    c = wave_sum_i64(c);
    int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    if (lane == 0) { s_a[wv] = a; s_b[wv] = b; s_c[wv] = c; }
    __syncthreads();
    if (threadIdx.x == 0) {
        long long ta = 0, tb = 0, tc = 0;
        for (int k = 0; k < 256 / WAVE; k++) { ta += s_a[k]; tb += s_b[k]; tc += s_c[k]; }
        atomicMax(&out[0], (unsigned long long)ta);
        atomicMax(&out[1], (unsigned long long)tb);
        atomicMax(&out[2], (unsigned long long)tc);
    }
}

// flags[r] = (cls[r] == c) for the scan that places path c's nodes; flags[n] = 0
__global__ void k_class_flags(const int *cls, int c, long long *flags, long long n)
{
    long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (r < n) flags[r] = cls[r] == c ? 1 : 0;
    else if (r == n) flags[r] = 0;
}

// path c's list (ascending order positions) with its node records (at pbase[c] of the
// shared record array), and its first list position per queue
__global__ void k_class_scatter(const int *cls, int c, const long long *scan, int *list, long long n, int q,
                                long long nq, long long *qoff, const int *order, const long long *rowptr,
                                const int *deg, const long long *pbase, NodeRec *prec)
{
    long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (r < n && cls[r] == c) {
        const long long i = scan[r];
        const int x = order[r];
        list[i] = (int)r;
        NodeRec nr;
        nr.rb = rowptr[x];
        nr.x = x;
        nr.d = deg[x];
        prec[pbase[c] + i] = nr;
    }
    if (r <= nq) {
        long long p = r * q < n ? r * q : n;
        qoff[r] = scan[p];
    }
}

// pbase[c + 1] = pbase[c] + the number of path-c nodes (scan[n])
__global__ void k_path_base(const long long *scan, long long n, int c, long long *pbase)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) pbase[c + 1] = pbase[c] + scan[n];
}

// work items of every table-path node: its neighbours, its own memberships and one spare;
// the number of table-path nodes nt is read on the device (the path list's length), and
// the counts are written for all n + 1 positions (0 from nt on)
__global__ void k_titem_counts(Ctx cx, const long long *nt_dev, long long n, long long *cnt)
{
    long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (p > n) return;
    if (p >= *nt_dev) { cnt[p] = 0; return; }
    NodeHdr hx = cx.nh[cx.order[cx.plist[LF_PATH_TABLE][p]]];
    cnt[p] = (long long)hx.deg + hx.cnt + 1;
}

__global__ void k_queue_items(const long long *titem_base, const long long *qoff_t, long long nq, long long *out)
{
    long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (k <= nq) out[k] = titem_base[qoff_t[k]];
}

// owner of every work item; waves stride over the nt table-path nodes.  Nothing is written
// if the items exceed the buffer's capacity (the host then grows it and runs this again).
__global__ void __launch_bounds__(256) k_titem_fill(Ctx cx, const long long *nt_dev, long long cap)
{
    const long long nt = *nt_dev;
    if (cx.titem_base[nt] > cap) return;
    const int lane = threadIdx.x & (WAVE - 1);
    const long long nw = (long long)gridDim.x * (blockDim.x / WAVE);
    for (long long p = (blockIdx.x * (long long)blockDim.x + threadIdx.x) / WAVE; p < nt; p += nw) {
        long long a = cx.titem_base[p], b = cx.titem_base[p + 1];
        for (long long f = a + lane; f < b; f += WAVE) cx.titem_node[f] = (int)p;
    }
}

// the membership lines of an iteration, from the slot layout (nodes whose capacity fits a
// line keep their memberships inline, the others point into the slot array)
__global__ void __launch_bounds__(256) k_line_build(Ctx cx)
{
    const long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (x >= cx.n) return;
    const NodeHdr hx = cx.nh[x];
    const long long cap = cx.nh[x + 1].off - hx.off;
    NodeLine l;
    l.cnt = hx.cnt;
    l.deg = hx.deg;
    l.off = cap <= LINE_SLOTS ? -1 : hx.off;
#pragma unroll
    for (int t = 0; t < LINE_SLOTS; t++) {
        Slot sl = {-1, 0};
        if (l.off < 0 && t < hx.cnt) sl = cx.slot[hx.off + t];
        l.s[t] = sl;
    }
    cx.ln[x] = l;
}

// back to the slot layout at the end of an iteration (or of a stop within one): the
// memberships in order without the ones left (holes), and their count
__global__ void __launch_bounds__(256) k_line_back(Ctx cx)
{
    const long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (x >= cx.n) return;
    const NodeLine l = cx.ln[x];
    const long long o = cx.nh[x].off;
    int w = 0;
    if (l.off < 0) {
#pragma unroll
        for (int t = 0; t < LINE_SLOTS; t++)
            if (t < l.cnt && l.s[t].comm >= 0) cx.slot[o + w++] = l.s[t];
    } else {
        for (int t = 0; t < l.cnt; t++) {
            const Slot sl = cx.slot[o + t];
            if (sl.comm >= 0) cx.slot[o + w++] = sl;
        }
    }
    cx.nh[x].cnt = w;
}

// in-count units of every node in node order (one per INB neighbours; ubase = their
// exclusive scan), and the first unit of every queue
__global__ void k_unit_counts(const int *order, const int *deg, long long n, long long *cnt)
{
    const long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (r < n) cnt[r] = (deg[order[r]] + INB - 1) / INB;
    else if (r == n) cnt[n] = 0;
}

__global__ void k_unit_fill(const int *order, const long long *rowptr, const int *deg, const long long *ubase,
                            long long n, UnitRec *unit, long long cap)
{
    const long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int x = order[r], d = deg[x];
    const long long rb = rowptr[x], b = ubase[r];
    for (int k = 0; k * INB < d; k++) {
        if (b + k >= cap) break;            // cannot happen: cap bounds the total
        UnitRec u;
        u.rb = rb + (long long)k * INB;
        u.x = x;
        u.r = (int)r;
        u.cnt = d - k * INB < INB ? d - k * INB : INB;
        u.pad = 0;
        unit[b + k] = u;
    }
}

__global__ void k_queue_units(const long long *ubase, long long n, int q, long long nq, long long *out)
{
    const long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (k <= nq) out[k] = ubase[k * q < n ? k * q : n];
}

__global__ void k_empty_table(GEntry *t, long long n)
{
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i < n) t[i].key = GEMPTY;
}

// ------------------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------------------
void lf_free_iteration_buffers(lf_handle *h)
{
    void **ptrs[] = {(void **)&h->dj, (void **)&h->dl, (void **)&h->djd, (void **)&h->dld,
                     (void **)&h->big_idx,
                     (void **)&h->big_bj, (void **)&h->big_bl, (void **)&h->big_cj, (void **)&h->big_cl,
                     (void **)&h->big_ln,
                     (void **)&h->gt, (void **)&h->occ, (void **)&h->occ_key, (void **)&h->occ_d,
                     (void **)&h->unit, (void **)&h->dpos, (void **)&h->part_rec, (void **)&h->macc,
                     (void **)&h->titem_base, (void **)&h->titem_node};
    for (void **p : ptrs) {
        lf_dev_free(h, *p);
        *p = nullptr;
    }
    h->q_cap = 0;
    h->gT = 0;
    h->unit_cap = 0;
    h->part_cap = 0;
    h->mslot_cap = 0;
    h->titem_cap = 0;
}

// The iteration start's report (device dq, copied to the pinned host hqoff), for nq
// queues: per path the first list position of every queue ([LF_PATH_COUNT][nq + 1]),
// the first table-path work item of every queue, the first in-count unit of every queue,
// then 4 bounds of k_chunk_bounds.
#define REP_ITEMS(nq) ((long long)LF_PATH_COUNT * ((nq) + 1))
#define REP_UNITS(nq) ((long long)(LF_PATH_COUNT + 1) * ((nq) + 1))
#define REP_BOUNDS(nq) ((long long)(LF_PATH_COUNT + 2) * ((nq) + 1))
#define REP_LEN(nq) (REP_BOUNDS(nq) + 4)

// Start of an iteration, first half: everything the host does not need to see, queued on
// the stream, ending with one copy of the queue offsets and bounds to pinned host memory.
// The second half (size_queue_complete) runs once that copy has landed.
static int size_queue_enqueue(lf_handle *h, long long q)
{
    TmpScope tmp_scope(h);
    hipStream_t st = h->stream;
    const int BS = 256;
    long long n = h->n;
    bool moved = false;
    if (q > h->q_cap) {
        void **ptrs[] = {(void **)&h->dj, (void **)&h->dl, (void **)&h->djd, (void **)&h->dld, (void **)&h->dpos,
                         (void **)&h->big_idx,
                         (void **)&h->big_bj, (void **)&h->big_bl, (void **)&h->big_cj, (void **)&h->big_cl,
                         (void **)&h->big_ln};
        for (void **p : ptrs) {
            lf_dev_free(h, *p);
            *p = nullptr;
        }
        LF_TRY(lf_dev_alloc(h, (void **)&h->dpos, sizeof(int) * q));
        LF_TRY(lf_dev_alloc(h, (void **)&h->dj, sizeof(int) * q));
        LF_TRY(lf_dev_alloc(h, (void **)&h->dl, sizeof(int) * q));
        LF_TRY(lf_dev_alloc(h, (void **)&h->djd, sizeof(double) * q));
        LF_TRY(lf_dev_alloc(h, (void **)&h->dld, sizeof(double) * q));
        LF_TRY(lf_dev_alloc(h, (void **)&h->big_idx, sizeof(int) * q));
        LF_TRY(lf_dev_alloc(h, (void **)&h->big_bj, sizeof(unsigned long long) * q));
        LF_TRY(lf_dev_alloc(h, (void **)&h->big_bl, sizeof(unsigned long long) * q));
        LF_TRY(lf_dev_alloc(h, (void **)&h->big_cj, sizeof(int) * q));
        LF_TRY(lf_dev_alloc(h, (void **)&h->big_cl, sizeof(int) * q));
        LF_TRY(lf_dev_alloc(h, (void **)&h->big_ln, sizeof(NodeLine) * q));
        h->q_cap = q;
        moved = true;
    }
    // paths of this iteration, then bounds of the table path and in-count items
    const long long nq = (n + q - 1) / q;
    Ctx cx = lf_ctx(h);
    hipLaunchKernelGGL(k_node_bounds, dim3(grid_for((n + NB_NODES - 1) / NB_NODES * WAVE, BS)), dim3(BS), 0, st,
                       cx, h->vbound, h->cls,
                       h->eval_wave_cap < 2 * VSMALL ? h->eval_wave_cap : 2 * VSMALL, h->eval_med_cap,
                       h->eval_grp_cap);
    if (h->hqoff_cap < nq + 1) {            // pinned, so the one copy below is truly asynchronous
        // (the last copy into the old buffer was read by the previous iteration start)
        if (h->hqoff) lf_host_release(h->hqoff, sizeof(long long) * h->hqoff_len);
        h->hqoff = nullptr;
        h->hqoff_cap = 0;
        if (lf_host_alloc((void **)&h->hqoff, sizeof(long long) * REP_LEN(nq)) != LF_OK)
            return lf_set_error(h, LF_ENOMEM, "host queue offsets");
        h->hqoff_cap = nq + 1;
        h->hqoff_len = REP_LEN(nq);
    }
    const long long nrep = REP_LEN(nq);    // list offsets, queue items, queue units, bounds
    if (nrep > h->dq_cap) {                 // kept across the two halves (and iterations)
        lf_dev_free(h, h->dq);
        h->dq = nullptr;
        LF_TRY(lf_dev_alloc(h, (void **)&h->dq, sizeof(long long) * (nrep + nrep / 4 + 64)));
        h->dq_cap = nrep + nrep / 4 + 64;
    }
    long long *dq = h->dq;
    if (!h->titem_base) {
        LF_TRY(lf_dev_alloc(h, (void **)&h->titem_base, sizeof(long long) * (n + 1)));
        moved = true;
    }
    LF_TRY(lf_zero(h, h->pbase, sizeof(long long)));
    for (int c = 0; c < LF_PATH_COUNT; c++) {
        // titem_base serves as the flag array until the table-path items are laid out
        hipLaunchKernelGGL(k_class_flags, dim3(grid_for(n + 1, BS)), dim3(BS), 0, st, (const int *)h->cls, c,
                           h->titem_base, n);
        LF_TRY(lf_exclusive_scan_i64(h, h->titem_base, h->cscan, n + 1));
        long long m = (n > nq ? n : nq) + 1;
        hipLaunchKernelGGL(k_class_scatter, dim3(grid_for(m, BS)), dim3(BS), 0, st, (const int *)h->cls, c,
                           (const long long *)h->cscan, h->plist[c], n, (int)q, nq, dq + c * (nq + 1),
                           (const int *)h->order, (const long long *)h->rowptr, (const int *)h->deg,
                           (const long long *)h->pbase, h->prec_all);
        hipLaunchKernelGGL(k_path_base, dim3(1), dim3(1), 0, st, (const long long *)h->cscan, n, c, h->pbase);
    }
    unsigned long long *dout = (unsigned long long *)(dq + REP_BOUNDS(nq));
    LF_TRY(lf_zero(h, dout, sizeof(unsigned long long) * 4));
    hipLaunchKernelGGL(k_chunk_bounds, dim3((unsigned)nq), dim3(BS), 0, st, cx, (const long long *)h->vbound,
                       (const int *)h->cls, (int)q, dout);
    // static work-item layout of the table-path nodes (list position p owns deg + cnt + 1),
    // all on the device: the table path's length is the last queue offset of its list
    const long long *nt_dev = dq + LF_PATH_TABLE * (nq + 1) + nq;
    hipLaunchKernelGGL(k_titem_counts, dim3(grid_for(n + 1, BS)), dim3(BS), 0, st, lf_ctx(h), nt_dev, n, h->cscan);
    LF_TRY(lf_exclusive_scan_i64(h, h->cscan, h->titem_base, n + 1));
    if (!h->titem_node) {
        long long want = 4096 + n / 4;
        LF_TRY(lf_dev_alloc(h, (void **)&h->titem_node, sizeof(int) * want));
        h->titem_cap = want;
        moved = true;
    }
    unsigned fill_grid = grid_for(n * WAVE, BS);
    if (fill_grid > 2048) fill_grid = 2048;
    if (fill_grid < 1) fill_grid = 1;
    hipLaunchKernelGGL(k_titem_fill, dim3(fill_grid), dim3(BS), 0, st, lf_ctx(h), nt_dev, h->titem_cap);
    // first table-path work item of every queue (sizes the table-visit role)
    hipLaunchKernelGGL(k_queue_items, dim3(grid_for(nq + 1, BS)), dim3(BS), 0, st, (const long long *)h->titem_base,
                       (const long long *)(dq + LF_PATH_TABLE * (nq + 1)), nq, dq + REP_ITEMS(nq));
    // in-count units of every node in node order, and the first unit of every queue
    {
        const long long ucap = n + 2 * h->ne / INB + 1;   // >= sum of ceil(degree / INB)
        if (ucap > h->unit_cap) {
            lf_dev_free(h, h->unit);
            h->unit = nullptr;
            LF_TRY(lf_dev_alloc(h, (void **)&h->unit, sizeof(UnitRec) * ucap));
            h->unit_cap = ucap;
            moved = true;
        }
        long long *ucnt = nullptr, *ubase = nullptr;
        LF_TRY(lf_tmp_alloc(h, (void **)&ucnt, sizeof(long long) * (n + 1)));
        LF_TRY(lf_tmp_alloc(h, (void **)&ubase, sizeof(long long) * (n + 1)));
        hipLaunchKernelGGL(k_unit_counts, dim3(grid_for(n + 1, BS)), dim3(BS), 0, st, (const int *)h->order,
                           (const int *)h->deg, n, ucnt);
        LF_TRY(lf_exclusive_scan_i64(h, ucnt, ubase, n + 1));
        if (n > 0)
            hipLaunchKernelGGL(k_unit_fill, dim3(grid_for(n, BS)), dim3(BS), 0, st, (const int *)h->order,
                               (const long long *)h->rowptr, (const int *)h->deg, (const long long *)ubase, n, h->unit,
                               h->unit_cap);
        hipLaunchKernelGGL(k_queue_units, dim3(grid_for(nq + 1, BS)), dim3(BS), 0, st, (const long long *)ubase, n,
                           (int)q, nq, dq + REP_UNITS(nq));
    }
    // the host's one wait of the iteration start: list offsets per queue and path, the
    // queues' first table items, the bounds
    LF_HIP(h, hipMemcpyAsync(h->hqoff, dq, sizeof(long long) * nrep, hipMemcpyDeviceToHost, st));
    LF_HIP(h, hipGetLastError());
    h->pending_moved = moved;
    h->fill_grid = fill_grid;
    return LF_OK;
}

// second half: the host reads what the first half copied (the caller has waited for it)
// and grows whatever it found too small
static int size_queue_complete(lf_handle *h, long long q)
{
    hipStream_t st = h->stream;
    const int BS = 256;
    const long long n = h->n;
    const long long nq = (n + q - 1) / q;
    bool moved = h->pending_moved;
    h->second_half_work = false;
    const unsigned fill_grid = h->fill_grid;
    const long long *nt_dev = h->dq + LF_PATH_TABLE * (nq + 1) + nq;
    const unsigned long long *hb = (const unsigned long long *)(h->hqoff + REP_BOUNDS(nq));
    {   // the records of path c start after those of the paths before it
        long long base = 0;
        for (int c = 0; c < LF_PATH_COUNT; c++) {
            h->prec[c] = h->prec_all + base;
            base += h->hqoff[c * (nq + 1) + nq];
        }
    }
    long long keys = (long long)hb[1] + 64;
    if (keys >= (1ll << 30))
        return lf_set_error(h, LF_EOVERFLOW, "queue of %lld nodes too large for the table path", q);
    const long long nt = h->hqoff[LF_PATH_TABLE * (nq + 1) + nq];
    const long long items = h->hqoff[REP_ITEMS(nq) + nq];
    if (items > h->titem_cap) {             // rare: grow and lay the items out again
        lf_dev_free(h, h->titem_node);
        h->titem_node = nullptr;
        long long want = (h->phase_graphs ? 4 : 2) * items + 1024;
        LF_TRY(lf_dev_alloc(h, (void **)&h->titem_node, sizeof(int) * want));
        h->titem_cap = want;
        moved = true;
        if (nt > 0) {
            hipLaunchKernelGGL(k_titem_fill, dim3(fill_grid), dim3(BS), 0, st, lf_ctx(h), nt_dev, h->titem_cap);
            h->second_half_work = true;
        }
    }
    long long T = 1024;
    while (T < 2 * keys) T <<= 1;
    if (T > h->gT) {
        if (h->phase_graphs) T *= 4;        // a batch member's graphs survive more growth
        void **ptrs[] = {(void **)&h->gt, (void **)&h->occ, (void **)&h->occ_key, (void **)&h->occ_d};
        for (void **p : ptrs) {
            lf_dev_free(h, *p);
            *p = nullptr;
        }
        LF_TRY(lf_dev_alloc(h, (void **)&h->gt, sizeof(GEntry) * T));
        LF_TRY(lf_dev_alloc(h, (void **)&h->occ, sizeof(int) * T));
        LF_TRY(lf_dev_alloc(h, (void **)&h->occ_key, sizeof(unsigned long long) * T));
        LF_TRY(lf_dev_alloc(h, (void **)&h->occ_d, sizeof(double) * T));
        LF_HIP(h, hipMemsetAsync(h->gt, 0, sizeof(GEntry) * T, st));
        h->second_half_work = true;
        hipLaunchKernelGGL(k_empty_table, dim3(grid_for(T, BS)), dim3(BS), 0, st, h->gt, T);
        h->gT = T;
        moved = true;
    }
    long long pcap = 2 * q + (h->cm_cap + n) / PART + 64;
    if (pcap > h->part_cap) {
        if (h->phase_graphs) pcap *= 2;
        lf_dev_free(h, h->part_rec);
        h->part_rec = nullptr;
        LF_TRY(lf_dev_alloc(h, (void **)&h->part_rec, sizeof(PartRec) * pcap));
        h->part_cap = pcap;
        moved = true;
    }
    long long mcap = 2 * q + 64;
    if (mcap > h->mslot_cap) {
        lf_dev_free(h, h->macc);
        h->macc = nullptr;
        LF_TRY(lf_dev_alloc(h, (void **)&h->macc, sizeof(long long) * MACC * mcap));
        h->mslot_cap = mcap;
        moved = true;
    }
    if (moved) h->graph_version++;
    return LF_OK;
}

// Start of an iteration: buffers and path lists for queues of qq nodes, counters reset.
// lf_iter_begin_enqueue queues the work; lf_iter_begin_complete must follow once it is done
// (after a stream sync or a completed event recorded behind it).
static int begin_enqueue_plain(lf_handle *h, long long qq)
{
    LF_TRY(size_queue_enqueue(h, qq));
    if (h->n > 0) {
        if (!h->lines) {
            LF_TRY(lf_dev_alloc(h, (void **)&h->lines, sizeof(NodeLine) * h->n));
            h->graph_version++;
        }
        hipLaunchKernelGGL(k_line_build, dim3(grid_for(h->n, 256)), dim3(256), 0, h->stream, lf_ctx(h));
    }
    LF_TRY(lf_zero(h, &h->ctr->joins, sizeof(unsigned long long) * 2));
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(WAVE), 0, h->stream, lf_ctx(h));
    return LF_OK;
}

// ---- iteration starts and ends replayed from graphs --------------------------------
// A member of a batch repeats the same launch sequence at every iteration start (and end):
// the same buffers, sizes and temporaries, with only the slot buffer alternating.  A run
// that will allocate nothing (the host makes the run's own size checks first) is captured
// and later runs in the same state replay the graph: one host call for some thirty
// launches and copies.  The key covers whatever the launches bake in (the Ctx, every
// allocation, the temporaries' position, the options the start reads, the queue size and
// the slot parity); after a change the next run is captured again (the graph is updated
// in place).
static int finish_enqueue_plain(lf_handle *h);

static unsigned long long fnv_add(unsigned long long k, const void *p, size_t n)
{
    const unsigned char *b = (const unsigned char *)p;
    for (size_t i = 0; i < n; i++) k = (k ^ b[i]) * 1099511628211ull;
    return k;
}

static unsigned long long phase_key(lf_handle *h, long long qq, int which)
{
    unsigned long long k = 14695981039346656037ull;
    Ctx cx = lf_ctx(h);
    cx.qtag = 0;
    // the path lists' record pointers move with the path counts at every start and are
    // read only by the queue kernels
    for (int c = 0; c < LF_PATH_COUNT; c++) cx.prec[c] = nullptr;
    k = fnv_add(k, &cx, sizeof cx);
    const long long v[] = {which, qq, h->cur, h->profiling, h->tmp_chunk, (long long)h->tmp_off,
                           h->eval_wave_cap, h->eval_med_cap, h->eval_grp_cap,
                           (long long)h->allocs->size(), (long long)h->tmp_chunks->size()};
    k = fnv_add(k, v, sizeof v);
    k = fnv_add(k, h->allocs->data(), sizeof(void *) * h->allocs->size());
    k = fnv_add(k, h->alloc_sizes->data(), sizeof(size_t) * h->alloc_sizes->size());
    for (const TmpChunk &c : *h->tmp_chunks) k = fnv_add(k, &c, sizeof c);
    const void *hp[] = {h->hqoff, h->hrep};
    k = fnv_add(k, hp, sizeof hp);
    return k;
}

void lf_phase_graphs_drop(lf_handle *h)
{
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) {
            if (h->pg[a][b].exec) (void)hipGraphExecDestroy(h->pg[a][b].exec);
            h->pg[a][b].exec = nullptr;
            h->pg[a][b].key = 0;
        }
}

// capture one plain run of the start (which = 0) or end (1) on the capture stream; the
// host-side effects of the run (slot parity, start bookkeeping) happen as in a plain run.
// *exec, if set, is updated in place when the new graph has its shape (a moved buffer
// changes only kernel arguments), else replaced.
static int capture_phase(lf_handle *h, int which, long long qq, hipGraphExec_t *exec)
{
    if (!h->cap_stream) LF_HIP(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    hipStream_t saved = h->stream;
    LF_HIP(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    h->stream = h->cap_stream;
    int rc = which == 0 ? begin_enqueue_plain(h, qq) : finish_enqueue_plain(h);
    h->stream = saved;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
    if (rc == LF_OK && (e != hipSuccess || !g)) rc = lf_set_error(h, LF_EDEVICE, "iteration phase capture failed");
    if (rc == LF_OK && *exec) {
        hipGraphNode_t err_node = nullptr;
        hipGraphExecUpdateResult res;
        if (hipGraphExecUpdate(*exec, g, &err_node, &res) != hipSuccess || res != hipGraphExecUpdateSuccess) {
            (void)hipGetLastError();
            (void)hipGraphExecDestroy(*exec);
            *exec = nullptr;
        }
    }
    if (rc == LF_OK && !*exec && hipGraphInstantiate(exec, g, nullptr, nullptr, 0) != hipSuccess) {
        *exec = nullptr;
        rc = lf_set_error(h, LF_EDEVICE, "iteration phase graph instantiation failed");
    }
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return rc;
}

// whether a start (0) or end (1) would allocate: its size checks, made on the host
// beforehand (the temporaries it takes exist once it has run plainly)
static bool phase_allocates(lf_handle *h, int which, long long qq)
{
    if (!h->phase_ran[which]) return true;
    const long long n = h->n;
    if (which == 1) return !h->cm_node || h->slot_used + n + 1 > h->slot_capb[1 - h->cur];
    const long long nq = (n + qq - 1) / qq;
    const long long nrep = REP_LEN(nq);
    const long long ucap = n + 2 * h->ne / INB + 1;
    return qq > h->q_cap || h->hqoff_cap < nq + 1 || nrep > h->dq_cap || !h->titem_base || !h->titem_node ||
           ucap > h->unit_cap || (n > 0 && !h->lines);
}

// one iteration start (0) or end (1), from a graph where the state allows
static int run_phase(lf_handle *h, int which, long long qq)
{
    if (!h->phase_graphs || h->profiling) {
        h->phase_runs[0]++;
        h->phase_ran[which] = 1;
        return which == 0 ? begin_enqueue_plain(h, qq) : finish_enqueue_plain(h);
    }
    PhaseGraph &pg = h->pg[which][h->cur];
    const unsigned long long key = phase_key(h, qq, which);
    const bool allocates = phase_allocates(h, which, qq);
    if (!allocates && pg.exec && pg.key == key) {
        LF_HIP(h, hipGraphLaunch(pg.exec, h->stream));
        h->phase_runs[2]++;
        if (which == 0) {
            h->pending_moved = false;
            h->fill_grid = pg.fill_grid;
        } else {
            h->cur = 1 - h->cur;
        }
        return LF_OK;
    }
    if (!allocates) {
        LF_TRY(capture_phase(h, which, qq, &pg.exec));
        pg.key = key;
        pg.fill_grid = h->fill_grid;
        LF_HIP(h, hipGraphLaunch(pg.exec, h->stream));
        h->phase_runs[1]++;
        return LF_OK;
    }
    h->phase_runs[0]++;
    h->phase_ran[which] = 1;
    return which == 0 ? begin_enqueue_plain(h, qq) : finish_enqueue_plain(h);
}

int lf_iter_begin_enqueue(lf_handle *h, long long qq) { return run_phase(h, 0, qq); }

int lf_iter_finish_enqueue(lf_handle *h) { return run_phase(h, 1, 0); }

int lf_iter_begin_complete(lf_handle *h, long long qq, long long *nq)
{
    LF_TRY(size_queue_complete(h, qq));
    *nq = (h->n + qq - 1) / qq;
    return LF_OK;
}

int lf_iter_begin(lf_handle *h, long long qq, long long *nq)
{
    LF_TRY(lf_iter_begin_enqueue(h, qq));
    LF_HIP(h, hipStreamSynchronize(h->stream));
    return lf_iter_begin_complete(h, qq, nq);
}

// Parameters and grids of queue k (of nq).  compact_grids sizes the grid-stride kernels by
// the queue instead of by the whole device (for many graphs sharing one launch).
void lf_queue_params(lf_handle *h, long long k, long long nq, long long qq, bool compact_grids, QStep *qs,
                     QGrids *g)
{
    const long long *qo = h->hqoff;                                // [path][nq + 1]
    const long long *hit = h->hqoff + REP_ITEMS(nq);   // first table-path work item per queue
    const long long *hu = h->hqoff + REP_UNITS(nq);    // first in-count unit per queue
    const long long start = k * qq;
    const int clen = (int)((h->n - start) < qq ? (h->n - start) : qq);
    int ls[LF_PATH_COUNT], ln[LF_PATH_COUNT];
    for (int c = 0; c < LF_PATH_COUNT; c++) {
        ls[c] = (int)qo[c * (nq + 1) + k];
        ln[c] = (int)(qo[c * (nq + 1) + k + 1] - ls[c]);
    }
    const int gb = h->hub_blocks;
    int rbk = h->refresh_blocks;
    if (compact_grids) {
        int want = (int)grid_for(clen, 8);
        if (want < rbk) rbk = want;
    }
    qs->cstart = (int)start;
    qs->clen = clen;
    qs->wcap = h->eval_wave_cap < 2 * VSMALL ? h->eval_wave_cap : 2 * VSMALL;
    qs->mcap = h->eval_med_cap;
    qs->gcap = h->eval_grp_cap;
    qs->ls = ls[LF_PATH_SMALL];
    qs->ln = ln[LF_PATH_SMALL];
    BigRoles &br = qs->br;
    const long long titems = hit[k + 1] - hit[k];
    br.bt = ln[LF_PATH_TABLE] > 0 ? (int)grid_for(titems, 2 * EWB * WAVE) : 0;
    if (br.bt > gb) br.bt = gb;
    br.bg = ln[LF_PATH_GROUP] < gb ? ln[LF_PATH_GROUP] : gb;
    // a single graph's medium-path nodes take one k_eval block each (one visit per thread,
    // seven blocks per CU); in a multi-graph step they are a role of k_eval_big (one wave
    // per node), as is everything there
    const bool own_med = !compact_grids;
    br.bm = own_med ? 0 : (int)grid_for(ln[LF_PATH_MED], GT / WAVE);
    // a queue with many small-path nodes gives them blocks of k_eval too (more blocks per
    // CU than the fused kernel's LDS allows); otherwise they are a role of k_eval_big
    const bool own_small = !compact_grids && ln[LF_PATH_SMALL] >= SMALL_OWN_LAUNCH;
    br.ns = own_small ? 0 : ln[LF_PATH_SMALL];
    br.bs = (int)grid_for(br.ns, GT / WAVE);
    br.lt = ls[LF_PATH_TABLE];
    br.nt = ln[LF_PATH_TABLE];
    br.lg = ls[LF_PATH_GROUP];
    br.ng = ln[LF_PATH_GROUP];
    br.lm = ls[LF_PATH_MED];
    br.nm = own_med ? 0 : ln[LF_PATH_MED];
    qs->ub = hu[k];
    qs->un = (int)(hu[k + 1] - hu[k]);
    qs->es = own_small ? (int)grid_for(ln[LF_PATH_SMALL], EW) : 0;
    qs->em = own_med ? ln[LF_PATH_MED] : 0;
    g->eval = qs->es + qs->em;
    g->big = br.bt + br.bg + br.bm + br.bs;
    if (g->big < 1 && g->eval == 0) g->big = 1;   // block 0 resets the queue's counters
    g->fin = ln[LF_PATH_TABLE] > 0 ? (compact_grids ? (br.bt > 0 ? br.bt : 1) : gb) : 0;
    g->apply = (int)grid_for(clen, 256) + (int)grid_for(qs->un, 256 / WAVE);
    g->refresh = rbk;
}

// the kernels of one queue of one graph, in order, on the handle's stream
int lf_launch_queue(lf_handle *h, Ctx &cx, const QStep &qs, const QGrids &g)
{
    hipStream_t st = h->stream;
    cx.qtag = h->qtag++;
    if (g.eval > 0) {
        LF_TRY(lf_prof_begin(h, LF_K_EVAL));
        hipLaunchKernelGGL(k_eval, dim3(g.eval), dim3(EW * WAVE), 0, st, cx, qs);
        LF_TRY(lf_prof_end(h, LF_K_EVAL, 1));
    }
    if (g.big > 0) {
        LF_TRY(lf_prof_begin(h, LF_K_EVAL_BIG));
        hipLaunchKernelGGL(k_eval_big, dim3(g.big), dim3(GT), 0, st, cx, qs);
        LF_TRY(lf_prof_end(h, LF_K_EVAL_BIG, 1));
    }
    if (g.fin > 0) {
        LF_TRY(lf_prof_begin(h, LF_K_TAB_FINAL));
        hipLaunchKernelGGL(k_big_final, dim3(g.fin), dim3(256), 0, st, cx, qs);
        LF_TRY(lf_prof_end(h, LF_K_TAB_FINAL, 1));
        LF_TRY(lf_prof_begin(h, LF_K_TAB_TIE));
        hipLaunchKernelGGL(k_big_tie, dim3(g.fin), dim3(256), 0, st, cx, qs);
        LF_TRY(lf_prof_end(h, LF_K_TAB_TIE, 1));
    }
    LF_TRY(lf_prof_begin(h, LF_K_APPLY_EDIT));
    hipLaunchKernelGGL(k_apply, dim3(g.apply), dim3(256), 0, st, cx, qs);
    LF_TRY(lf_prof_end(h, LF_K_APPLY_EDIT, 1));
    LF_TRY(lf_prof_begin(h, LF_K_REFRESH));
    hipLaunchKernelGGL(k_refresh, dim3(g.refresh), dim3(256), 0, st, cx, qs);
    LF_TRY(lf_prof_end(h, LF_K_REFRESH, 1));
    h->prof.chunks++;
    h->prof.node_evals += qs.clen;
    return LF_OK;
}

// One queue of each of nm graphs: four grids (k_big_final and k_big_tie share one), each
// block finding its graph from dboff (LF_MULTI_GRIDS arrays of first-block offsets, at
// stride cap + 1, each with nm + 1 entries); total[i] = blocks of grid i.
int lf_launch_multi(hipStream_t st, const Member *dmem, const int *dboff, int cap, int nm, const int *total)
{
    const int *o = dboff;
    if (total[0] > 0) hipLaunchKernelGGL(k_eval_big_multi, dim3(total[0]), dim3(GT), 0, st, dmem, o, nm);
    o += cap + 1;
    if (total[1] > 0) {
        hipLaunchKernelGGL(k_big_final_multi, dim3(total[1]), dim3(256), 0, st, dmem, o, nm);
        hipLaunchKernelGGL(k_big_tie_multi, dim3(total[1]), dim3(256), 0, st, dmem, o, nm);
    }
    o += cap + 1;
    if (total[2] > 0) hipLaunchKernelGGL(k_apply_multi, dim3(total[2]), dim3(256), 0, st, dmem, o, nm);
    o += cap + 1;
    if (total[3] > 0) hipLaunchKernelGGL(k_refresh_multi, dim3(total[3]), dim3(256), 0, st, dmem, o, nm);
    return hipGetLastError() == hipSuccess ? LF_OK : LF_EDEVICE;
}

// The multi-graph kernels in launch order, the grid each uses and its block size, for
// building a graph of one batch step.
void lf_multi_kernels(const void **fn, int *grid, int *block)
{
    const void *f[LF_MULTI_KERNELS] = {(const void *)k_eval_big_multi, (const void *)k_big_final_multi,
                                       (const void *)k_big_tie_multi, (const void *)k_apply_multi,
                                       (const void *)k_refresh_multi};
    const int gr[LF_MULTI_KERNELS] = {0, 1, 1, 2, 3};
    const int b[LF_MULTI_KERNELS] = {GT, 256, 256, 256, 256};
    for (int i = 0; i < LF_MULTI_KERNELS; i++) {
        fn[i] = f[i];
        grid[i] = gr[i];
        block[i] = b[i];
    }
}

// End of an iteration: counters reset, degenerate communities removed, exact score.
// End of an iteration, in the same two halves as its start.
// the membership lines back into the slot layout (a batch member leaving mid-iteration)
int lf_lines_back(lf_handle *h)
{
    if (h->n > 0 && h->lines)
        hipLaunchKernelGGL(k_line_back, dim3(grid_for(h->n, 256)), dim3(256), 0, h->stream, lf_ctx(h));
    return hipGetLastError() == hipSuccess ? LF_OK : LF_EDEVICE;
}

static int finish_enqueue_plain(lf_handle *h)
{
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(WAVE), 0, h->stream, lf_ctx(h));
    if (h->n > 0) hipLaunchKernelGGL(k_line_back, dim3(grid_for(h->n, 256)), dim3(256), 0, h->stream, lf_ctx(h));
    LF_HIP(h, hipGetLastError());
    LF_TRY(lf_prof_begin(h, LF_K_ITEREND));
    LF_TRY(lf_iteration_end_enqueue(h));
    LF_TRY(lf_prof_end(h, LF_K_ITEREND, 8));
    return LF_OK;
}

int lf_iter_finish_complete(lf_handle *h, long long *joins, long long *leaves, long long *live)
{
    LF_TRY(lf_iteration_end_complete(h, joins, leaves, live));
    return lf_dev_error_status(h, h->last_dev_error);   // the flags came with the iteration-end report
}

int lf_iter_finish(lf_handle *h, long long *joins, long long *leaves, long long *live)
{
    LF_TRY(lf_iter_finish_enqueue(h));
    LF_HIP(h, hipStreamSynchronize(h->stream));
    return lf_iter_finish_complete(h, joins, leaves, live);
}

int lf_iterate(lf_handle *h, int q, double theta, int max_iters, lf_run_info *out)
{
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
    double prev = h->Wt;
    for (int it = 0; it < max_iters; it++) {
        long long nq = 0;
        LF_TRY(lf_iter_begin(h, qq, &nq));
        Ctx cx = lf_ctx(h);
        for (long long k = 0; k < nq; k++) {
            QStep qs;
            QGrids g;
            lf_queue_params(h, k, nq, qq, false, &qs, &g);
            LF_TRY(lf_launch_queue(h, cx, qs, g));
        }
        long long joins = 0, leaves = 0, live = 0;
        LF_TRY(lf_iter_finish(h, &joins, &leaves, &live));
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
    LF_TRY(lf_prof_flush(h));
    {
        unsigned long long w[LF_PATH_COUNT][5], aw[LF_APPLY_COUNT];
        LF_HIP(h, hipMemcpy(w, h->ctr->work, sizeof(w), hipMemcpyDeviceToHost));
        LF_HIP(h, hipMemcpy(aw, h->ctr->apply, sizeof(aw), hipMemcpyDeviceToHost));
        for (int k = 0; k < LF_APPLY_COUNT; k++) h->prof.apply_work[k] = (long long)aw[k];
        h->prof.visits = 0;
        h->prof.candidates = 0;
        for (int p = 0; p < LF_PATH_COUNT; p++) {
            h->prof.path_nodes[p] = (long long)w[p][0];
            h->prof.path_neighbours[p] = (long long)w[p][1];
            h->prof.path_visits[p] = (long long)w[p][2];
            h->prof.path_candidates[p] = (long long)w[p][3];
            h->prof.path_own[p] = (long long)w[p][4];
            h->prof.visits += (long long)w[p][2];
            h->prof.candidates += (long long)w[p][3];
        }
    }
    out->wtilde = h->Wt;
    out->wcc_hat = h->Wt / h->cc;
    return LF_OK;
}
