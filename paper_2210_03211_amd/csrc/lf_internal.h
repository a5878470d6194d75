// lf_internal.h -- handle layout and host helpers shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "lazyfox.h"
#include "exact.h"

// Membership record of one node: its slot range in the slot array and its degree.
struct NodeHdr {
    long long off;   // first slot
    int cnt;         // memberships in use
    int deg;         // degree
};

// One membership slot: community id and in = |N(x) ∩ C|.
struct Slot {
    int comm;
    int in;
};

// One node's memberships for the queue kernels, one 64-byte line: membership count,
// degree and up to LINE_SLOTS memberships inline (off = -1); a node whose slot capacity
// exceeds LINE_SLOTS keeps its memberships in the slot array from `off` on.  The lines
// are built from the slot layout at every iteration start and written back at its end,
// so within an iteration one gather of a node's line serves its whole membership list.
#define LINE_SLOTS 6
struct __align__(64) NodeLine {
    int cnt;
    int deg;
    long long off;           // -1: memberships inline; else the first slot in the slot array
    Slot s[LINE_SLOTS];
};
static_assert(sizeof(NodeLine) == 64, "one 64-byte line per node");

// One in-count unit: up to INB consecutive neighbours of the node at order position r
// (units are laid out for every node at the start of an iteration, so a queue's units are
// a contiguous range; the apply step skips those of nodes that did not move).
struct UnitRec {
    long long rb;            // adjacency position of the unit's first neighbour
    int x;                   // the node
    int r;                   // its order position
    int cnt;                 // neighbours in the unit (1 .. INB)
    int pad;
};

// One re-sum part: up to PART entries of a touched community's member list, planned at
// the community's first touch in a queue from the list's capacity (fixed within an
// iteration); size, list length and overflow are read when the part is summed.
struct PartRec {
    long long base;          // the community's member-list offset
    int C;                   // the community (-1: an empty record after a flagged overflow)
    int k, parts;            // this part and the community's number of parts
    int cap;                 // member-list capacity
    int ms;                  // carry-save counter slot of a multi-part community (-1: one part)
    int pad;
};

// A node of a path list with what its evaluation reads first (row offset, id, degree), so
// that its adjacency gathers can start without first resolving the order position.
struct NodeRec {
    long long rb;    // first adjacency position
    int x;           // node id
    int d;           // degree
};

// One community, one 64-byte line: everything a candidate evaluation reads.  The exact
// sums S+ / S- (sum of g over the members at size s+1 / s-1) are stored as 160-bit
// non-negative fixed point (lowest bit 2^-120; every such sum is below 2^31).
struct __align__(64) CommRec {
    int s;                 // members
    int pad;
    long long m;           // internal edges
    double W;              // cc-free score fl(p * R(sum g))
    unsigned Sp[5];
    unsigned Sm[5];
};

// One entry of the table path's global hash table, one 64-byte line: key (node, community),
// neighbour count, the first visiting neighbour's (in-count, degree) kept inline (its
// correction is computed when the entry is finalised), and four correction digits for
// every later visit.
struct __align__(64) GEntry {
    unsigned long long key;
    int cnt;
    int ii;                // inline visit: in-count of the neighbour
    int idy;               // inline visit: degree of the neighbour (0 = none)
    int pad;
    long long d[4];
    long long pad2;
};

// Device-side counters and flags (one struct in device memory).  The per-queue counters
// are reset by the first kernel of every queue.
struct DevCounters {
    unsigned long long joins;      // per iteration
    unsigned long long leaves;     // per iteration
    unsigned long long work[LF_PATH_COUNT][5]; // evaluation work per path (cumulative): nodes,
                                   // neighbours, visits, candidates, own memberships
    unsigned long long apply[LF_APPLY_COUNT];  // apply work (cumulative, LF_APPLY_*)
    int tcount;                    // communities re-summed at initialisation
    int unused0;
    int unused1;
    int occ_cnt;                   // occupied entries of the global table (queue)
    int unused2;
    int parts_total;               // re-sum parts (queue)
    int mslots;                    // multi-part re-sum accumulators in use (queue)
    int refresh_next;              // work counter of the full re-sum at initialisation
    int ovf_cnt;                   // joiners that did not fit their member list (iteration)
    int undecided;                 // initial clustering rounds
    int error;                     // bit flags, see LF_DEVERR_*
    int live;                      // communities with >= 2 members (iteration end)
    int max_mem;                   // largest membership count (iteration end)
    int pad[3];
    X256 score;
};

#define LF_DEVERR_INEXACT 1        // a value did not fit the exact accumulator
#define LF_DEVERR_INCOUNT 2        // in-count bookkeeping disagreed with a recount
#define LF_DEVERR_ODD 4            // odd internal-degree sum
#define LF_DEVERR_SLOTS 8          // a node ran out of membership slots
#define LF_DEVERR_CAP 16           // a per-queue work buffer was sized too small

// Everything a kernel needs, passed by value.
struct Ctx {
    long long n;
    int K;
    const long long *rowptr;
    const int *col;
    const int *deg;
    const int *order;
    NodeHdr *nh;
    Slot *slot;
    NodeLine *ln;            // per-node membership lines (within an iteration)
    CommRec *cr;             // community records
    long long *cm_off;       // member-list capacity offsets (K + 1)
    int *cm_len;             // member-list fill (may exceed capacity: overflow)
    int *cm_node;            // member lists
    int *tflag;              // touched flag per community (1: in this queue, 2: removed)
    int *tlist;              // community list of the re-sum at initialisation
    unsigned qtag;           // tag of the current queue (unique within a run)
    int *ovf_node;           // overflow joiners (node, community)
    int *ovf_comm;
    int *ovf_flag;
    int *dj, *dl;            // decisions of the current queue
    double *djd, *dld;
    int *dpos;               // [q] slot count of each queued node when it was evaluated
                             // (where a join is appended)
    DevCounters *ctr;
    // table path (nodes whose candidates do not fit one wave), indexed by queue position j
    int *big_idx;            // [q] evaluation state of queue index j (Q_* in iterate.hip)
    // evaluation path of every node for the current iteration: per path the order
    // positions of its nodes, ascending (a queue's nodes of a path are contiguous)
    int *plist[LF_PATH_COUNT];
    const NodeRec *prec[LF_PATH_COUNT];   // parallel to plist: the node's record
    const int *rank;         // [n] order position of each node
    const int *col_rank;     // [2 ne] order position of col[e], beside col
    long long *titem_base;   // [table-path nodes + 1] first work item of each
    int *titem_node;         // [items] table-path list position owning each item
    unsigned long long *big_bj, *big_bl;   // [q] best join / leave change (bits; 0 = none)
    int *big_cj, *big_cl;    // [q] lowest community id among the best
    NodeLine *big_ln;        // [q] a table-path node's line at the queue start
    GEntry *gt;                // [gT] key (j << 32 | C), empty = ~0
    int *occ;                  // [gT] occupied entries
    unsigned long long *occ_key;  // [gT] key | leave << 63
    double *occ_d;             // [gT] change of each occupied entry
    long long gmask;           // gT - 1
    // in-count units of the current iteration (every node's, in node order)
    const UnitRec *unit;
    // re-sum parts
    PartRec *part_rec;       // [part_cap] the re-sum parts of the queue
    int *part_done;          // [K] parts of a multi-part community finished
    long long *macc;         // [mslot_cap * 19] carry-save accumulators
    int part_cap, mslot_cap;
    int stats;               // collect the per-path work counters
};

// Block roles of k_eval_big: [0, bt) walk the table-path work items, the next bg blocks
// evaluate workgroup-path nodes (one node per block at a time), the last bm blocks
// medium-path nodes (one node per wave).
struct BigRoles {
    int bt, bg, bm, bs;      // blocks per role (table, workgroup, medium, small)
    int ns;                  // small-path nodes in this launch (the rest: k_eval)
    int lt, nt;              // table-path list positions of the queue
    int lg, ng;              // workgroup-path list positions
    int lm, nm;              // medium-path list positions
};

// Everything the kernels of one queue need besides the graph's Ctx.
struct QStep {
    int cstart, clen;        // the queue: order positions [cstart, cstart + clen)
    int wcap, mcap, gcap;    // LDS table sizes of the small, medium and workgroup paths
    int ls, ln;              // small-path list positions
    int es, em;              // k_eval: blocks of small-path nodes (four per block), then one
                             // block per medium-path node (the first em of list br.lm)
    BigRoles br;
    long long ub;            // the queue's in-count units: [ub, ub + un)
    int un;
};

// One graph's queue in a multi-graph launch.
struct Member {
    Ctx cx;
    QStep qs;
};

// launch grids of one queue's kernels (0 = not launched)
struct QGrids {
    int eval, big, fin, apply, refresh;
};

struct TmpChunk {
    void *ptr;
    size_t size;
};

struct TmpMark {
    int chunk;
    size_t off;
};

// An iteration start or end captured into a graph, for one slot-buffer parity: key of
// the state it was captured in, and what the start leaves on the host.
struct PhaseGraph {
    unsigned long long key;
    hipGraphExec_t exec;
    unsigned fill_grid;
};

struct lf_handle {
    int device;
    hipStream_t stream;
    bool own_stream;
    char err[512];
    int state;               // 0 empty, 1 graph loaded, 2 communities initialised
    long long n, ne;
    int K;
    int max_deg;
    // graph
    long long *rowptr;
    int *col;
    int *deg;
    long long *orig_id;      // device, n entries (identity without relabel)
    // node statistics
    unsigned long long *tri;
    double *ccl;
    int *order;
    int *rank;
    int *col_rank;
    double cc;
    long long T;
    // partition
    NodeHdr *nh;
    Slot *slot[2];
    NodeLine *lines;         // [n] membership lines of the current iteration
    int cur;
    long long slot_capb[2];  // capacity of each slot buffer
    CommRec *cr;
    long long *cm_off;
    int *cm_len;
    int *cm_node;
    long long cm_cap;        // capacity of cm_node
    int *tflag, *tlist;
    unsigned qtag;           // next queue tag
    int *ovf_node, *ovf_comm, *ovf_flag;
    int *dj, *dl;
    double *djd, *dld;
    int *dpos;
    long long q_cap;         // capacity of the per-queue arrays
    // table path and work lists (sized per iteration)
    int *big_idx;
    int *cls;                // [n] evaluation path per order position (this iteration)
    long long *cscan;        // [n + 1] scan scratch of the path lists
    int *plist[LF_PATH_COUNT];
    NodeRec *prec_all;       // [n] node records of all path lists, path after path
    long long *pbase;        // [LF_PATH_COUNT + 1] device: first record of each path
    NodeRec *prec[LF_PATH_COUNT];   // host-set views into prec_all
    long long *titem_base;
    int *titem_node;
    long long titem_cap;
    long long *hqoff;        // pinned host: [LF_PATH_COUNT][nq + 1] first list position per
                             // queue, then [nq + 1] first table-path work item per queue,
                             // then the 4 bounds of k_chunk_bounds
    long long hqoff_cap;     // queues (nq + 1) it has room for
    long long hqoff_len;     // its length in long longs (as allocated)
    long long *hrep;         // pinned host report of an iteration end (REP_* entries)
    long long slot_used;     // slot entries of the current layout (nh[n].off)
    int last_dev_error;      // device error flags read with the last iteration-end report
    long long *dq;           // [dq_cap] device: what the iteration start copies to hqoff
    long long dq_cap;
    bool pending_moved;      // buffers moved in the first half of an iteration start
    bool second_half_work;   // the second half of the last start queued device work
    unsigned fill_grid;      // grid of the table work-item fill of that start
    unsigned long long *big_bj, *big_bl;
    int *big_cj, *big_cl;
    NodeLine *big_ln;
    GEntry *gt;
    int *occ;
    unsigned long long *occ_key;
    double *occ_d;
    long long gT;
    UnitRec *unit;           // [unit_cap] in-count units of the iteration
    long long unit_cap;
    PartRec *part_rec;
    int *part_done;
    long long *macc;
    long long part_cap, mslot_cap;
    long long *vbound;       // [n] per-node bounds used to size the per-queue buffers
    int graph_version;       // bumped whenever a buffer used by captured launches moves
    DevCounters *ctr;
    double Wt;               // cc-free partition score
    // tuning
    int eval_wave_cap;       // table entries per wave in the small wave path
    int eval_med_cap;        // table entries per wave in the medium wave path
    int eval_grp_cap;        // table entries per workgroup in the workgroup path
    int tri_lds_cap;         // 0 = auto
    int hub_blocks;          // workgroups of the table-path evaluation kernels
    int refresh_blocks;      // workgroups of the in-count and re-sum kernels
    // profiling
    int profiling;           // bit mask of timed kernel classes (1 << LF_K_*)
    int prof_stride;         // bracket every prof_stride-th launch of a per-queue class
    long long prof_seq[LF_K_COUNT];   // launches of each class seen while timing
    int prof_skip;           // classes whose current launch is not bracketed (bit mask)
    lf_profile prof;
    hipEvent_t ev0, ev1;
    std::vector<hipEvent_t> *evpool;   // start/stop pairs recorded without host sync
    std::vector<int> *evkind;          // kernel class of each recorded pair
    std::vector<int> *evlaunch;        // launches bracketed by each pair
    int evused;                        // pairs recorded and not yet folded into prof
    // allocation registry
    std::vector<void *> *allocs;
    std::vector<size_t> *alloc_sizes;
    std::vector<TmpChunk> *tmp_chunks;      // scratch arena (lf_tmp_alloc)
    int tmp_chunk;
    size_t tmp_off;
    size_t dev_bytes, dev_bytes_peak;   // device memory the handle holds (now / at most)
    // iteration starts and ends replayed from graphs (members of a batch)
    int phase_graphs;
    PhaseGraph pg[2][2];                // [start, end][slot parity]
    long long phase_runs[3];            // starts and ends run plainly, captured, replayed
    int phase_ran[2];                   // a start / an end has run plainly (its temporaries exist)
    hipStream_t cap_stream;             // the stream they are captured on
};

// ---- host helpers --------------------------------------------------------------------
int lf_set_error(lf_handle *h, int code, const char *fmt, ...);

#define LF_HIP(h, expr)                                                                    \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return lf_set_error((h), LF_EDEVICE, "%s failed: %s (%s:%d)", #expr,           \
                                hipGetErrorString(e_), __FILE__, __LINE__);                \
    } while (0)

#define LF_TRY(expr)                                                                       \
    do {                                                                                   \
        int rc_ = (expr);                                                                  \
        if (rc_ != LF_OK) return rc_;                                                      \
    } while (0)

int lf_dev_alloc(lf_handle *h, void **p, size_t bytes);
void lf_dev_free(lf_handle *h, void *p);
// size an lf_dev_alloc request occupies; a block whose device work has completed goes
// back to the per-device cache (or to HIP)
size_t lf_alloc_class(size_t bytes);
void lf_dev_release(int device, void *p, size_t bytes);
int lf_host_alloc(void **p, size_t bytes);       // pinned, from the same kind of cache
int lf_zero(lf_handle *h, void *p, size_t bytes); // kernel fill on h->stream (bytes % 4 == 0)
void lf_phase_graphs_drop(lf_handle *h);
extern "C" int lf_batch_detach(lf_batch *b, int32_t member_id, hipEvent_t *left);
void lf_host_release(void *p, size_t bytes);
int lf_tmp_alloc(lf_handle *h, void **p, size_t bytes);
TmpMark lf_tmp_mark(lf_handle *h);
void lf_tmp_release(lf_handle *h, TmpMark m);
// temporaries of the enclosing scope come from the arena and go back at its end
struct TmpScope {
    lf_handle *h;
    TmpMark m;
    explicit TmpScope(lf_handle *hh) : h(hh), m(lf_tmp_mark(hh)) {}
    ~TmpScope() { lf_tmp_release(h, m); }
};
Ctx lf_ctx(lf_handle *h);

// profiling brackets around a launch sequence on the handle's stream; events are only
// resolved by lf_prof_flush (end of an API call), so timing never stalls the host
int lf_prof_begin(lf_handle *h, int kind);
int lf_prof_end(lf_handle *h, int kind, int launches);
int lf_prof_begin_on(lf_handle *h, int kind, hipStream_t st);
int lf_prof_end_on(lf_handle *h, int kind, int launches, hipStream_t st);
int lf_prof_flush(lf_handle *h);

// ---- primitives (prims.hip) ------------------------------------------------------------
int lf_sort_u64(lf_handle *h, unsigned long long *keys, unsigned long long *keys_alt, long long n,
                int end_bit, unsigned long long **result);
int lf_sort_pairs_u64_i32(lf_handle *h, unsigned long long *keys, unsigned long long *keys_alt,
                          int *vals, int *vals_alt, long long n, int end_bit,
                          unsigned long long **rkeys, int **rvals);
int lf_sort_pairs_u32_i32(lf_handle *h, unsigned *keys, unsigned *keys_alt, int *vals,
                          int *vals_alt, long long n, unsigned **rkeys, int **rvals);
int lf_exclusive_scan_i64(lf_handle *h, const long long *in, long long *out, long long n);
int lf_exclusive_scan_i32_to_i64(lf_handle *h, const int *in, long long *out, long long n);
int lf_sort_dev_u64(lf_handle *h, unsigned long long *keys, int *vals, long long n, int end_bit);
int lf_sort_dev_u32(lf_handle *h, unsigned *keys, int *vals, long long n);
int lf_scan_dev(lf_handle *h, const void *in, int in_bytes, long long *out, long long n);

// ---- graph stages (graph.hip) ------------------------------------------------------------
int lf_build_graph(lf_handle *h, long long n, long long npairs, const long long *src,
                   const long long *dst, unsigned flags);
int lf_node_stats(lf_handle *h);
int lf_exact_sum_dev(lf_handle *h, const double *v, long long n, double *out);
#define LF_EXACT_PARTIALS 1024     // block partial sums of the exact sum (fixed grid)
int lf_exact_sum_run(lf_handle *h, const double *v, long long n, double *out, X192 *part, int *err, double *dout);

// ---- community stages (communities.hip) ----------------------------------------------------
// Exact-WCC pass over the triangles (wcc_hit in graph.hip): compact sorted memberships
// (node x's community ids at [moff[x], moff[x + 1])), per-membership triangle counters and
// per-oriented-edge "closes a triangle" flags.
struct WccTri {
    const long long *moff;
    const int *mid;
    int *tcm;
    unsigned char *eflag;
};
int lf_triangle_pass(lf_handle *h, const WccTri *wt, int *launches, long long **oro_out, int **orc_out);

int lf_initial_clustering(lf_handle *h);
int lf_partition_from_cover(lf_handle *h, const long long *off, const int *ids, long long total, int n_comms);
int lf_check_cover(lf_handle *h, const long long *off, const int *ids, long long total, int n_comms, int *maxid);
int lf_iterate(lf_handle *h, int q, double theta, int max_iters, lf_run_info *out);
// one LazyFox iteration split into its host steps (shared by lf_run_iterations and the
// multi-graph batch): sizing and path lists, per-queue parameters, and the iteration end
int lf_iter_begin(lf_handle *h, long long qq, long long *nq);
// the same in two halves: work queued on the handle's stream, then the host's part once
// that work is done (a stream sync or a completed event behind it)
int lf_iter_begin_enqueue(lf_handle *h, long long qq);
int lf_iter_begin_complete(lf_handle *h, long long qq, long long *nq);
void lf_queue_params(lf_handle *h, long long k, long long nq, long long qq, bool compact_grids, QStep *qs,
                     QGrids *g);
int lf_launch_queue(lf_handle *h, Ctx &cx, const QStep &qs, const QGrids &g);
int lf_launch_multi(hipStream_t st, const Member *dmem, const int *dboff, int cap, int nm, const int *total);
#define LF_MULTI_GRIDS 4         // per-step launches of a batch with grids of their own
#define LF_MULTI_KERNELS 5       // kernels of a batch step (k_big_final and k_big_tie share a grid)
void lf_multi_kernels(const void **fn, int *grid, int *block);
int lf_iter_finish(lf_handle *h, long long *joins, long long *leaves, long long *live);
int lf_lines_back(lf_handle *h);          // lines -> slot layout (mid-iteration stop)
int lf_iter_finish_enqueue(lf_handle *h);
int lf_iter_finish_complete(lf_handle *h, long long *joins, long long *leaves, long long *live);
int lf_iteration_end_enqueue(lf_handle *h);
int lf_iteration_end_complete(lf_handle *h, long long *joins, long long *leaves, long long *live);
int lf_check_dev_error(lf_handle *h);
int lf_dev_error_status(lf_handle *h, int e);
void lf_free_iteration_buffers(lf_handle *h);
int lf_fetch_memberships(lf_handle *h, long long *offsets, int *comm_ids, long long capacity,
                         long long *total, int *in_counts);
void lf_free_partition(lf_handle *h);
