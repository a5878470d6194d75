/*
 * lazyfox.h -- C ABI of the MI355X (gfx950) LazyFox hot-path library.
 *
 * The library runs the data-parallel hot path of LazyFox (Garrels et al., arXiv 2210.03211)
 * on one GPU: graph preprocessing, per-node triangles / clustering coefficients / node
 * order, the greedy initial clustering, and LazyFox iterations (queue-batched evaluation of
 * the WCC-hat change of every join and leave action, argmax decision, bulk apply, stopping
 * rule and removal of degenerate communities).
 *
 * Conventions for every function below:
 *  - return value: LF_OK (0) or a negative LF_E* status; the text of the last error is
 *    available from lf_last_error(h);
 *  - "host" pointers are ordinary CPU memory owned by the caller; "device" pointers are
 *    HIP device memory on the handle's device, also owned by the caller;
 *  - inputs are copied: the caller may free or reuse them after the call returns;
 *  - every call is synchronous with respect to the host and stream-ordered on the handle's
 *    HIP stream; a handle must be used by one host thread at a time, separate handles are
 *    independent;
 *  - node ids are dense 0..n-1 after lf_load_graph; community ids are the creation index of
 *    the initial clustering (0..K-1) and are never renumbered.
 */
#ifndef LAZYFOX_H
#define LAZYFOX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define LF_OK 0
#define LF_EINVAL (-1)      /* bad argument: q < 1, theta NaN or < 0, id out of range, ... */
#define LF_ESTATE (-2)      /* call out of order (e.g. run before init) */
#define LF_ENOMEM (-3)      /* device or host allocation failed */
#define LF_EDEVICE (-4)     /* HIP runtime error (text in lf_last_error) */
#define LF_ERANGE (-5)      /* caller buffer too small */
#define LF_EOVERFLOW (-6)   /* size beyond the supported integer ranges */
#define LF_EAGAIN (-7)      /* not ready yet (a batch member or server job still runs) */
#define LF_EINTERNAL (-8)   /* an internal consistency check failed */

/* lf_load_graph flags */
#define LF_RELABEL 1u       /* compact the ids that occur to 0..n-1, order-preserving */
#define LF_DEVICE_PTR 2u    /* src/dst are device pointers (else host pointers) */

typedef struct lf_handle lf_handle;

/* Result of lf_run_iterations.  The four array pointers are caller-owned host buffers
   (any may be NULL): wtilde_hist has max_iters + 1 entries (entry 0 = before iteration 1),
   the others max_iters entries. */
typedef struct {
    int32_t iterations;     /* iterations run in this call */
    int32_t converged;      /* stopping rule met (or nothing to optimise) */
    int32_t hit_max;        /* stopped because max_iters was reached */
    int32_t pad;
    double wcc_hat;         /* WCC-hat(P) of the final partition (0 if cc == 0) */
    double wtilde;          /* cc * WCC-hat(P): the cc-free partition score */
    double *wtilde_hist;
    int64_t *joins;         /* join actions applied per iteration */
    int64_t *leaves;        /* leave actions applied per iteration */
    int64_t *communities;   /* communities with >= 2 members after each iteration */
} lf_run_info;

/* Per-kernel timing, collected with HIP events on the handle's stream when profiling is
   enabled (lf_set_profiling).  The set-up phases are timed as a whole; every kernel of a
   queue (chunk) is timed on its own, so one event pair brackets exactly one launch. */
#define LF_K_BUILD 0        /* graph build (sorts, CSR) */
#define LF_K_TRIANGLES 1    /* triangle counting (all launches) */
#define LF_K_ORDER 2        /* CC, cc reduction, node order */
#define LF_K_INITCLUST 3    /* initial clustering and state set-up */
#define LF_K_EVAL 4         /* k_eval: small wave path (<= 64 visits) of queues with many
                               such nodes */
#define LF_K_EVAL_BIG 5     /* k_eval_big: the other evaluation paths of a queue, by block
                               role: table-path visits, workgroup path (<= 1024 visits),
                               medium wave path (<= 256), small path of smaller queues */
#define LF_K_TAB_FINAL 6    /* k_big_final: table path, candidate changes and maxima */
#define LF_K_TAB_TIE 7      /* k_big_tie: table path, lowest id among equal maxima */
#define LF_K_APPLY_EDIT 8   /* k_apply: the bulk apply of a queue: membership edits, sizes,
                               member lists and re-sum planning beside the in-count changes
                               around the moved nodes */
#define LF_K_APPLY_IN 9     /* no longer launched (its work is part of k_apply); kept so
                               that the class indices stay the same */
#define LF_K_REFRESH 10     /* k_refresh: exact re-sums of the touched communities */
#define LF_K_ITEREND 11     /* iteration end: degenerate removal, compaction, score */
#define LF_K_COUNT 12
#define LF_PROF_COUNTERS_BIT 16 /* profiling mask bit: also count the evaluation work per
                                   path (adds a few global atomics to those kernels) */
#define LF_PATH_SMALL 0     /* evaluation paths for the per-path work counters */
#define LF_PATH_MED 1
#define LF_PATH_GROUP 2
#define LF_PATH_TABLE 3
#define LF_PATH_COUNT 4
/* apply-step work counters (bit 1 << LF_PROF_COUNTERS_BIT), per step of Algorithm 2's
   bulk apply: nodes that moved, own memberships the edits scanned, in-count units of
   moved nodes, neighbours in those units, their memberships scanned, re-sum parts,
   touched communities re-summed, members re-summed, and the memberships those members
   scanned */
#define LF_APPLY_MOVES 0
#define LF_APPLY_OWN_SLOTS 1
#define LF_APPLY_IN_ITEMS 2
#define LF_APPLY_IN_NEIGHBOURS 3
#define LF_APPLY_IN_SLOTS 4
#define LF_APPLY_PARTS 5
#define LF_APPLY_TOUCHED 6
#define LF_APPLY_MEMBERS 7
#define LF_APPLY_MEMBER_SLOTS 8
#define LF_APPLY_COUNT 9
typedef struct {
    int64_t launches[LF_K_COUNT];
    double ms[LF_K_COUNT];
    int64_t chunks;          /* chunks processed */
    int64_t node_evals;      /* queued-node evaluations */
    int64_t visits;          /* neighbour-membership visits in the evaluation kernels */
    int64_t candidates;      /* candidate communities evaluated */
    /* per evaluation path (LF_PATH_*): nodes it decided, their neighbours, the
       neighbour memberships it visited and the candidates it scored */
    int64_t path_nodes[LF_PATH_COUNT];
    int64_t path_neighbours[LF_PATH_COUNT];
    int64_t path_visits[LF_PATH_COUNT];
    int64_t path_candidates[LF_PATH_COUNT];
    int64_t path_own[LF_PATH_COUNT];   /* the decided nodes' own memberships */
    int64_t apply_work[LF_APPLY_COUNT];
} lf_profile;

/* Create a handle on HIP device `device`.  `hip_stream` is a hipStream_t (for example
   torch.cuda.current_stream().cuda_stream) or NULL for a library-owned stream.
   flags: reserved, pass 0. */
int lf_create(lf_handle **out, int device, void *hip_stream, uint32_t flags);

/* Free every device and host resource of the handle.  NULL is accepted. */
int lf_destroy(lf_handle *h);

/* Text of the last error on this handle (static storage owned by the handle). */
const char *lf_last_error(lf_handle *h);

/*
 * Input and preprocessing (Methods, "Input Data" and "Preprocessing": multi-edge removal,
 * dense node labels).  src[e], dst[e] (int64, n_pairs entries, host or device memory per
 * LF_DEVICE_PTR) are undirected edges; duplicates and both directions are allowed and
 * merged, self-loops are dropped.  Without LF_RELABEL ids must lie in [0, n) (isolated
 * nodes are allowed); with LF_RELABEL the argument n is ignored and the ids that occur in
 * a non-self-loop pair are compacted to 0..n-1 in increasing order.
 * Builds a symmetric CSR with every row sorted ascending.  Resets any previous state.
 * Errors: LF_EINVAL (negative sizes, id out of range), LF_EOVERFLOW (n >= 2^31 or
 * 2|E| >= 2^31), LF_ENOMEM, LF_EDEVICE.
 */
int lf_load_graph(lf_handle *h, int64_t n, int64_t n_pairs, const int64_t *src,
                  const int64_t *dst, uint32_t flags);

/*
 * Node statistics and initial clustering (Methods, "Node Order", "Initial Clustering";
 * global cc from the WCC-hat subsection): triangles k_i, local CC(i) = k_i / (d_i(d_i-1)/2)
 * (0 if d_i <= 1), node order by CC descending, then degree descending, then id
 * ascending; cc = mean of all local CCs; greedy clustering in node order (a node without a
 * community opens one and its unassigned neighbours join it); per-community size, internal
 * edges and WCC-hat.  Calling it again restarts from the initial clustering.
 * Errors: LF_ESTATE (no graph), LF_ENOMEM, LF_EDEVICE.
 */
int lf_init_communities(lf_handle *h);

/*
 * Warm start (Methods, "Initial Clustering", last paragraph: an existing division of the
 * network can take the place of the greedy initial clustering, for instance a partition to
 * be turned into an overlapping cover, or the memberships saved from an earlier run to
 * resume it).  Node statistics and order as for lf_init_communities; the given cover then
 * becomes the partition and every maintained quantity (in-counts, sizes, internal edges,
 * exact sums, scores) is counted from its definition, so resuming from the memberships
 * after k iterations continues that run exactly.
 *   offsets   int64[n + 1], offsets[0] = 0, non-decreasing, offsets[n] = total
 *   comm_ids  int32[total]: node x's communities at [offsets[x], offsets[x + 1]), any
 *             order, each in [0, n_comms) and at most once per node; ids are kept as given
 *             (empty and one-member communities are allowed; the first iteration end
 *             removes those with fewer than two members)
 *   n_comms   number of community ids; < 0: the largest id + 1
 *   flags     LF_DEVICE_PTR: both arrays are device pointers (else host); read only
 * The library copies what it needs; the caller keeps ownership of both arrays.
 * Errors: LF_ESTATE (no graph), LF_EINVAL (bad offsets, id out of range, an id twice for
 * a node; the previous partition is then kept), LF_EOVERFLOW, LF_ENOMEM, LF_EDEVICE.
 */
int lf_init_from_memberships(lf_handle *h, const int64_t *offsets, const int32_t *comm_ids,
                             int64_t total, int32_t n_comms, uint32_t flags);

/*
 * Exact WCC of the current partition (Methods, WCC-hat subsection, paragraph "WCC"), the
 * triangle-based score that WCC-hat estimates.  For a member x of C, with t(x,S) the
 * triangles of x whose two other nodes lie in S and vt(x,S) the nodes of S that close at
 * least one triangle with x:
 *   WCC(x,C) = t(x,C) / t(x,V) * vt(x,V) / (|C \ {x}| + vt(x, V \ C)), 0 if t(x,V) = 0,
 * evaluated in FP64 as (t / t_V) * (vt_V / (|C| - 1 + vt_out)); WCC(C) = sum over x in C,
 * WCC(P) = sum over C, both summed exactly and rounded once.  Outputs are caller-owned host
 * buffers; all but wcc may be NULL:
 *   wcc        WCC(P)
 *   wcc_comm   double[K], K = communities created (lf_get_graph_info); 0 for removed ids
 *   wcc_node, t_xc, vt_xc   one entry per membership in the lf_get_memberships order
 *              (node by node, community ids ascending): WCC(x,C), t(x,C), vt(x, V \ C)
 *   vt_x       int32[n]: vt(x, V)
 * Errors: LF_ESTATE (no communities), LF_EOVERFLOW (a term outside the exact range),
 * LF_ENOMEM, LF_EDEVICE.
 */
int lf_exact_wcc(lf_handle *h, double *wcc, double *wcc_comm, double *wcc_node, int32_t *t_xc,
                 int32_t *vt_xc, int32_t *vt_x);

/*
 * F1-Score of the current partition against a reference cover (Methods, "F1-Score for
 * Overlapping Communities"): each detected community C' with at least one member is
 * matched to the reference community C with the largest F1(C', C), the harmonic mean of
 * precision |C n C'| / |C'| and recall |C n C'| / |C|, evaluated as the single correctly
 * rounded division 2 |C n C'| / (|C| + |C'|); the score is the mean of the maxima (exact
 * sum rounded once, divided by the number of detected communities; 0 if there are none).
 *   offsets, ids  the reference cover as for lf_init_from_memberships (ids >= 0, at most
 *                 once per node, any order); host pointers, or device with LF_DEVICE_PTR;
 *                 read only
 *   f1            the score (required)
 *   best, match   optional caller-owned host buffers of K entries (K = communities created,
 *                 lf_get_graph_info): the maximum F1 of each detected id (0 for empty ids or
 *                 no overlap) and the lowest reference id reaching it (-1 if none)
 * Errors: LF_ESTATE, LF_EINVAL (bad cover), LF_ENOMEM, LF_EDEVICE.
 */
int lf_cover_f1(lf_handle *h, const int64_t *offsets, const int32_t *ids, int64_t total,
                uint32_t flags, double *f1, double *best, int32_t *match);

/* lf_postprocess flags */
#define LF_PP_DUPLICATES 1u   /* remove a community whose members equal a lower id's */
#define LF_PP_CONTAINED 2u    /* remove a community whose members are a strict subset of
                                 another community's */
#define LF_PP_APPLY 4u        /* also take the removed communities out of the partition */

/*
 * Optional post-processing of the final cover (Methods, "Post-processing": the result may
 * hold duplicated communities and communities contained in others, which some uses do not
 * want).  Communities with at least one member are compared: with LF_PP_DUPLICATES a
 * community is removed if another one has exactly its members and a lower id, with
 * LF_PP_CONTAINED if its members are a strict subset of another one's (so what remains is
 * the distinct maximal communities, each under its lowest id).  Outputs, caller-owned host
 * buffers, may be NULL: keep uint8[K] (K = communities created, lf_get_graph_info) with 1
 * for each community kept and 0 for removed or empty ids; removed int64[2] = communities
 * removed as duplicates, as contained (a community that is both counts as a duplicate).
 * With LF_PP_APPLY the removed communities lose all their members and the state (in-counts,
 * sizes, exact sums, score) is rebuilt from the remaining cover as by
 * lf_init_from_memberships; ids are kept.
 * Errors: LF_EINVAL (unknown flags), LF_ESTATE, LF_ENOMEM, LF_EDEVICE.
 */
int lf_postprocess(lf_handle *h, uint32_t flags, uint8_t *keep, int64_t *removed);

/*
 * LazyFox iterations (Methods, "Node Changes", Algorithm 2, "Stopping Criteria",
 * "Post-processing").  Each iteration walks the node order in consecutive queues of
 * `queue_size` nodes (the last one partial); every node of a queue gets its best join
 * (largest strictly positive WCC-hat gain over communities of its neighbours it is not
 * in) and best leave (same over its own communities), ties to the lowest community id,
 * all evaluated on the state at the start of the queue; then all of them are applied.
 * After each iteration communities with fewer than two members are removed; the run stops
 * when the relative WCC-hat improvement over the previous iteration is below `threshold`
 * (iteration 1 compares with the initial clustering), or after `max_iters` iterations.
 * A later call continues from the current partition.  `out` may be NULL.
 * Errors: LF_EINVAL (queue_size < 1, threshold NaN or < 0, max_iters < 0), LF_ESTATE.
 */
int lf_run_iterations(lf_handle *h, int32_t queue_size, double threshold, int32_t max_iters,
                      lf_run_info *out);

/*
 * Memberships of every node (host buffers).  offsets: n + 1 entries; comm_ids: capacity
 * entries; per node the community ids ascending.  With offsets == NULL or comm_ids == NULL
 * only *total is written (two-call pattern).  LF_ERANGE if capacity < *total.
 */
int lf_get_memberships(lf_handle *h, int64_t *offsets, int32_t *comm_ids, int64_t capacity,
                       int64_t *total);

/* Graph sizes: nodes, undirected edges, communities created by the initial clustering
   (-1 before lf_init_communities).  Any pointer may be NULL. */
int lf_get_graph_info(lf_handle *h, int64_t *n, int64_t *nedges, int64_t *ncommunities);

/* The CSR built by lf_load_graph (host buffers: rowptr n + 1, col 2|E|) and, with
   LF_RELABEL, the input id of every dense node (orig_ids n entries; may be NULL). */
int lf_get_csr(lf_handle *h, int64_t *rowptr, int32_t *col, int64_t *orig_ids);

/* Node statistics (host buffers of n entries; any may be NULL): triangles k_i, local
   clustering coefficient, node order (order[r] = node processed r-th). */
int lf_get_node_stats(lf_handle *h, int64_t *tri, double *cc_local, int32_t *order);

/* Scores (any pointer may be NULL): WCC-hat(P), global cc, number of triangles T,
   cc-free score cc * WCC-hat(P). */
int lf_get_scores(lf_handle *h, double *wcc_hat, double *cc, int64_t *triangles,
                  double *wtilde);

/* Per community id (host buffers of ncommunities entries; any may be NULL): member count,
   internal edges, cc-free score p_C * sum_x g (WCC-hat(C) * cc). */
int lf_get_communities(lf_handle *h, int32_t *size, int64_t *internal_edges, double *score);

/* in[j] = |N(x) ∩ C| for the j-th membership in the lf_get_memberships listing. */
int lf_get_in_counts(lf_handle *h, int32_t *in, int64_t capacity);

/* Kernel timing: `mask` selects the kernels to time (bit 1 << LF_K_*; 0 = off).
   HIP events are recorded around each timed launch on the handle's stream and resolved at
   the end of the API call, so timing does not stall the host.  chunks and node_evals are
   always counted; the work counters only with bit 1 << LF_PROF_COUNTERS_BIT. */
int lf_set_profiling(lf_handle *h, int mask);
int lf_get_profile(lf_handle *h, lf_profile *out);
int lf_reset_profile(lf_handle *h);

/* Tuning options (lf_set_option / lf_get_option).  Results never depend on them. */
#define LF_OPT_TRI_LDS_CAP 1       /* max out-list length staged in LDS by the workgroup
                                      triangle kernel (0 = as much as LDS holds); longer
                                      out-lists use global scratch */
#define LF_OPT_HUB_BLOCKS 3        /* most workgroups of the table path and of the workgroup
                                      path per launch */
#define LF_OPT_REFRESH_BLOCKS 4    /* workgroups of the in-count and re-sum kernels */
#define LF_OPT_WAVE_TABLE 5        /* candidate-table entries per wave in the wave path
                                      (power of two, 16 .. 128); nodes needing more go to
                                      the medium wave path */
#define LF_OPT_MED_TABLE 6         /* candidate-table entries per wave in the medium wave
                                      path (power of two, 16 .. 512); nodes needing more
                                      go to the workgroup path */
#define LF_OPT_GRP_TABLE 7         /* candidate-table entries per workgroup in the
                                      workgroup path (power of two, 16 .. 2048); nodes
                                      needing more go to the global-table path */
#define LF_OPT_PROF_STRIDE 8       /* kernel timing (lf_set_profiling) brackets only every
                                      k-th launch of each per-queue kernel class (1 ..
                                      65536, default 1 = every launch); the profile's
                                      launches count the bracketed ones */
int lf_set_option(lf_handle *h, int option, int64_t value);
int lf_get_option(lf_handle *h, int option, int64_t *value);

/*
 * Autotuner of the options above that shape the evaluation (where the medium, workgroup
 * and table paths start: LF_OPT_WAVE_TABLE, LF_OPT_MED_TABLE, LF_OPT_GRP_TABLE) and the
 * launches (LF_OPT_HUB_BLOCKS, LF_OPT_REFRESH_BLOCKS).  Needs initialised communities.
 * Candidates are timed on `trial_iters` iterations of queue size `queue_size` from the
 * initial clustering (coordinate descent, one option at a time); the fastest is set on
 * the handle, which is left at its initial clustering again.  The choice is remembered
 * for the graph's class (log2 degree histogram, log2 queue size, log2 node count) within
 * the process; a handle of a known class takes it without trials (from_cache = 1).
 * Results of lf_run_iterations do not depend on the choice.
 */
typedef struct {
    int64_t value[5];       /* WAVE_TABLE, MED_TABLE, GRP_TABLE, HUB_BLOCKS, REFRESH_BLOCKS */
    float default_ms;       /* trial time with the options the handle had */
    float best_ms;          /* trial time with the chosen options */
    int32_t trials;
    int32_t from_cache;
} lf_tune_result;
int lf_autotune(lf_handle *h, int32_t queue_size, int32_t trial_iters, lf_tune_result *out);
/* Forget every remembered class. */
int lf_autotune_forget(void);

/*
 * Diagnostic: the exact sum of n doubles (device pointer), rounded once to nearest-even,
 * computed by the library's device accumulator (the one behind every score sum).
 * Values must be finite with magnitude in [2^-113, 2^30] or zero; LF_EOVERFLOW otherwise.
 */
int lf_debug_exact_sum(lf_handle *h, const double *values_dev, int64_t n, double *out);

/*
 * lf_debug_exact_sum without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, result and errors as lf_debug_exact_sum, plus LF_EINVAL for
 * n > LF_NOALLOC_MAX_VALUES (2^40: with every |value| <= 2^30 the exact partial sums then
 * stay inside the device accumulator).  Its scratch (1024 block partial sums, a range
 * flag and the result, 32 KiB) is a fixed device array of the library, one per GPU, held
 * until the process ends; every call on a GPU uses that GPU's copy, so calls that overlap
 * on one GPU (from any handles or threads) race and must be serialised by the caller.
 * The call calls no hipMalloc or hipFree; it waits for the handle's stream.
 */
#define LF_NOALLOC_MAX_VALUES (1ll << 40)
int lf_exact_sum_noalloc(lf_handle *h, const double *values_dev, int64_t n, double *out);

/*
 * Diagnostics of the library's own device primitives (the sorts behind "Remove
 * Multi-Edges" and "Node Order" in Methods, and the prefix sums behind every compaction).
 * lf_debug_sort_pairs: stable LSD radix sort in place of n keys (device, uint64) by their
 *   bits [0, end_bit), 0 <= end_bit <= 64, with the int32 values (device, may be NULL)
 *   moved alongside.  lf_debug_sort_pairs_u32: the same for uint32 keys (all 32 bits),
 *   values required.  Both: n < 2^31 (LF_EOVERFLOW otherwise).
 * lf_debug_exclusive_scan: out[i] = sum of in[0..i) as int64, for in of n int32
 *   (in_bytes = 4) or int64 (in_bytes = 8) entries (device); in and out may alias.
 * Temporaries come from the handle's scratch arena; the calls wait for the stream.
 */
int lf_debug_sort_pairs(lf_handle *h, uint64_t *keys_dev, int32_t *vals_dev, int64_t n, int32_t end_bit);
int lf_debug_sort_pairs_u32(lf_handle *h, uint32_t *keys_dev, int32_t *vals_dev, int64_t n);
int lf_debug_exclusive_scan(lf_handle *h, const void *in_dev, int32_t in_bytes, int64_t *out_dev, int64_t n);

/* Device memory the handle holds now and at most so far (bytes). */
int lf_get_memory(lf_handle *h, uint64_t *bytes, uint64_t *peak);

/*
 * Many graphs advanced together (Algorithm 2 run for each of them).  A batch holds handles
 * whose communities are initialised; each lf_batch_step runs one queue of every member
 * still iterating, with one launch per kernel covering all members, and performs a
 * member's iteration start and end (path lists, degenerate removal, exact score, stopping
 * rule of "Stopping Criteria") between steps.  Each member computes exactly what
 * lf_run_iterations(queue_size, threshold, max_iters) computes on it alone.
 *
 * lf_batch_create: `hip_stream` as for lf_create (NULL = a batch-owned stream); members'
 *   work runs on it.  lf_batch_add: the handle (same device, state after
 *   lf_init_communities) joins; while a member, it runs on the batch's stream and must not
 *   be used otherwise.  *member_id identifies it.  LF_ESTATE before lf_init_communities.
 * lf_batch_step: *running = members still iterating afterwards.
 * lf_batch_member_info: LF_OK and `out` filled as by lf_run_iterations when the member is
 *   done; LF_EAGAIN while it iterates; its error status if it failed.
 * lf_batch_remove: the member leaves (done or not); its handle returns to its own stream.
 * lf_batch_destroy: removes every member (handles are not destroyed) and frees the batch.
 */
typedef struct lf_batch lf_batch;
int lf_batch_create(lf_batch **out, int device, void *hip_stream);
int lf_batch_add(lf_batch *b, lf_handle *h, int32_t queue_size, double threshold, int32_t max_iters,
                 int32_t *member_id);
int lf_batch_step(lf_batch *b, int32_t *running);
int lf_batch_member_info(lf_batch *b, int32_t member_id, lf_run_info *out);
int lf_batch_remove(lf_batch *b, int32_t member_id);
int lf_batch_destroy(lf_batch *b);
const char *lf_batch_last_error(lf_batch *b);
/* on != 0 (the default): each step replays a graph of the per-step launches,
   captured once, with the step's grids and member count set on its kernel nodes;
   on = 0: the launches are issued one by one.  Results are the same either way. */
int lf_batch_set_graph(lf_batch *b, int32_t on);

/*
 * Serving: community-detection jobs on graphs of uneven size.  lf_server_submit copies a
 * job's edge list (host memory, as for lf_load_graph without flags) and queues it;
 * LF_ENOMEM if its estimated device footprint exceeds the whole budget.  Each
 * lf_server_tick admits queued jobs in arrival order while their estimated footprints fit
 * the budget and fewer than max_batch jobs run, runs one batch step, and hands finished
 * jobs over for retirement.  Four worker threads of the server, each with a stream of its
 * own, load admitted jobs (graph load, initial clustering; they join the batch at the
 * next tick) and retire finished ones (memberships copied to host memory, device memory
 * returned to the library's allocation cache; the job is done at the next tick after
 * that), so the ticking thread never waits for either.  A job's footprint stays reserved
 * from admission until its retirement has completed; jobs that arrived meanwhile are
 * admitted as memory frees up.  *pending = jobs queued or running.
 * lf_server_poll: *state = 0 queued, 1 running, 2 done, < 0 failed with that status.
 * lf_server_take_done: ids of the jobs that finished or failed since the last call (in
 *   completion order, at most capacity; *count = how many were written), so a caller can
 *   fetch exactly those instead of polling every job.
 * lf_server_fetch: results of a done job, two-call pattern as lf_get_memberships
 *   (LF_EAGAIN if not done); after a copy of the memberships the job is forgotten.
 * lf_server_stats: device bytes reserved by admitted jobs, the budget, running and queued
 *   jobs.  A job's results equal those of lf_run_iterations on its graph alone.
 */
typedef struct lf_server lf_server;
int lf_server_create(lf_server **out, int device, void *hip_stream, uint64_t hbm_budget, int32_t max_batch);
int lf_server_submit(lf_server *s, int64_t n, int64_t n_pairs, const int64_t *src, const int64_t *dst,
                     int32_t queue_size, double threshold, int32_t max_iters, int64_t *job_id);
int lf_server_tick(lf_server *s, int32_t *pending);
int lf_server_poll(lf_server *s, int64_t job_id, int32_t *state);
int lf_server_take_done(lf_server *s, int64_t *ids, int32_t capacity, int32_t *count);
int lf_server_fetch(lf_server *s, int64_t job_id, int64_t *offsets, int32_t *comm_ids, int64_t capacity,
                    int64_t *total, lf_run_info *info);
int lf_server_stats(lf_server *s, uint64_t *used, uint64_t *budget, int32_t *running, int32_t *queued);
int lf_server_destroy(lf_server *s);
const char *lf_server_last_error(lf_server *s);
/* Host milliseconds spent so far in ms[0..4]: admission (graph load and initial
   clustering) and retirement (results copied back, device state released), summed over
   the worker threads, in ms[0] and ms[2]; batch steps; handing jobs to and from the
   workers (batch add, member info, detach); whole ticks; ms[5] the
   part of the batch steps spent waiting for the device; ms[6] the batch steps that
   launched work and ms[7] the queues they ran (counts); ms[8..10] the host time of the
   steps in iteration starts and ends, in per-member queue parameters, and in the
   descriptor upload and launch; ms[11..13] the iteration starts and ends of retired jobs
   that ran plainly, were captured into graphs, and were replayed from them (counts).
   ms holds 14 values. */
int lf_server_timing(lf_server *s, double *ms);
/* Graph replay of the server's batch steps (lf_batch_set_graph); on by default. */
int lf_server_set_graph(lf_server *s, int32_t on);

#ifdef __cplusplus
}
#endif
#endif
