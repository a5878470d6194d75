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

// Device-side counters and flags (one struct in device memory).
struct DevCounters {
    unsigned long long joins;      // per iteration
    unsigned long long leaves;     // per iteration
    unsigned long long visits;     // evaluation statistics (cumulative)
    unsigned long long cands;
    int tcount;                    // touched communities in the current chunk
    int hub_count;                 // nodes deferred to the workgroup evaluation path
    int hub_next;                  // work counter of the workgroup evaluation kernel
    int refresh_next;              // work counter of the community re-sum kernel
    int ovf_cnt;                   // joiners that did not fit their community's member list
    int undecided;                 // initial clustering rounds
    int error;                     // bit flags, see LF_DEVERR_*
    int live;                      // communities with >= 2 members (iteration end)
    int max_mem;                   // largest membership count (iteration end)
    int pad[3];
    X256 score;                    // exact partition score (iteration end)
};

#define LF_DEVERR_INEXACT 1        // a value did not fit the exact accumulator
#define LF_DEVERR_INCOUNT 2        // in-count bookkeeping disagreed with a recount
#define LF_DEVERR_ODD 4            // odd internal-degree sum
#define LF_DEVERR_SLOTS 8          // a node ran out of membership slots

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
    int *cs;                 // community size
    long long *cm;           // internal edges
    double *cW;              // cc-free community score
    X192 *cSp;               // exact sum of g at size s+1
    X192 *cSm;               // exact sum of g at size s-1
    long long *cm_off;       // member-list capacity offsets (K + 1)
    int *cm_len;             // member-list fill (may exceed capacity: overflow)
    int *cm_node;            // member lists
    int *tflag;              // touched flag per community
    int *tlist;              // touched list
    int *joined_to;          // community joined in the current chunk (-1 otherwise)
    int *ovf_node;           // overflow joiners (node, community)
    int *ovf_comm;
    int *ovf_flag;
    int *dj, *dl;            // decisions of the current chunk
    double *djd, *dld;
    int *hub_list;
    DevCounters *ctr;
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
    double cc;
    long long T;
    // partition
    NodeHdr *nh;
    Slot *slot[2];
    int cur;
    long long slot_capb[2];  // capacity of each slot buffer
    int *cs;
    long long *cm;
    double *cW;
    X192 *cSp, *cSm;
    long long *cm_off;
    int *cm_len;
    int *cm_node;
    long long cm_cap;        // capacity of cm_node
    int *tflag, *tlist, *joined_to;
    int *ovf_node, *ovf_comm, *ovf_flag;
    int *dj, *dl;
    double *djd, *dld;
    int *hub_list;
    long long q_cap;         // capacity of the decision / touched arrays
    DevCounters *ctr;
    double Wt;               // cc-free partition score
    // generic device scratch
    void *tmp;
    size_t tmp_bytes;
    // tuning
    int eval_wave_cap;       // table entries per wave in the wave evaluation path
    int hub_lds_entries;     // table entries of the workgroup evaluation path
    int hub_blocks;          // resident workgroups of the workgroup evaluation path
    int refresh_blocks;      // resident workgroups of the community re-sum kernel
    // profiling
    int profiling;
    lf_profile prof;
    hipEvent_t ev0, ev1;
    // allocation registry
    std::vector<void *> *allocs;
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
int lf_ensure_tmp(lf_handle *h, size_t bytes);
Ctx lf_ctx(lf_handle *h);

// profiling brackets around a launch sequence on the handle's stream
int lf_prof_begin(lf_handle *h);
int lf_prof_end(lf_handle *h, int kind, int launches);

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

// ---- graph stages (graph.hip) ------------------------------------------------------------
int lf_build_graph(lf_handle *h, long long n, long long npairs, const long long *src,
                   const long long *dst, unsigned flags);
int lf_node_stats(lf_handle *h);
int lf_exact_sum_dev(lf_handle *h, const double *v, long long n, double *out);

// ---- community stages (communities.hip) ----------------------------------------------------
int lf_initial_clustering(lf_handle *h);
int lf_iterate(lf_handle *h, int q, double theta, int max_iters, lf_run_info *out);
int lf_fetch_memberships(lf_handle *h, long long *offsets, int *comm_ids, long long capacity,
                         long long *total, int *in_counts);
void lf_free_partition(lf_handle *h);
