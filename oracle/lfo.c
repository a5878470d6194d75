/*
 * lfo.c -- CPU oracle for the LazyFox hot path.  TEST INFRASTRUCTURE ONLY: the test-suite,
 * the smoke check and the CPU-baseline leg of the benchmark load it; the product library
 * never does, and the two share no code.
 *
 * Plain, slow, obviously-correct C that follows Garrels, Khodabakhsh, Renard, Baum,
 * "LazyFox: Fast and parallelized overlapping community detection in large graphs"
 * (arXiv 2210.03211), section Methods:
 *
 *   lfo_load_graph        Preprocessing: "Remove Multi-Edges", "Dense Node Labels"
 *   lfo_init_communities  Preprocessing: "Node Order" (clustering-coefficient equation),
 *                         "Initial Clustering"; global cc from the WCC-hat subsection
 *   lfo_init_from_memberships  the same with an existing division in place of the greedy
 *                         initial clustering ("Initial Clustering", last paragraph)
 *   eval_*                WCC-hat definition (mean-field triangle estimate, upper bounds on
 *                         vt, the per-node / per-community / per-partition sums) and
 *                         "Node Changes" (join and leave actions, Algorithm 1)
 *   run_chunk             Algorithm 2: a queue of q nodes is evaluated on one frozen state,
 *                         then all changes are applied together
 *   end_iteration         "Stopping Criteria" and "Post-processing" (degenerate communities)
 *   lfo_exact_wcc         WCC of a partition from exact triangle counts (WCC paragraph of the
 *                         WCC-hat subsection), to set beside the WCC-hat estimate
 *   lfo_postprocess       removal of duplicated and contained communities ("Post-processing")
 *   lfo_cover_f1          F1-Score against a reference cover ("F1-Score for Overlapping
 *                         Communities")
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *  - self-loops are dropped; node order ties: degree descending, then id ascending;
 *  - cc is the mean of the local CCs over all n nodes (zeros included);
 *  - density of a community p = 2 m / (s (s-1)), s < 2 -> 0, in the partition scored;
 *  - WCC-hat(x,C) = p * g(i,d,s) / cc with g = i(i-1) / ((d-1)(s-1+d-i)), g = 0 if i<2
 *    or d<2: the paper's estimator with E[t(x,C)] = C(i,2) p, E[t(x,V)] = C(d,2) cc,
 *    |C\{x}| = s-1 and deg(x, V\C) = d-i substituted;
 *  - cc > 0 is a common positive factor of every WCC-hat term, so decisions and the relative
 *    stopping test use the cc-free scores  W(C) = p * sum g  and  Wt = sum_C W(C);
 *  - a move is taken only for a strictly positive change; ties -> lowest community id;
 *  - best join and best leave are both applied; all sums that feed a decision are exact
 *    (see xsum below) and rounded once, so no result depends on summation order;
 *  - stop when Wt_{t-1} == 0 or (Wt_t - Wt_{t-1}) / Wt_{t-1} < theta (strict); communities
 *    with fewer than two members are removed at the end of every iteration.
 *
 * Two evaluation modes give bit-identical results (a test checks it):
 *   mode bit 0 clear: "naive"   -- the score of C' is re-summed over all its members;
 *   mode bit 0 set:   "factored" -- exact stored sums S+ / S- of C's members at size s+1 /
 *                     s-1 plus exact corrections for x's neighbours in C (same exact value);
 *   mode bit 1 clear: per-member neighbour counts of touched communities re-counted from
 *                     scratch after a chunk; set: updated incrementally (same values).
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no FMA contraction, no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define LFO_OK 0
#define LFO_EINVAL (-1)
#define LFO_ESTATE (-2)
#define LFO_ENOMEM (-3)
#define LFO_ERANGE (-5)
#define LFO_EOVERFLOW (-6)

#define LFO_RELABEL 1u

/* ------------------------------------------------------------------------------------ */
/* Exact accumulator: a 512-bit two's-complement integer scaled by 2^-256.               */
/* Every double the method sums lies in [2^-200, 2^200] with its lowest set bit above     */
/* 2^-256, so the sum below is exact; xs_round rounds it once to nearest-even.            */
/* ------------------------------------------------------------------------------------ */
#define XL 8
#define XLSB 256
typedef struct { uint64_t w[XL]; } xsum;

static void xs_clear(xsum *a) { memset(a, 0, sizeof *a); }

static void xs_add_int(xsum *a, const uint64_t *t)
{
    uint64_t c = 0;
    for (int k = 0; k < XL; k++) {
        uint64_t s = a->w[k] + t[k];
        uint64_t c1 = s < t[k];
        uint64_t s2 = s + c;
        uint64_t c2 = s2 < c;
        a->w[k] = s2;
        c = c1 | c2;
    }
}

static void xs_sub_int(xsum *a, const uint64_t *t)
{
    uint64_t b = 0;
    for (int k = 0; k < XL; k++) {
        uint64_t x = a->w[k];
        uint64_t d = x - t[k];
        uint64_t b1 = x < t[k];
        uint64_t d2 = d - b;
        uint64_t b2 = d < b;
        a->w[k] = d2;
        b = b1 | b2;
    }
}

static int xs_err = 0; /* set if a value could not be represented exactly (never expected) */

/* a += v, exactly */
static void xs_add(xsum *a, double v)
{
    if (v == 0.0) return;
    if (!isfinite(v)) { xs_err = 1; return; }
    int neg = v < 0.0;
    double av = neg ? -v : v;
    int e;
    double f = frexp(av, &e);                 /* av = f * 2^e, f in [0.5, 1) */
    uint64_t mant = (uint64_t)ldexp(f, 53);   /* exact 53-bit integer */
    int sh = e - 53 + XLSB;                   /* weight of mant's lowest bit, in bits */
    if (sh < 0 || sh + 53 > 64 * XL - 2) { xs_err = 1; return; }
    uint64_t t[XL];
    memset(t, 0, sizeof t);
    int li = sh / 64, bi = sh % 64;
    t[li] = mant << bi;
    if (bi >= 12) t[li + 1] = mant >> (64 - bi);
    if (neg) xs_sub_int(a, t); else xs_add_int(a, t);
}

static void xs_add_xs(xsum *a, const xsum *b) { xs_add_int(a, b->w); }

/* correctly rounded (to nearest, ties to even) double value of a */
static double xs_round(const xsum *a)
{
    xsum m = *a;
    int neg = (int)(m.w[XL - 1] >> 63);
    if (neg) {
        uint64_t c = 1;
        for (int k = 0; k < XL; k++) {
            uint64_t x = ~m.w[k] + c;
            c = (c && x == 0) ? 1 : 0;
            m.w[k] = x;
        }
    }
    int top = -1;
    for (int k = XL - 1; k >= 0; k--)
        if (m.w[k]) { top = k * 64 + 63 - __builtin_clzll(m.w[k]); break; }
    if (top < 0) return 0.0;
    double r;
    if (top <= 52) {
        r = ldexp((double)m.w[0], -XLSB);
    } else {
        int lo = top - 52;
        int li = lo / 64, bi = lo % 64;
        uint64_t mant = m.w[li] >> bi;
        if (bi && li + 1 < XL) mant |= m.w[li + 1] << (64 - bi);
        mant &= (1ULL << 53) - 1;
        int rb = top - 53;
        int round = (int)((m.w[rb / 64] >> (rb % 64)) & 1);
        int sticky = 0;
        int sb = top - 54;
        if (sb >= 0) {
            int sli = sb / 64, sbi = sb % 64;
            uint64_t mask = (sbi == 63) ? ~0ULL : ((1ULL << (sbi + 1)) - 1);
            if (m.w[sli] & mask) sticky = 1;
            for (int k = 0; k < sli; k++) if (m.w[k]) sticky = 1;
        }
        if (round && (sticky || (mant & 1))) mant++;
        if (mant == (1ULL << 53)) { mant >>= 1; top++; }
        r = ldexp((double)mant, top - 52 - XLSB);
    }
    return neg ? -r : r;
}

/* ------------------------------------------------------------------------------------ */
/* The two scalar pieces of WCC-hat                                                       */
/* ------------------------------------------------------------------------------------ */

/* density p of a community with s members and m internal edges (its "density p") */
static double density(int64_t s, int64_t m)
{
    if (s < 2) return 0.0;
    return (double)(2 * m) / (double)(s * (s - 1));
}

/*
 * g(i, d, s) = WCC-hat(x, C) * cc / p for a member x with d = deg(x,V), i = deg(x,C) and
 * s = |C|:  E[t(x,C)] / E[t(x,V)] * deg(x,V) / (|C\{x}| + deg(x,V\C)) with the mean-field
 * estimates C(i,2) p and C(d,2) cc substituted.  Zero when E[t(x,V)] = 0 (d < 2) and when
 * C(i,2) = 0 (i < 2).  Numerator and denominator are integers, one rounding.
 */
static double g_term(int64_t i, int64_t d, int64_t s)
{
    if (d < 2 || i < 2) return 0.0;
    int64_t num = i * (i - 1);
    int64_t den = (d - 1) * (s - 1 + d - i);
    return (double)num / (double)den;
}

/* ------------------------------------------------------------------------------------ */
/* State                                                                                 */
/* ------------------------------------------------------------------------------------ */
typedef struct {
    int32_t cnt, cap;
    int32_t *comm;   /* community ids, ascending */
    int32_t *in;     /* in[j] = deg(x, comm[j]) = |N(x) ∩ comm[j]| */
} memb_t;

typedef struct {
    int32_t cnt, cap;
    int32_t *node;   /* members, unordered */
} cmem_t;

typedef struct {
    int64_t n, nedges;
    int64_t *rowptr;
    int32_t *col;
    int32_t *deg;
    int64_t *orig_id;     /* dense label -> input id (relabel) or identity */
    /* node statistics */
    int64_t *tri;
    double *ccl;
    int32_t *order, *rank;
    double cc;
    int64_t T;
    int inited;
    /* partition */
    int32_t K, Kcap;
    memb_t *mem;
    cmem_t *cm;
    int64_t *m;           /* internal edges */
    double *W;            /* cc-free community score fl(p * R(sum g)) */
    xsum *S0, *Sp, *Sm;   /* exact sums of g at size s, s+1, s-1 */
    double Wt;            /* cc-free partition score R(sum W) */
    int64_t iter_done;
    int64_t chunk_limit;  /* > 0: run_iterations stops after this many queues (timing samples) */
    int64_t chunks_done;  /* queues evaluated and applied by the last run_iterations */
    char err[256];
} lfo;

typedef struct {
    int32_t iterations, converged, hit_max, pad;
    double wcc_hat, wtilde;
    double *wtilde_hist;   /* caller buffer, max_iters + 1 entries (0 = before iteration 1) */
    int64_t *joins;        /* caller buffers, max_iters entries each (may be NULL) */
    int64_t *leaves;
    int64_t *communities;
} lfo_run_info;

static void *xmalloc(size_t sz) { void *p = malloc(sz ? sz : 1); if (!p) { fprintf(stderr, "lfo: out of memory\n"); abort(); } return p; }
static void *xcalloc(size_t n, size_t sz) { void *p = calloc(n ? n : 1, sz ? sz : 1); if (!p) { fprintf(stderr, "lfo: out of memory\n"); abort(); } return p; }

static void free_partition(lfo *h)
{
    if (h->mem) {
        for (int64_t x = 0; x < h->n; x++) { free(h->mem[x].comm); free(h->mem[x].in); }
        free(h->mem);
    }
    if (h->cm) {
        for (int32_t c = 0; c < h->K; c++) free(h->cm[c].node);
        free(h->cm);
    }
    free(h->m); free(h->W); free(h->S0); free(h->Sp); free(h->Sm);
    h->mem = NULL; h->cm = NULL; h->m = NULL; h->W = NULL; h->S0 = h->Sp = h->Sm = NULL;
    h->K = 0;
}

static void free_graph(lfo *h)
{
    free_partition(h);
    free(h->rowptr); free(h->col); free(h->deg); free(h->orig_id);
    free(h->tri); free(h->ccl); free(h->order); free(h->rank);
    h->rowptr = NULL; h->col = NULL; h->deg = NULL; h->orig_id = NULL;
    h->tri = NULL; h->ccl = NULL; h->order = h->rank = NULL;
    h->n = h->nedges = 0;
    h->inited = 0;
}

lfo *lfo_create(void) { return (lfo *)xcalloc(1, sizeof(lfo)); }
void lfo_destroy(lfo *h) { if (!h) return; free_graph(h); free(h); }
const char *lfo_last_error(lfo *h) { return h ? h->err : "null handle"; }

/* ------------------------------------------------------------------------------------ */
/* Preprocessing                                                                          */
/* ------------------------------------------------------------------------------------ */
static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

static int64_t find_id(const int64_t *ids, int64_t n, int64_t v)
{
    int64_t lo = 0, hi = n - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (ids[mid] == v) return mid;
        if (ids[mid] < v) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/*
 * Input: an undirected, unweighted edge list (both directions and duplicates allowed).
 * Self-loops are dropped, every pair canonicalised to (min, max), duplicates removed
 * ("Remove Multi-Edges").  With LFO_RELABEL the ids that occur are compacted to 0..n-1 in
 * increasing order ("Dense Node Labels"); otherwise ids must lie in [0, n).
 * Result: symmetric CSR with every row sorted ascending.
 */
int lfo_load_graph(lfo *h, int64_t n, int64_t npairs, const int64_t *src, const int64_t *dst,
                   uint32_t flags)
{
    if (!h) return LFO_EINVAL;
    if (npairs < 0 || (!(flags & LFO_RELABEL) && n < 0)) {
        snprintf(h->err, sizeof h->err, "negative size");
        return LFO_EINVAL;
    }
    free_graph(h);
    int64_t *ids = NULL;
    if (flags & LFO_RELABEL) {
        ids = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)(2 * npairs));
        int64_t k = 0;
        for (int64_t e = 0; e < npairs; e++) {
            if (src[e] == dst[e]) continue;
            ids[k++] = src[e];
            ids[k++] = dst[e];
        }
        qsort(ids, (size_t)k, sizeof(int64_t), cmp_i64);
        int64_t u = 0;
        for (int64_t j = 0; j < k; j++) if (j == 0 || ids[j] != ids[j - 1]) ids[u++] = ids[j];
        n = u;
    } else {
        for (int64_t e = 0; e < npairs; e++)
            if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) {
                snprintf(h->err, sizeof h->err, "edge %lld has an id outside [0, %lld)",
                         (long long)e, (long long)n);
                return LFO_EINVAL;
            }
    }
    if (n >= (1LL << 31) - 1) { snprintf(h->err, sizeof h->err, "too many nodes"); free(ids); return LFO_EOVERFLOW; }
    uint64_t *key = (uint64_t *)xmalloc(sizeof(uint64_t) * (size_t)npairs);
    int64_t k = 0;
    for (int64_t e = 0; e < npairs; e++) {
        int64_t a = src[e], b = dst[e];
        if (a == b) continue;                              /* self-loop */
        if (ids) { a = find_id(ids, n, a); b = find_id(ids, n, b); }
        if (a > b) { int64_t t = a; a = b; b = t; }
        key[k++] = (uint64_t)a * (uint64_t)n + (uint64_t)b;
    }
    qsort(key, (size_t)k, sizeof(uint64_t), cmp_u64);
    int64_t ne = 0;
    for (int64_t j = 0; j < k; j++) if (j == 0 || key[j] != key[j - 1]) key[ne++] = key[j];
    h->n = n;
    h->nedges = ne;
    h->deg = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    for (int64_t j = 0; j < ne; j++) {
        h->deg[key[j] / (uint64_t)n]++;
        h->deg[key[j] % (uint64_t)n]++;
    }
    h->rowptr = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)(n + 1));
    h->rowptr[0] = 0;
    for (int64_t x = 0; x < n; x++) h->rowptr[x + 1] = h->rowptr[x] + h->deg[x];
    h->col = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(2 * ne));
    int64_t *pos = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)(n + 1));
    memcpy(pos, h->rowptr, sizeof(int64_t) * (size_t)(n + 1));
    /* keys are sorted by (a, b): row r first receives every a < r ascending (as the b of
       (a, r)) and then every b > r ascending, so each row ends up sorted */
    for (int64_t j = 0; j < ne; j++) {
        int64_t a = (int64_t)(key[j] / (uint64_t)n), b = (int64_t)(key[j] % (uint64_t)n);
        h->col[pos[a]++] = (int32_t)b;
        h->col[pos[b]++] = (int32_t)a;
    }
    free(pos);
    free(key);
    h->orig_id = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    for (int64_t x = 0; x < n; x++) h->orig_id[x] = ids ? ids[x] : x;
    free(ids);
    return LFO_OK;
}

/* k_x = number of edges between two neighbours of x: for every neighbour y, count the
   neighbours of y that are also neighbours of x; every such edge is seen from both ends. */
static void count_triangles(lfo *h, int nthreads)
{
    int64_t n = h->n;
    h->tri = (int64_t *)xcalloc((size_t)n, sizeof(int64_t));
#pragma omp parallel num_threads(nthreads)
    {
        int64_t *mark = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)(n ? n : 1));
        for (int64_t z = 0; z < n; z++) mark[z] = -1;
#pragma omp for schedule(dynamic, 64)
        for (int64_t x = 0; x < n; x++) {
            for (int64_t e = h->rowptr[x]; e < h->rowptr[x + 1]; e++) mark[h->col[e]] = x;
            int64_t twice = 0;
            for (int64_t e = h->rowptr[x]; e < h->rowptr[x + 1]; e++) {
                int32_t y = h->col[e];
                for (int64_t f = h->rowptr[y]; f < h->rowptr[y + 1]; f++)
                    if (mark[h->col[f]] == x) twice++;
            }
            h->tri[x] = twice / 2;
        }
        free(mark);
    }
}

static const lfo *g_sort_h; /* comparator context (single sort at a time) */
static int cmp_order(const void *pa, const void *pb)
{
    int32_t a = *(const int32_t *)pa, b = *(const int32_t *)pb;
    const lfo *h = g_sort_h;
    if (h->ccl[a] != h->ccl[b]) return h->ccl[a] > h->ccl[b] ? -1 : 1;   /* CC descending */
    if (h->deg[a] != h->deg[b]) return h->deg[a] > h->deg[b] ? -1 : 1;   /* degree descending */
    return (a > b) - (a < b);                                             /* id ascending */
}

static int32_t memb_find(const memb_t *mb, int32_t c)
{
    int32_t lo = 0, hi = mb->cnt - 1;
    while (lo <= hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (mb->comm[mid] == c) return mid;
        if (mb->comm[mid] < c) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

static void memb_insert(memb_t *mb, int32_t c, int32_t in)
{
    if (mb->cnt == mb->cap) {
        mb->cap = mb->cap ? 2 * mb->cap : 2;
        mb->comm = (int32_t *)realloc(mb->comm, sizeof(int32_t) * (size_t)mb->cap);
        mb->in = (int32_t *)realloc(mb->in, sizeof(int32_t) * (size_t)mb->cap);
        if (!mb->comm || !mb->in) abort();
    }
    int32_t j = mb->cnt;
    while (j > 0 && mb->comm[j - 1] > c) { mb->comm[j] = mb->comm[j - 1]; mb->in[j] = mb->in[j - 1]; j--; }
    mb->comm[j] = c;
    mb->in[j] = in;
    mb->cnt++;
}

static void memb_remove(memb_t *mb, int32_t c)
{
    int32_t j = memb_find(mb, c);
    if (j < 0) abort();
    for (; j + 1 < mb->cnt; j++) { mb->comm[j] = mb->comm[j + 1]; mb->in[j] = mb->in[j + 1]; }
    mb->cnt--;
}

static void cmem_add(cmem_t *cm, int32_t x)
{
    if (cm->cnt == cm->cap) {
        cm->cap = cm->cap ? 2 * cm->cap : 4;
        cm->node = (int32_t *)realloc(cm->node, sizeof(int32_t) * (size_t)cm->cap);
        if (!cm->node) abort();
    }
    cm->node[cm->cnt++] = x;
}

static void cmem_remove(cmem_t *cm, int32_t x)
{
    for (int32_t j = 0; j < cm->cnt; j++)
        if (cm->node[j] == x) { cm->node[j] = cm->node[cm->cnt - 1]; cm->cnt--; return; }
    abort();
}

static int32_t in_of(const lfo *h, int32_t y, int32_t c)
{
    int32_t j = memb_find(&h->mem[y], c);
    return j < 0 ? -1 : h->mem[y].in[j];
}

/* refresh m, W, S0, S+, S- of community c from its members and their (correct) in-counts */
static void refresh_comm(lfo *h, int32_t c)
{
    const cmem_t *cm = &h->cm[c];
    int64_t s = cm->cnt, sumi = 0;
    xsum S0, Sp, Sm;
    xs_clear(&S0); xs_clear(&Sp); xs_clear(&Sm);
    for (int32_t j = 0; j < cm->cnt; j++) {
        int32_t y = cm->node[j];
        int64_t i = in_of(h, y, c), d = h->deg[y];
        sumi += i;
        xs_add(&S0, g_term(i, d, s));
        xs_add(&Sp, g_term(i, d, s + 1));
        xs_add(&Sm, g_term(i, d, s - 1));
    }
    if (sumi % 2) { fprintf(stderr, "lfo: odd internal degree sum\n"); abort(); }
    h->m[c] = sumi / 2;
    h->S0[c] = S0; h->Sp[c] = Sp; h->Sm[c] = Sm;
    h->W[c] = density(s, h->m[c]) * xs_round(&S0);
}

static double partition_score(const lfo *h)
{
    xsum a;
    xs_clear(&a);
    for (int32_t c = 0; c < h->K; c++) xs_add(&a, h->W[c]);
    return xs_round(&a);
}

/* Node statistics: triangles, local CC, node order ("Node Order") and global cc */
static void node_statistics(lfo *h, int nthreads)
{
    int64_t n = h->n;
    free(h->tri); free(h->ccl); free(h->order); free(h->rank);
    if (nthreads < 1) nthreads = 1;
    count_triangles(h, nthreads);
    h->ccl = (double *)xmalloc(sizeof(double) * (size_t)(n ? n : 1));
    int64_t tsum = 0;
    xsum ccsum;
    xs_clear(&ccsum);
    for (int64_t x = 0; x < n; x++) {
        int64_t d = h->deg[x];
        h->ccl[x] = d > 1 ? (double)h->tri[x] / (double)(d * (d - 1) / 2) : 0.0;
        xs_add(&ccsum, h->ccl[x]);
        tsum += h->tri[x];
    }
    h->T = tsum / 3;
    h->cc = n > 0 ? xs_round(&ccsum) / (double)n : 0.0;
    h->order = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    h->rank = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    for (int64_t x = 0; x < n; x++) h->order[x] = (int32_t)x;
    g_sort_h = h;
    qsort(h->order, (size_t)n, sizeof(int32_t), cmp_order);
    for (int64_t r = 0; r < n; r++) h->rank[h->order[r]] = (int32_t)r;
}

/* community arrays for K ids, all empty */
static void alloc_partition(lfo *h, int32_t K)
{
    int64_t n = h->n;
    h->K = K;
    h->mem = (memb_t *)xcalloc((size_t)(n ? n : 1), sizeof(memb_t));
    h->cm = (cmem_t *)xcalloc((size_t)(K ? K : 1), sizeof(cmem_t));
    h->m = (int64_t *)xcalloc((size_t)(K ? K : 1), sizeof(int64_t));
    h->W = (double *)xcalloc((size_t)(K ? K : 1), sizeof(double));
    h->S0 = (xsum *)xcalloc((size_t)(K ? K : 1), sizeof(xsum));
    h->Sp = (xsum *)xcalloc((size_t)(K ? K : 1), sizeof(xsum));
    h->Sm = (xsum *)xcalloc((size_t)(K ? K : 1), sizeof(xsum));
}

/*
 * Node statistics and the greedy initial clustering: walk the nodes in order; a node
 * without a community opens a new one, and each of its neighbours that has no community
 * yet joins it.
 */
int lfo_init_communities(lfo *h, int nthreads)
{
    if (!h || !h->rowptr) return LFO_ESTATE;
    int64_t n = h->n;
    free_partition(h);
    node_statistics(h, nthreads);

    int32_t *comm_of = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    for (int64_t x = 0; x < n; x++) comm_of[x] = -1;
    int32_t K = 0;
    for (int64_t r = 0; r < n; r++) {
        int32_t x = h->order[r];
        if (comm_of[x] >= 0) continue;
        int32_t c = K++;
        comm_of[x] = c;
        for (int64_t e = h->rowptr[x]; e < h->rowptr[x + 1]; e++)
            if (comm_of[h->col[e]] < 0) comm_of[h->col[e]] = c;
    }
    alloc_partition(h, K);
    for (int64_t x = 0; x < n; x++) {
        int32_t i = 0;
        for (int64_t e = h->rowptr[x]; e < h->rowptr[x + 1]; e++) i += comm_of[h->col[e]] == comm_of[x];
        memb_insert(&h->mem[x], comm_of[x], i);
        cmem_add(&h->cm[comm_of[x]], (int32_t)x);
    }
    free(comm_of);
    for (int32_t c = 0; c < K; c++) refresh_comm(h, c);
    h->Wt = partition_score(h);
    h->inited = 1;
    h->iter_done = 0;
    return xs_err ? LFO_EOVERFLOW : LFO_OK;
}

/*
 * Warm start ("Initial Clustering": an existing division of the network can take the
 * place of the greedy one).  Node statistics and order are computed as for the greedy
 * start; the given memberships become the partition.  offsets[n + 1] (offsets[0] = 0,
 * non-decreasing, offsets[n] = total) and ids[total] list each node's communities in any
 * order, each id in [0, n_comms) and at most once per node; n_comms < 0 takes the largest
 * id + 1.  Empty and one-member communities are allowed, as after the greedy start.  Every
 * maintained quantity (in-counts, sizes, internal edges, exact sums, scores) is counted
 * from its definition.
 */
int lfo_init_from_memberships(lfo *h, const int64_t *offsets, const int32_t *ids, int64_t total,
                              int32_t n_comms, int nthreads)
{
    if (!h || !h->rowptr) return LFO_ESTATE;
    int64_t n = h->n;
    if (!offsets || (total > 0 && !ids) || total < 0) return LFO_EINVAL;
    if (offsets[0] != 0 || offsets[n] != total) {
        snprintf(h->err, sizeof h->err, "offsets must start at 0 and end at total");
        return LFO_EINVAL;
    }
    int64_t maxid = -1;
    for (int64_t x = 0; x < n; x++) {
        if (offsets[x + 1] < offsets[x]) {
            snprintf(h->err, sizeof h->err, "offsets decrease at node %lld", (long long)x);
            return LFO_EINVAL;
        }
        for (int64_t a = offsets[x]; a < offsets[x + 1]; a++) {
            if (ids[a] < 0 || (n_comms >= 0 && ids[a] >= n_comms)) {
                snprintf(h->err, sizeof h->err, "community id %d of node %lld out of range", ids[a], (long long)x);
                return LFO_EINVAL;
            }
            if (ids[a] > maxid) maxid = ids[a];
            for (int64_t b = offsets[x]; b < a; b++)
                if (ids[b] == ids[a]) {
                    snprintf(h->err, sizeof h->err, "node %lld lists community %d twice", (long long)x, ids[a]);
                    return LFO_EINVAL;
                }
        }
    }
    int32_t K = n_comms >= 0 ? n_comms : (int32_t)(maxid + 1);
    free_partition(h);
    node_statistics(h, nthreads);
    alloc_partition(h, K);
    for (int64_t x = 0; x < n; x++)
        for (int64_t a = offsets[x]; a < offsets[x + 1]; a++) {
            memb_insert(&h->mem[x], ids[a], 0);
            cmem_add(&h->cm[ids[a]], (int32_t)x);
        }
    /* i_x(C) = |N(x) ∩ C| for every membership, from the now complete member lists */
    for (int64_t x = 0; x < n; x++)
        for (int32_t j = 0; j < h->mem[x].cnt; j++) {
            int32_t c = h->mem[x].comm[j], i = 0;
            for (int64_t e = h->rowptr[x]; e < h->rowptr[x + 1]; e++) i += memb_find(&h->mem[h->col[e]], c) >= 0;
            h->mem[x].in[j] = i;
        }
    for (int32_t c = 0; c < K; c++) refresh_comm(h, c);
    h->Wt = partition_score(h);
    h->inited = 1;
    h->iter_done = 0;
    return xs_err ? LFO_EOVERFLOW : LFO_OK;
}

/* ------------------------------------------------------------------------------------ */
/* Node changes: the best join and the best leave of node x on the current state          */
/* ------------------------------------------------------------------------------------ */
typedef struct {
    int64_t *mark;      /* mark[y] == stamp  <=>  y in N(x) */
    int64_t *cseen;     /* cseen[c] == stamp <=>  c already a candidate */
    int32_t *cidx;      /* candidate index of c */
    int64_t stamp;
    int32_t ncap;
    int32_t *cand;      /* candidate communities */
    int32_t *kcnt;      /* |N(x) ∩ c| */
    xsum *acc;          /* factored mode: exact correction sums */
} scratch_t;

static void scratch_init(scratch_t *w, const lfo *h)
{
    w->mark = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)(h->n ? h->n : 1));
    w->cseen = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)(h->K ? h->K : 1));
    w->cidx = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(h->K ? h->K : 1));
    for (int64_t y = 0; y < h->n; y++) w->mark[y] = -1;
    for (int32_t c = 0; c < h->K; c++) w->cseen[c] = -1;
    w->stamp = 0;
    w->ncap = 64;
    w->cand = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)w->ncap);
    w->kcnt = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)w->ncap);
    w->acc = (xsum *)xmalloc(sizeof(xsum) * (size_t)w->ncap);
}

static void scratch_free(scratch_t *w)
{
    free(w->mark); free(w->cseen); free(w->cidx); free(w->cand); free(w->kcnt); free(w->acc);
}

static int32_t cand_slot(scratch_t *w, int32_t c, int32_t *ncand)
{
    if (w->cseen[c] == w->stamp) return w->cidx[c];
    if (*ncand == w->ncap) {
        w->ncap *= 2;
        w->cand = (int32_t *)realloc(w->cand, sizeof(int32_t) * (size_t)w->ncap);
        w->kcnt = (int32_t *)realloc(w->kcnt, sizeof(int32_t) * (size_t)w->ncap);
        w->acc = (xsum *)realloc(w->acc, sizeof(xsum) * (size_t)w->ncap);
        if (!w->cand || !w->kcnt || !w->acc) abort();
    }
    int32_t j = (*ncand)++;
    w->cseen[c] = w->stamp;
    w->cidx[c] = j;
    w->cand[j] = c;
    w->kcnt[j] = 0;
    xs_clear(&w->acc[j]);
    return j;
}

typedef struct { int32_t join, leave; double join_d, leave_d; } decision_t;

/* candidate list output for the debug entry point */
typedef struct { int32_t cap, n; int32_t *comm; double *delta; int32_t *is_leave; } cand_out_t;

static void consider(int32_t c, double d, int32_t *best, double *bestd)
{
    /* strictly positive change only; larger wins, equal -> lowest community id */
    if (!(d > 0.0)) return;
    if (*best < 0 || d > *bestd || (d == *bestd && c < *best)) { *best = c; *bestd = d; }
}

/*
 * Change of the cc-free partition score when x joins (or leaves) community c.  Only c's
 * own score changes: x's other communities keep their members, sizes and internal
 * degrees.  naive: R(sum over the members of C' of g at the new in-counts and size).
 */
static double delta_naive(const lfo *h, const scratch_t *w, int32_t x, int32_t c, int is_leave, int32_t k)
{
    const cmem_t *cm = &h->cm[c];
    int64_t s = cm->cnt;
    int64_t s2 = is_leave ? s - 1 : s + 1;
    int64_t m2 = is_leave ? h->m[c] - k : h->m[c] + k;
    xsum S;
    xs_clear(&S);
    for (int32_t j = 0; j < cm->cnt; j++) {
        int32_t y = cm->node[j];
        if (y == x) continue;
        int64_t i = in_of(h, y, c) + (w->mark[y] == w->stamp ? (is_leave ? -1 : 1) : 0);
        xs_add(&S, g_term(i, h->deg[y], s2));
    }
    if (!is_leave) xs_add(&S, g_term(k, h->deg[x], s2));
    double pS = density(s2, m2) * xs_round(&S);
    return pS - h->W[c];
}

/* factored: the same exact value from the stored S+ / S- plus x's neighbours' corrections */
static double delta_factored(const lfo *h, const scratch_t *w, int32_t j, int32_t x, int is_leave)
{
    int32_t c = w->cand[j];
    int64_t s = h->cm[c].cnt, k = w->kcnt[j];
    xsum S = is_leave ? h->Sm[c] : h->Sp[c];
    xs_add_xs(&S, &w->acc[j]);
    double pS;
    if (is_leave) {
        xs_add(&S, -g_term(k, h->deg[x], s - 1));
        pS = density(s - 1, h->m[c] - k) * xs_round(&S);
    } else {
        xs_add(&S, g_term(k, h->deg[x], s + 1));
        pS = density(s + 1, h->m[c] + k) * xs_round(&S);
    }
    return pS - h->W[c];
}

static void eval_node(const lfo *h, scratch_t *w, int32_t x, int mode, decision_t *out, cand_out_t *co)
{
    w->stamp++;
    int32_t ncand = 0;
    const memb_t *mx = &h->mem[x];
    for (int64_t e = h->rowptr[x]; e < h->rowptr[x + 1]; e++) w->mark[h->col[e]] = w->stamp;
    /* leave candidates: every community of x (even with no neighbour in it) */
    for (int32_t a = 0; a < mx->cnt; a++) cand_slot(w, mx->comm[a], &ncand);
    /* join candidates: communities of x's neighbours that x is not part of */
    for (int64_t e = h->rowptr[x]; e < h->rowptr[x + 1]; e++) {
        int32_t y = h->col[e];
        const memb_t *my = &h->mem[y];
        for (int32_t a = 0; a < my->cnt; a++) {
            int32_t c = my->comm[a];
            int32_t j = cand_slot(w, c, &ncand);
            w->kcnt[j]++;
            if (mode & 1) {
                int64_t i = my->in[a], d = h->deg[y], s = h->cm[c].cnt;
                int is_leave = memb_find(mx, c) >= 0;
                if (is_leave) {
                    xs_add(&w->acc[j], g_term(i - 1, d, s - 1));
                    xs_add(&w->acc[j], -g_term(i, d, s - 1));
                } else {
                    xs_add(&w->acc[j], g_term(i + 1, d, s + 1));
                    xs_add(&w->acc[j], -g_term(i, d, s + 1));
                }
            }
        }
    }
    decision_t r = { -1, -1, 0.0, 0.0 };
    if (co) co->n = 0;
    for (int32_t j = 0; j < ncand; j++) {
        int32_t c = w->cand[j];
        int32_t ia = memb_find(mx, c);
        int is_leave = ia >= 0;
        if (is_leave && w->kcnt[j] != mx->in[ia]) { fprintf(stderr, "lfo: in-count mismatch\n"); abort(); }
        double d = (mode & 1) ? delta_factored(h, w, j, x, is_leave)
                              : delta_naive(h, w, x, c, is_leave, w->kcnt[j]);
        if (is_leave) consider(c, d, &r.leave, &r.leave_d);
        else consider(c, d, &r.join, &r.join_d);
        if (co && co->n < co->cap) {
            co->comm[co->n] = c; co->delta[co->n] = d; co->is_leave[co->n] = is_leave; co->n++;
        }
    }
    *out = r;
}

/* ------------------------------------------------------------------------------------ */
/* Bulk apply of one queue's decisions                                                    */
/* ------------------------------------------------------------------------------------ */
static void apply_chunk(lfo *h, const int32_t *nodes, int32_t cnt, const decision_t *dec, int mode,
                        int32_t *joined_to, char *touched, int32_t *tlist)
{
    int32_t nt = 0;
    for (int32_t j = 0; j < cnt; j++) {
        int32_t x = nodes[j];
        if (dec[j].leave >= 0) {
            int32_t c = dec[j].leave;
            memb_remove(&h->mem[x], c);
            cmem_remove(&h->cm[c], x);
            if (!touched[c]) { touched[c] = 1; tlist[nt++] = c; }
        }
        if (dec[j].join >= 0) {
            int32_t c = dec[j].join;
            memb_insert(&h->mem[x], c, 0);
            cmem_add(&h->cm[c], x);
            joined_to[x] = c;
            if (!touched[c]) { touched[c] = 1; tlist[nt++] = c; }
        }
    }
    if (mode & 2) {
        /* incremental in-counts: a surviving member y of c gains one per neighbour that
           joined c and loses one per neighbour that left c; a new member is counted fresh */
        for (int32_t j = 0; j < cnt; j++) {
            int32_t x = nodes[j], J = dec[j].join, L = dec[j].leave;
            if (J < 0 && L < 0) continue;
            int32_t fresh = 0;
            for (int64_t e = h->rowptr[x]; e < h->rowptr[x + 1]; e++) {
                int32_t y = h->col[e];
                memb_t *my = &h->mem[y];
                if (J >= 0) {
                    int32_t a = memb_find(my, J);
                    if (a >= 0) { fresh++; if (joined_to[y] != J) my->in[a]++; }
                }
                if (L >= 0) {
                    int32_t a = memb_find(my, L);
                    if (a >= 0 && joined_to[y] != L) my->in[a]--;
                }
            }
            if (J >= 0) h->mem[x].in[memb_find(&h->mem[x], J)] = fresh;
        }
    } else {
        /* from scratch: every member of a touched community recounts its neighbours in it */
        for (int32_t t = 0; t < nt; t++) {
            int32_t c = tlist[t];
            const cmem_t *cm = &h->cm[c];
            for (int32_t a = 0; a < cm->cnt; a++) {
                int32_t y = cm->node[a];
                int32_t i = 0;
                for (int64_t e = h->rowptr[y]; e < h->rowptr[y + 1]; e++)
                    i += memb_find(&h->mem[h->col[e]], c) >= 0;
                h->mem[y].in[memb_find(&h->mem[y], c)] = i;
            }
        }
    }
    for (int32_t t = 0; t < nt; t++) { refresh_comm(h, tlist[t]); touched[tlist[t]] = 0; }
    for (int32_t j = 0; j < cnt; j++) joined_to[nodes[j]] = -1;
}

/* from-scratch recount of every maintained quantity; returns the number of mismatches */
int64_t lfo_check_state(lfo *h)
{
    if (!h || !h->inited) return -1;
    int64_t bad = 0;
    for (int64_t x = 0; x < h->n; x++) {
        const memb_t *mx = &h->mem[x];
        for (int32_t a = 0; a < mx->cnt; a++) {
            int32_t c = mx->comm[a], i = 0;
            if (a > 0 && mx->comm[a - 1] >= c) bad++;
            for (int64_t e = h->rowptr[x]; e < h->rowptr[x + 1]; e++) i += memb_find(&h->mem[h->col[e]], c) >= 0;
            if (i != mx->in[a]) bad++;
        }
    }
    int32_t *cnt = (int32_t *)xcalloc((size_t)(h->K ? h->K : 1), sizeof(int32_t));
    for (int64_t x = 0; x < h->n; x++)
        for (int32_t a = 0; a < h->mem[x].cnt; a++) cnt[h->mem[x].comm[a]]++;
    for (int32_t c = 0; c < h->K; c++) {
        if (cnt[c] != h->cm[c].cnt) bad++;
        for (int32_t a = 0; a < h->cm[c].cnt; a++) if (memb_find(&h->mem[h->cm[c].node[a]], c) < 0) bad++;
        int64_t mm = 0;
        for (int32_t a = 0; a < h->cm[c].cnt; a++) {
            int32_t y = h->cm[c].node[a];
            for (int64_t e = h->rowptr[y]; e < h->rowptr[y + 1]; e++)
                mm += (h->col[e] > y) && memb_find(&h->mem[h->col[e]], c) >= 0;
        }
        if (mm != h->m[c]) bad++;
        double W = h->W[c];
        xsum S0 = h->S0[c], Sp = h->Sp[c], Sm = h->Sm[c];
        refresh_comm(h, c);
        if (W != h->W[c] || memcmp(&S0, &h->S0[c], sizeof S0) || memcmp(&Sp, &h->Sp[c], sizeof Sp) ||
            memcmp(&Sm, &h->Sm[c], sizeof Sm)) bad++;
    }
    free(cnt);
    return bad;
}

/* "Post-processing": communities with fewer than two members are removed */
static void end_iteration(lfo *h)
{
    for (int32_t c = 0; c < h->K; c++) {
        if (h->cm[c].cnt == 1) {
            int32_t y = h->cm[c].node[0];
            memb_remove(&h->mem[y], c);
            h->cm[c].cnt = 0;
            refresh_comm(h, c);
        }
    }
    h->Wt = partition_score(h);
}

int lfo_run_iterations(lfo *h, int32_t q, double theta, int32_t max_iters, int32_t mode,
                       int32_t nthreads, int32_t check_every_chunk, lfo_run_info *info)
{
    if (!h) return LFO_EINVAL;
    if (!h->inited) { snprintf(h->err, sizeof h->err, "init_communities not called"); return LFO_ESTATE; }
    if (q < 1 || isnan(theta) || theta < 0.0 || max_iters < 0) {
        snprintf(h->err, sizeof h->err, "bad argument");
        return LFO_EINVAL;
    }
    if (nthreads < 1) nthreads = 1;
    info->iterations = 0; info->converged = 0; info->hit_max = 0;
    if (info->wtilde_hist) info->wtilde_hist[0] = h->Wt;
    if (h->cc == 0.0) {       /* no triangle: every WCC-hat is 0, nothing to optimise */
        info->converged = 1;
        info->wtilde = h->Wt;
        info->wcc_hat = 0.0;
        return LFO_OK;
    }
    int64_t n = h->n;
    int32_t *joined_to = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    for (int64_t x = 0; x < n; x++) joined_to[x] = -1;
    char *touched = (char *)xcalloc((size_t)(h->K ? h->K : 1), 1);
    int32_t *tlist = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(2 * (int64_t)q + 2));
    int64_t qq = q < n ? q : (n ? n : 1);
    decision_t *dec = (decision_t *)xmalloc(sizeof(decision_t) * (size_t)qq);
    scratch_t *ws = (scratch_t *)xmalloc(sizeof(scratch_t) * (size_t)nthreads);
    for (int t = 0; t < nthreads; t++) scratch_init(&ws[t], h);
    double prev = h->Wt;
    int rc = LFO_OK;
    h->chunks_done = 0;
    for (int32_t it = 0; it < max_iters; it++) {
        int64_t joins = 0, leaves = 0;
        for (int64_t start = 0; start < n; start += q) {
            /* a timing sample ends after a fixed number of queues, mid-iteration */
            if (h->chunk_limit > 0 && h->chunks_done >= h->chunk_limit) goto done;
            int32_t cnt = (int32_t)((n - start) < q ? (n - start) : q);
            const int32_t *nodes = h->order + start;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
            for (int32_t j = 0; j < cnt; j++) {
                int tid = 0;
#ifdef _OPENMP
                tid = omp_get_thread_num();
#endif
                eval_node(h, &ws[tid], nodes[j], mode, &dec[j], NULL);
            }
            for (int32_t j = 0; j < cnt; j++) { joins += dec[j].join >= 0; leaves += dec[j].leave >= 0; }
            apply_chunk(h, nodes, cnt, dec, mode, joined_to, touched, tlist);
            h->chunks_done++;
            if (check_every_chunk && lfo_check_state(h) != 0) {
                snprintf(h->err, sizeof h->err, "state check failed (iteration %d, chunk at %lld)",
                         it + 1, (long long)start);
                rc = LFO_ESTATE;
                goto done;
            }
        }
        end_iteration(h);
        h->iter_done++;
        info->iterations = it + 1;
        if (info->wtilde_hist) info->wtilde_hist[it + 1] = h->Wt;
        if (info->joins) info->joins[it] = joins;
        if (info->leaves) info->leaves[it] = leaves;
        if (info->communities) {
            int64_t live = 0;
            for (int32_t c = 0; c < h->K; c++) live += h->cm[c].cnt >= 2;
            info->communities[it] = live;
        }
        /* "Stopping Criteria": relative improvement against the previous iteration */
        int stop = (prev == 0.0) || ((h->Wt - prev) / prev < theta);
        prev = h->Wt;
        if (stop) { info->converged = 1; break; }
    }
    if (!info->converged && info->iterations == max_iters) info->hit_max = 1;
done:
    for (int t = 0; t < nthreads; t++) scratch_free(&ws[t]);
    free(ws); free(dec); free(tlist); free(touched); free(joined_to);
    info->wtilde = h->Wt;
    info->wcc_hat = h->Wt / h->cc;
    if (xs_err) rc = LFO_EOVERFLOW;
    return rc;
}

/* ------------------------------------------------------------------------------------ */
/* Getters and debug entry points                                                        */
/* ------------------------------------------------------------------------------------ */
int64_t lfo_num_nodes(lfo *h) { return h ? h->n : -1; }
/* Timing samples: lfo_run_iterations stops after `limit` queues (0 = no limit); the
   state is then mid-iteration and only good for timing.  lfo_chunks_done: queues the last
   lfo_run_iterations evaluated and applied. */
void lfo_set_chunk_limit(lfo *h, int64_t limit) { if (h) h->chunk_limit = limit > 0 ? limit : 0; }
int64_t lfo_chunks_done(lfo *h) { return h ? h->chunks_done : -1; }
int64_t lfo_num_edges(lfo *h) { return h ? h->nedges : -1; }
int32_t lfo_num_communities_created(lfo *h) { return h ? h->K : -1; }

int lfo_get_csr(lfo *h, int64_t *rowptr, int32_t *col)
{
    if (!h || !h->rowptr) return LFO_ESTATE;
    memcpy(rowptr, h->rowptr, sizeof(int64_t) * (size_t)(h->n + 1));
    memcpy(col, h->col, sizeof(int32_t) * (size_t)(2 * h->nedges));
    return LFO_OK;
}

int lfo_get_orig_ids(lfo *h, int64_t *ids)
{
    if (!h || !h->rowptr) return LFO_ESTATE;
    memcpy(ids, h->orig_id, sizeof(int64_t) * (size_t)h->n);
    return LFO_OK;
}

int lfo_get_node_stats(lfo *h, int64_t *tri, double *ccl, int32_t *order)
{
    if (!h || !h->inited) return LFO_ESTATE;
    if (tri) memcpy(tri, h->tri, sizeof(int64_t) * (size_t)h->n);
    if (ccl) memcpy(ccl, h->ccl, sizeof(double) * (size_t)h->n);
    if (order) memcpy(order, h->order, sizeof(int32_t) * (size_t)h->n);
    return LFO_OK;
}

int lfo_get_scores(lfo *h, double *wcc_hat, double *cc, int64_t *triangles, double *wtilde)
{
    if (!h || !h->inited) return LFO_ESTATE;
    if (cc) *cc = h->cc;
    if (triangles) *triangles = h->T;
    if (wtilde) *wtilde = h->Wt;
    if (wcc_hat) *wcc_hat = h->cc > 0.0 ? h->Wt / h->cc : 0.0;
    return LFO_OK;
}

int lfo_get_memberships(lfo *h, int64_t *offsets, int32_t *comm_ids, int64_t capacity, int64_t *total)
{
    if (!h || !h->inited) return LFO_ESTATE;
    int64_t tot = 0;
    for (int64_t x = 0; x < h->n; x++) tot += h->mem[x].cnt;
    *total = tot;
    if (!offsets || !comm_ids) return LFO_OK;
    if (capacity < tot) return LFO_ERANGE;
    int64_t p = 0;
    for (int64_t x = 0; x < h->n; x++) {
        offsets[x] = p;
        for (int32_t a = 0; a < h->mem[x].cnt; a++) comm_ids[p++] = h->mem[x].comm[a];
    }
    offsets[h->n] = p;
    return LFO_OK;
}

/* ------------------------------------------------------------------------------------ */
/* Exact WCC of the current partition (WCC paragraph of the WCC-hat subsection)          */
/* ------------------------------------------------------------------------------------ */
static int row_has(const lfo *h, int32_t x, int32_t z)   /* z in N(x)? (rows are sorted) */
{
    int64_t lo = h->rowptr[x], hi = h->rowptr[x + 1] - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (h->col[mid] == z) return 1;
        if (h->col[mid] < z) lo = mid + 1; else hi = mid - 1;
    }
    return 0;
}

/*
 * The WCC terms of node x, one per community C of x (ascending ids):
 *   t(x,C)     triangles of x whose two other nodes are both in C,
 *   t(x,V)     all triangles of x (k_x),
 *   vt(x,S)    nodes of S that close at least one triangle with x (the third node anywhere),
 *   WCC(x,C) = t(x,C) / t(x,V) * vt(x,V) / (|C \ {x}| + vt(x,V \ C)), 0 if t(x,V) = 0,
 * evaluated in FP64 as  (t / t_V) * (vt_V / (|C| - 1 + vt_{V\C}))  (three roundings).
 * Outputs t, vtc, w per community of x, and *vtx = vt(x,V).
 */
static void wcc_node_terms(const lfo *h, int32_t x, int32_t *has, int32_t *t, int32_t *vtc, double *w,
                           int32_t *vtx)
{
    const int64_t r0 = h->rowptr[x], d = h->rowptr[x + 1] - r0;
    int32_t vt = 0;
    for (int64_t a = 0; a < d; a++) {          /* does the edge x-y close a triangle? */
        int32_t y = h->col[r0 + a];
        has[a] = 0;
        for (int64_t f = h->rowptr[y]; f < h->rowptr[y + 1] && !has[a]; f++) has[a] = row_has(h, x, h->col[f]);
        vt += has[a];
    }
    *vtx = vt;
    const memb_t *mx = &h->mem[x];
    for (int32_t k = 0; k < mx->cnt; k++) {
        const int32_t c = mx->comm[k];
        int64_t twice = 0;
        int32_t out = 0;
        for (int64_t a = 0; a < d; a++) {
            int32_t y = h->col[r0 + a];
            const int y_in = memb_find(&h->mem[y], c) >= 0;
            if (has[a] && !y_in) out++;
            if (!y_in) continue;
            for (int64_t f = h->rowptr[y]; f < h->rowptr[y + 1]; f++) {
                int32_t z = h->col[f];
                if (memb_find(&h->mem[z], c) >= 0 && row_has(h, x, z)) twice++;   /* each pair twice */
            }
        }
        t[k] = (int32_t)(twice / 2);
        vtc[k] = out;
        const int64_t kx = h->tri[x], s = h->cm[c].cnt;
        w[k] = kx > 0 ? ((double)t[k] / (double)kx) * ((double)vt / (double)(s - 1 + out)) : 0.0;
    }
}

/*
 * WCC(P) = sum over communities C of WCC(C), WCC(C) = sum over x in C of WCC(x,C), both
 * summed exactly and rounded once.  Optional outputs (NULL to skip): wcc_comm[K] per
 * community id; per membership in the lfo_get_memberships order: wcc_node, t_xc, vt_xc;
 * vt_x[n] = vt(x,V).
 */
int lfo_exact_wcc(lfo *h, int nthreads, double *wcc, double *wcc_comm, double *wcc_node, int32_t *t_xc,
                  int32_t *vt_xc, int32_t *vt_x)
{
    if (!h || !h->inited || !wcc) return LFO_ESTATE;
    const int64_t n = h->n;
    int64_t *mo = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)(n + 1));
    mo[0] = 0;
    for (int64_t x = 0; x < n; x++) mo[x + 1] = mo[x] + h->mem[x].cnt;
    const int64_t tot = mo[n];
    int32_t *t = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(tot ? tot : 1));
    int32_t *vc = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(tot ? tot : 1));
    double *w = (double *)xmalloc(sizeof(double) * (size_t)(tot ? tot : 1));
    int32_t *vx = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel num_threads(nthreads)
    {
        int64_t maxd = 1;
        for (int64_t x = 0; x < n; x++) if (h->rowptr[x + 1] - h->rowptr[x] > maxd) maxd = h->rowptr[x + 1] - h->rowptr[x];
        int32_t *has = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)maxd);
#pragma omp for schedule(dynamic, 16)
        for (int64_t x = 0; x < n; x++) wcc_node_terms(h, (int32_t)x, has, t + mo[x], vc + mo[x], w + mo[x], vx + x);
        free(has);
    }
    xsum all;
    xs_clear(&all);
    xsum *per = (xsum *)xcalloc((size_t)(h->K ? h->K : 1), sizeof(xsum));
    for (int64_t x = 0; x < n; x++)
        for (int32_t k = 0; k < h->mem[x].cnt; k++) {
            xs_add(&all, w[mo[x] + k]);
            xs_add(&per[h->mem[x].comm[k]], w[mo[x] + k]);
        }
    *wcc = xs_round(&all);
    if (wcc_comm)
        for (int32_t c = 0; c < h->K; c++) wcc_comm[c] = xs_round(&per[c]);
    if (wcc_node) memcpy(wcc_node, w, sizeof(double) * (size_t)tot);
    if (t_xc) memcpy(t_xc, t, sizeof(int32_t) * (size_t)tot);
    if (vt_xc) memcpy(vt_xc, vc, sizeof(int32_t) * (size_t)tot);
    if (vt_x) memcpy(vt_x, vx, sizeof(int32_t) * (size_t)n);
    free(per); free(mo); free(t); free(vc); free(w); free(vx);
    return xs_err ? LFO_EOVERFLOW : LFO_OK;
}

/* the WCC terms of the listed nodes only (their memberships in ascending id order, the
   nodes one after another), for spot checks of large graphs */
int lfo_wcc_sample(lfo *h, const int32_t *nodes, int64_t count, double *wcc_node, int32_t *t_xc,
                   int32_t *vt_xc, int32_t *vt_x)
{
    if (!h || !h->inited) return LFO_ESTATE;
    int64_t p = 0;
    for (int64_t i = 0; i < count; i++) {
        int32_t x = nodes[i];
        if (x < 0 || x >= h->n) return LFO_EINVAL;
        int64_t d = h->rowptr[x + 1] - h->rowptr[x];
        int32_t *has = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(d ? d : 1));
        wcc_node_terms(h, x, has, t_xc + p, vt_xc + p, wcc_node + p, vt_x + i);
        free(has);
        p += h->mem[x].cnt;
    }
    return LFO_OK;
}

/* ------------------------------------------------------------------------------------ */
/* Post-processing of the final cover ("Post-processing": duplicated and contained       */
/* communities may be unwanted)                                                           */
/* ------------------------------------------------------------------------------------ */
/* is every member of community a also a member of community b? */
static int comm_subset(const lfo *h, int32_t a, int32_t b)
{
    for (int32_t j = 0; j < h->cm[a].cnt; j++)
        if (memb_find(&h->mem[h->cm[a].node[j]], b) < 0) return 0;
    return 1;
}

/*
 * Communities with at least one member are compared pairwise.  With LFO_PP_DUPLICATES a
 * community is removed if another one has exactly its members and a lower id; with
 * LFO_PP_CONTAINED if its members are a strict subset of another one's.  keep[K] (may be
 * NULL) receives 1 for every community kept (0 for removed and for empty ids);
 * removed[0] / removed[1] (may be NULL) count removals as duplicates / as contained (a
 * community that is both counts as a duplicate).  With LFO_PP_APPLY the removed
 * communities lose all their members and the state is rebuilt from the remaining cover
 * as by lfo_init_from_memberships.
 */
#define LFO_PP_DUPLICATES 1u
#define LFO_PP_CONTAINED 2u
#define LFO_PP_APPLY 4u
int lfo_postprocess(lfo *h, uint32_t flags, uint8_t *keep, int64_t *removed, int nthreads)
{
    if (!h || !h->inited) return LFO_ESTATE;
    const int32_t K = h->K;
    uint8_t *kp = (uint8_t *)xmalloc((size_t)(K ? K : 1));
    int64_t ndup = 0, ncont = 0;
    for (int32_t a = 0; a < K; a++) {
        const int32_t sa = h->cm[a].cnt;
        kp[a] = sa > 0;
        if (sa == 0) continue;
        int dup = 0, cont = 0;
        for (int32_t b = 0; b < K; b++) {
            if (b == a) continue;
            const int32_t sb = h->cm[b].cnt;
            if (sb < sa) continue;
            if (sb == sa && !((flags & LFO_PP_DUPLICATES) && b < a)) continue;
            if (sb > sa && !(flags & LFO_PP_CONTAINED)) continue;
            if (!comm_subset(h, a, b)) continue;
            if (sb == sa) dup = 1; else cont = 1;
        }
        if (dup) ndup++;
        else if (cont) ncont++;
        if (dup || cont) kp[a] = 0;
    }
    if (keep) memcpy(keep, kp, (size_t)K);
    if (removed) { removed[0] = ndup; removed[1] = ncont; }
    int rc = LFO_OK;
    if (flags & LFO_PP_APPLY) {
        const int64_t n = h->n;
        int64_t *off = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)(n + 1));
        int64_t tot = 0;
        for (int64_t x = 0; x < n; x++) tot += h->mem[x].cnt;
        int32_t *ids = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(tot ? tot : 1));
        int64_t p = 0;
        for (int64_t x = 0; x < n; x++) {
            off[x] = p;
            for (int32_t j = 0; j < h->mem[x].cnt; j++)
                if (kp[h->mem[x].comm[j]]) ids[p++] = h->mem[x].comm[j];
        }
        off[n] = p;
        rc = lfo_init_from_memberships(h, off, ids, p, K, nthreads);
        free(off);
        free(ids);
    }
    free(kp);
    return rc;
}

/* ------------------------------------------------------------------------------------ */
/* F1-Score of the partition against a reference cover (Methods, "F1-Score for           */
/* Overlapping Communities")                                                              */
/* ------------------------------------------------------------------------------------ */
/*
 * F1-Score(P', P) = (1 / |P'|) * sum over C' in P' of max over C in P of F1(C', C), with
 * precision |C n C'| / |C'|, recall |C n C'| / |C| and F1 their harmonic mean, which is
 * the rational 2 |C n C'| / (|C| + |C'|); it is evaluated as that one correctly rounded
 * division.  P' = the communities of the current partition with at least one member, P =
 * the non-empty communities of the reference cover (offsets[n + 1], ids; each id at most
 * once per node).  The maxima are summed exactly, rounded once, then divided by |P'|
 * (0 if P' is empty).  Optional per-id outputs (length K, 0 / -1 for empty ids): best[c]
 * the maximum F1 of community c, match[c] the lowest reference id reaching it (-1 if no
 * reference community meets c).
 */
int lfo_cover_f1(lfo *h, const int64_t *offsets, const int32_t *ids, int64_t total, double *f1, double *best,
                 int32_t *match)
{
    if (!h || !h->inited || !f1) return LFO_ESTATE;
    const int64_t n = h->n;
    if (offsets[0] != 0 || offsets[n] != total) return LFO_EINVAL;
    int32_t R = 0;
    for (int64_t x = 0; x < n; x++) {
        if (offsets[x + 1] < offsets[x]) return LFO_EINVAL;
        for (int64_t a = offsets[x]; a < offsets[x + 1]; a++) {
            if (ids[a] < 0) return LFO_EINVAL;
            for (int64_t b = offsets[x]; b < a; b++)
                if (ids[b] == ids[a]) return LFO_EINVAL;
            if (ids[a] + 1 > R) R = ids[a] + 1;
        }
    }
    int64_t *rsize = (int64_t *)xcalloc((size_t)(R ? R : 1), sizeof(int64_t));
    for (int64_t a = 0; a < total; a++) rsize[ids[a]]++;
    int64_t *inter = (int64_t *)xcalloc((size_t)(R ? R : 1), sizeof(int64_t));
    int32_t *touched = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(R ? R : 1));
    xsum acc;
    xs_clear(&acc);
    int64_t live = 0;
    for (int32_t c = 0; c < h->K; c++) {
        const cmem_t *cm = &h->cm[c];
        if (best) best[c] = 0.0;
        if (match) match[c] = -1;
        if (cm->cnt == 0) continue;
        live++;
        int32_t nt = 0;                       /* |C' n C| for every reference C meeting C' */
        for (int32_t j = 0; j < cm->cnt; j++) {
            const int32_t x = cm->node[j];
            for (int64_t a = offsets[x]; a < offsets[x + 1]; a++) {
                if (inter[ids[a]]++ == 0) touched[nt++] = ids[a];
            }
        }
        double mx = 0.0;
        int32_t arg = -1;
        for (int32_t k = 0; k < nt; k++) {
            const int32_t r = touched[k];
            const double f = (double)(2 * inter[r]) / (double)(rsize[r] + cm->cnt);
            if (arg < 0 || f > mx || (f == mx && r < arg)) { mx = f; arg = r; }
            inter[r] = 0;
        }
        xs_add(&acc, mx);
        if (best) best[c] = mx;
        if (match) match[c] = arg;
    }
    *f1 = live > 0 ? xs_round(&acc) / (double)live : 0.0;
    free(rsize); free(inter); free(touched);
    return xs_err ? LFO_EOVERFLOW : LFO_OK;
}

/* per-community size, internal edges and cc-free score (all created ids) */
int lfo_get_communities(lfo *h, int32_t *size, int64_t *m, double *W)
{
    if (!h || !h->inited) return LFO_ESTATE;
    for (int32_t c = 0; c < h->K; c++) {
        if (size) size[c] = h->cm[c].cnt;
        if (m) m[c] = h->m[c];
        if (W) W[c] = h->W[c];
    }
    return LFO_OK;
}

/* in-counts parallel to the membership listing of lfo_get_memberships */
int lfo_get_in_counts(lfo *h, int32_t *in, int64_t capacity)
{
    if (!h || !h->inited) return LFO_ESTATE;
    int64_t p = 0;
    for (int64_t x = 0; x < h->n; x++)
        for (int32_t a = 0; a < h->mem[x].cnt; a++) {
            if (p >= capacity) return LFO_ERANGE;
            in[p++] = h->mem[x].in[a];
        }
    return LFO_OK;
}

/* every candidate of node x on the current state, with its change of the cc-free score */
int lfo_eval_node(lfo *h, int32_t x, int32_t mode, int32_t cap, int32_t *comm, double *delta,
                  int32_t *is_leave, int32_t *ncand, int32_t *best_join, double *join_d,
                  int32_t *best_leave, double *leave_d)
{
    if (!h || !h->inited) return LFO_ESTATE;
    if (x < 0 || x >= h->n) return LFO_EINVAL;
    scratch_t w;
    scratch_init(&w, h);
    cand_out_t co = { cap, 0, comm, delta, is_leave };
    decision_t r;
    eval_node(h, &w, x, mode, &r, comm ? &co : NULL);
    scratch_free(&w);
    if (ncand) *ncand = co.n;
    *best_join = r.join; *join_d = r.join_d;
    *best_leave = r.leave; *leave_d = r.leave_d;
    return LFO_OK;
}

/* exact sum of v[0..n) rounded once to nearest-even (pins the accumulator) */
double lfo_exact_sum(const double *v, int64_t n)
{
    xsum a;
    xs_clear(&a);
    for (int64_t j = 0; j < n; j++) xs_add(&a, v[j]);
    return xs_round(&a);
}

double lfo_g(int64_t i, int64_t d, int64_t s) { return g_term(i, d, s); }
double lfo_density(int64_t s, int64_t m) { return density(s, m); }
int lfo_xs_error(void) { return xs_err; }
