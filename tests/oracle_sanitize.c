/*
 * Driver that runs the CPU oracle (oracle/lfo.c) under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built by tests/test_oracle_sanitize.py; test
 * infrastructure only).  Every check is a pin that holds independently of the oracle:
 *  - complete graph K_n: every node's clustering coefficient is 1, the greedy initial
 *    clustering puts all nodes in one community, W-tilde = n and no move improves it, so
 *    the run stops after one iteration (closed form of the WCC-hat estimator);
 *  - path 0-1-2-3-4: all clustering coefficients are 0, so the order is degree
 *    descending then id ascending, [1, 2, 3, 0, 4], and the greedy clustering gives
 *    {0, 1, 2} and {3, 4} (Methods, "Node Order", "Initial Clustering");
 *  - a triangle-free graph (even cycle): cc = 0, nothing to optimise, 0 iterations;
 *  - random graphs: the naive mode (every candidate re-summed) and the factored mode
 *    (stored exact sums plus corrections) give the same memberships and the same score
 *    bits, at one thread and at four, with the state re-checked after every queue;
 *  - the other entry points (warm start, exact WCC, post-processing, F1, prefix runs)
 *    run once on the final cover without a sanitizer report.
 * Prints "sanitize ok" and exits 0 when every check passes.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct lfo lfo;
typedef struct {
    int32_t iterations, converged, hit_max, pad;
    double wcc_hat, wtilde;
    double *wtilde_hist;
    int64_t *joins, *leaves, *communities;
} run_info;

lfo *lfo_create(void);
void lfo_destroy(lfo *h);
const char *lfo_last_error(lfo *h);
int lfo_load_graph(lfo *h, int64_t n, int64_t npairs, const int64_t *src, const int64_t *dst, uint32_t flags);
int lfo_init_communities(lfo *h, int nthreads);
int lfo_init_from_memberships(lfo *h, const int64_t *offsets, const int32_t *ids, int64_t total, int32_t n_comms,
                              int nthreads);
int lfo_run_iterations(lfo *h, int32_t q, double theta, int32_t max_iters, int32_t mode, int32_t nthreads,
                       int32_t check_every_chunk, run_info *info);
int64_t lfo_num_nodes(lfo *h);
int32_t lfo_num_communities_created(lfo *h);
int lfo_get_node_stats(lfo *h, int64_t *tri, double *ccl, int32_t *order);
int lfo_get_scores(lfo *h, double *wcc_hat, double *cc, int64_t *triangles, double *wtilde);
int lfo_get_memberships(lfo *h, int64_t *offsets, int32_t *comm_ids, int64_t capacity, int64_t *total);
int lfo_exact_wcc(lfo *h, int nthreads, double *wcc, double *wcc_comm, double *wcc_node, int32_t *t_xc,
                  int32_t *vt_out, int32_t *vt);
int lfo_postprocess(lfo *h, uint32_t flags, uint8_t *keep, int64_t *removed, int nthreads);
int lfo_cover_f1(lfo *h, const int64_t *offsets, const int32_t *ids, int64_t total, double *f1, double *best,
                 int32_t *match);
void lfo_set_chunk_limit(lfo *h, int64_t limit);
int64_t lfo_chunks_done(lfo *h);

static int failures = 0;
#define CHECK(cond, ...)                                                                   \
    do {                                                                                   \
        if (!(cond)) {                                                                     \
            fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__);                           \
            fprintf(stderr, __VA_ARGS__);                                                  \
            fprintf(stderr, "\n");                                                         \
            failures++;                                                                    \
        }                                                                                  \
    } while (0)

static lfo *load(int64_t n, int64_t m, const int64_t *s, const int64_t *d)
{
    lfo *h = lfo_create();
    CHECK(lfo_load_graph(h, n, m, s, d, 0) == 0, "load: %s", lfo_last_error(h));
    return h;
}

static run_info run(lfo *h, int q, int mode, int threads, double *hist)
{
    run_info ri;
    memset(&ri, 0, sizeof ri);
    ri.wtilde_hist = hist;
    CHECK(lfo_run_iterations(h, q, 0.01, 20, mode, threads, 1, &ri) == 0, "run: %s", lfo_last_error(h));
    return ri;
}

static void complete_graphs(void)
{
    for (int n = 3; n <= 10; n++) {
        int64_t s[64], d[64], m = 0;
        for (int a = 0; a < n; a++)
            for (int b = a + 1; b < n; b++) { s[m] = a; d[m] = b; m++; }
        lfo *h = load(n, m, s, d);
        CHECK(lfo_init_communities(h, 1) == 0, "init");
        double ccl[16];
        int64_t tri[16];
        int32_t order[16];
        lfo_get_node_stats(h, tri, ccl, order);
        for (int x = 0; x < n; x++) {
            CHECK(ccl[x] == 1.0, "K_%d cc(%d) = %g", n, x, ccl[x]);
            CHECK(tri[x] == (int64_t)(n - 1) * (n - 2) / 2, "K_%d triangles", n);
        }
        CHECK(lfo_num_communities_created(h) == 1, "K_%d: one initial community", n);
        double hist[32];
        run_info ri = run(h, 4, 3, 2, hist);
        CHECK(ri.iterations == 1 && ri.converged, "K_%d: one iteration", n);
        CHECK(ri.wtilde == (double)n, "K_%d: W-tilde %g != %d", n, ri.wtilde, n);
        lfo_destroy(h);
    }
}

static void path5(void)
{
    int64_t s[4] = {0, 1, 2, 3}, d[4] = {1, 2, 3, 4};
    lfo *h = load(5, 4, s, d);
    CHECK(lfo_init_communities(h, 1) == 0, "init");
    int64_t tri[5];
    double ccl[5];
    int32_t order[5];
    lfo_get_node_stats(h, tri, ccl, order);
    const int32_t want[5] = {1, 2, 3, 0, 4};
    for (int k = 0; k < 5; k++) CHECK(order[k] == want[k], "path order[%d] = %d", k, order[k]);
    int64_t off[6], total = 0;
    int32_t ids[16];
    CHECK(lfo_get_memberships(h, off, ids, 16, &total) == 0 && total == 5, "path memberships");
    const int32_t comm[5] = {0, 0, 0, 1, 1};
    for (int x = 0; x < 5; x++) CHECK(ids[off[x]] == comm[x], "path community of %d", x);
    double hist[32];
    run_info ri = run(h, 2, 3, 1, hist);
    CHECK(ri.iterations == 0 && ri.converged, "triangle-free path: 0 iterations");
    lfo_destroy(h);
    int64_t cs[8], cd[8];            /* 8-cycle: triangle-free as well */
    for (int k = 0; k < 8; k++) { cs[k] = k; cd[k] = (k + 1) % 8; }
    h = load(8, 8, cs, cd);
    CHECK(lfo_init_communities(h, 1) == 0, "init");
    ri = run(h, 3, 0, 1, hist);
    CHECK(ri.iterations == 0, "8-cycle: 0 iterations");
    lfo_destroy(h);
}

static uint64_t rng_state = 88172645463325252ull;
static uint64_t next_u64(void)       /* xorshift64 */
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return rng_state;
}

static void random_graphs(void)
{
    for (int trial = 0; trial < 12; trial++) {
        int n = 20 + (int)(next_u64() % 180);
        double p = 0.03 + (double)(next_u64() % 1000) / 1000.0 * 0.25;
        int64_t cap = (int64_t)n * n, m = 0;
        int64_t *s = malloc(sizeof(int64_t) * cap), *d = malloc(sizeof(int64_t) * cap);
        for (int a = 0; a < n; a++)
            for (int b = 0; b < n; b++)
                if (a != b && (double)(next_u64() % 1000000) / 1e6 < p / 2) { s[m] = a; d[m] = b; m++; }
        int q = 1 + (int)(next_u64() % 40);
        int64_t *off[2];
        int32_t *ids[2];
        int64_t tot[2];
        double hist[2][32];
        run_info ri[2];
        for (int v = 0; v < 2; v++) {
            lfo *h = load(n, m, s, d);
            CHECK(lfo_init_communities(h, v ? 4 : 1) == 0, "init");
            ri[v] = run(h, q, v ? 3 : 0, v ? 4 : 1, hist[v]);
            lfo_get_memberships(h, NULL, NULL, 0, &tot[v]);
            off[v] = malloc(sizeof(int64_t) * (n + 1));
            ids[v] = malloc(sizeof(int32_t) * (tot[v] + 1));
            lfo_get_memberships(h, off[v], ids[v], tot[v], &tot[v]);
            if (v == 1) {            /* the other entry points on the final cover */
                int32_t K = lfo_num_communities_created(h);
                double wcc = 0.0, f1 = 0.0;
                double *wc = malloc(sizeof(double) * (K + 1)), *wn = malloc(sizeof(double) * (tot[v] + 1));
                int32_t *t = malloc(sizeof(int32_t) * (tot[v] + 1)), *vo = malloc(sizeof(int32_t) * (tot[v] + 1));
                int32_t *vt = malloc(sizeof(int32_t) * (n + 1));
                CHECK(lfo_exact_wcc(h, 2, &wcc, wc, wn, t, vo, vt) == 0, "exact wcc: %s", lfo_last_error(h));
                uint8_t *keep = malloc((size_t)K + 1);
                int64_t removed[2] = {0, 0};
                CHECK(lfo_postprocess(h, 3u, keep, removed, 2) == 0, "postprocess: %s", lfo_last_error(h));
                double *ba = malloc(sizeof(double) * (K + 1));
                int32_t *bb = malloc(sizeof(int32_t) * (K + 1));
                CHECK(lfo_cover_f1(h, off[v], ids[v], tot[v], &f1, ba, bb) == 0, "f1: %s", lfo_last_error(h));
                CHECK(tot[v] == 0 || f1 == 1.0, "F1 of a cover with itself = 1 (%.17g)", f1);
                CHECK(lfo_init_from_memberships(h, off[v], ids[v], tot[v], K, 2) == 0, "warm: %s", lfo_last_error(h));
                double w1 = 0.0;
                lfo_get_scores(h, NULL, NULL, NULL, &w1);
                CHECK(w1 == ri[v].wtilde, "warm start reproduces the score");
                lfo_set_chunk_limit(h, 2);
                run_info pr;
                memset(&pr, 0, sizeof pr);
                CHECK(lfo_run_iterations(h, q, 0.0, 1, 3, 2, 0, &pr) == 0, "prefix run");
                CHECK(lfo_chunks_done(h) == ((n + q - 1) / q < 2 ? (n + q - 1) / q : 2), "prefix queues");
                lfo_set_chunk_limit(h, 0);
                free(wc); free(wn); free(t); free(vo); free(vt); free(keep); free(ba); free(bb);
            }
            lfo_destroy(h);
        }
        CHECK(ri[0].iterations == ri[1].iterations, "naive vs factored iterations");
        for (int k = 0; k <= ri[0].iterations && k < 32; k++)
            CHECK(hist[0][k] == hist[1][k], "naive vs factored score bits at %d", k);
        CHECK(tot[0] == tot[1], "naive vs factored membership count");
        if (tot[0] == tot[1]) {
            CHECK(memcmp(off[0], off[1], sizeof(int64_t) * (n + 1)) == 0, "offsets");
            CHECK(memcmp(ids[0], ids[1], sizeof(int32_t) * tot[0]) == 0, "community ids");
        }
        for (int v = 0; v < 2; v++) { free(off[v]); free(ids[v]); }
        free(s);
        free(d);
    }
}

int main(void)
{
    complete_graphs();
    path5();
    random_graphs();
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("sanitize ok\n");
    return 0;
}
