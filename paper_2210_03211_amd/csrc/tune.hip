// tune.hip -- autotuner of the launch shapes and evaluation-path thresholds.
//
// Results never depend on these options, so the tuner times candidates on the real work:
// from the handle's initial clustering it runs a few iterations per candidate (the same
// deterministic work each time), timed with HIP events on the handle's stream, and keeps
// the fastest.  The search is coordinate descent: one option at a time, over a short list
// of values, the others held at the best so far.  The choice is remembered for the
// graph's class -- the shape of its degree histogram (log2 buckets) and the size of its
// queues -- so further graphs of the class take it without trials.
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "lf_internal.h"

#define NBUCKET 24

__global__ void k_degree_buckets(const int *deg, long long n, unsigned long long *bucket)
{
    __shared__ unsigned long long s[NBUCKET];
    if (threadIdx.x < NBUCKET) s[threadIdx.x] = 0;
    __syncthreads();
    for (long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x; x < n; x += (long long)gridDim.x * blockDim.x) {
        int d = deg[x];
        int b = d <= 0 ? 0 : 32 - __clz(d);
        if (b >= NBUCKET) b = NBUCKET - 1;
        atomicAdd(&s[b], 1ull);
    }
    __syncthreads();
    if (threadIdx.x < NBUCKET && s[threadIdx.x]) atomicAdd(&bucket[threadIdx.x], s[threadIdx.x]);
}

namespace {

struct TuneChoice {
    int64_t v[5];
};

std::mutex g_tune_mu;
std::map<std::string, TuneChoice> g_tune_cache;

const int kOpts[5] = {LF_OPT_WAVE_TABLE, LF_OPT_MED_TABLE, LF_OPT_GRP_TABLE, LF_OPT_HUB_BLOCKS,
                      LF_OPT_REFRESH_BLOCKS};

// class of a graph: log2 degree histogram in steps of 1/16 of the nodes, and log2 of the
// queue size and of the node count
int graph_class(lf_handle *h, int q, std::string *key)
{
    unsigned long long *d = nullptr;
    LF_TRY(lf_tmp_alloc(h, (void **)&d, sizeof(unsigned long long) * NBUCKET));
    LF_HIP(h, hipMemsetAsync(d, 0, sizeof(unsigned long long) * NBUCKET, h->stream));
    if (h->n > 0) hipLaunchKernelGGL(k_degree_buckets, dim3(256), dim3(256), 0, h->stream, h->deg, h->n, d);
    unsigned long long b[NBUCKET];
    LF_HIP(h, hipMemcpyAsync(b, d, sizeof(b), hipMemcpyDeviceToHost, h->stream));
    LF_HIP(h, hipStreamSynchronize(h->stream));
    char buf[256];
    int len = 0;
    long long n = h->n > 0 ? h->n : 1;
    for (int k = 0; k < NBUCKET; k++)
        len += snprintf(buf + len, sizeof buf - len, "%d,", (int)((b[k] * 16 + n / 2) / n));
    int lq = 0, ln = 0;
    while ((1ll << (lq + 1)) <= q) lq++;
    while ((1ll << (ln + 1)) <= n) ln++;
    snprintf(buf + len, sizeof buf - len, "q%d,n%d", lq, ln);
    *key = buf;
    return LF_OK;
}

int set_all(lf_handle *h, const TuneChoice &c)
{
    for (int k = 0; k < 5; k++) LF_TRY(lf_set_option(h, kOpts[k], c.v[k]));
    return LF_OK;
}

// GPU milliseconds of `iters` iterations from the initial clustering with choice c
int trial(lf_handle *h, const TuneChoice &c, int q, int iters, float *ms)
{
    LF_TRY(set_all(h, c));
    LF_TRY(lf_init_communities(h));
    lf_run_info info;
    memset(&info, 0, sizeof info);
    LF_HIP(h, hipEventRecord(h->ev0, h->stream));
    LF_TRY(lf_iterate(h, q, 0.0, iters, &info));
    LF_HIP(h, hipEventRecord(h->ev1, h->stream));
    LF_HIP(h, hipEventSynchronize(h->ev1));
    LF_HIP(h, hipEventElapsedTime(ms, h->ev0, h->ev1));
    return LF_OK;
}

}  // namespace

extern "C" {

int lf_autotune(lf_handle *h, int32_t queue_size, int32_t trial_iters, lf_tune_result *out)
{
    if (!h || !out || queue_size < 1 || trial_iters < 1) return LF_EINVAL;
    if (h->state < 2) return lf_set_error(h, LF_ESTATE, "lf_autotune: communities not initialised");
    TmpScope tmp_scope(h);
    std::string key;
    LF_TRY(graph_class(h, queue_size, &key));
    memset(out, 0, sizeof *out);
    TuneChoice best;
    for (int k = 0; k < 5; k++) LF_TRY(lf_get_option(h, kOpts[k], &best.v[k]));
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            LF_TRY(set_all(h, it->second));
            for (int k = 0; k < 5; k++) out->value[k] = it->second.v[k];
            out->from_cache = 1;
            return LF_OK;
        }
    }
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device);
    const std::vector<int64_t> cand[5] = {
        {32, 64, 128},                           // wave-path table: where the medium path starts
        {128, 256, 512},                         // medium-path table: where the workgroup path starts
        {512, 1024, 2048},                       // workgroup-path table: where the table path starts
        {(int64_t)cus, 2 * (int64_t)cus, 4 * (int64_t)cus},   // workgroups of the table and workgroup roles
        {(int64_t)cus / 2, (int64_t)cus, 2 * (int64_t)cus, 4 * (int64_t)cus},   // in-count and re-sum kernels
    };
    float best_ms = 0.f;
    LF_TRY(trial(h, best, queue_size, trial_iters, &best_ms));
    out->default_ms = best_ms;
    int trials = 1;
    for (int k = 0; k < 5; k++) {
        for (int64_t v : cand[k]) {
            if (v == best.v[k]) continue;
            TuneChoice c = best;
            c.v[k] = v;
            float ms = 0.f;
            LF_TRY(trial(h, c, queue_size, trial_iters, &ms));
            trials++;
            if (ms < best_ms) {
                best_ms = ms;
                best = c;
            }
        }
    }
    LF_TRY(set_all(h, best));
    LF_TRY(lf_init_communities(h));              // back to the initial clustering
    for (int k = 0; k < 5; k++) out->value[k] = best.v[k];
    out->best_ms = best_ms;
    out->trials = trials;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = best;
    return LF_OK;
}

int lf_autotune_forget(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache.clear();
    return LF_OK;
}

}  // extern "C"
