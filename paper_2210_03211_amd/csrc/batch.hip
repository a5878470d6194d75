// batch.hip -- many graphs advanced together, and the serving runtime built on it.
//
// A batch holds handles whose communities are initialised.  lf_batch_step runs one
// queue of every member that is still iterating: the per-queue parameters of all members
// go to the device in one copy, then each of the per-queue launches covers every
// member (blocks find their graph from per-member block offsets), so a launch carries
// the work of many small graphs instead of leaving most of the device idle.  A member's
// iteration start and end (path lists, degenerate removal, exact score, stop test) run
// between steps.  Every member computes exactly what lf_run_iterations computes for it
// alone: its kernels read and write only its own buffers, and the launch shapes do not
// change a result.
//
// The server admits submitted jobs (edge lists copied to host memory) into the batch in
// arrival order while their estimated device footprint fits the budget, steps the batch,
// and retires finished jobs (memberships copied back, device memory released), so jobs
// that arrive while others run join as memory frees up.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <stdlib.h>
#include <thread>
#include <vector>

#include "lf_internal.h"

struct BatchMember {
    lf_handle *h;
    hipStream_t saved_stream;
    long long qq, nq, k;     // queue size, queues of the current iteration, next queue
    int max_iters;
    double theta;
    int it;                  // iterations completed
    int phase;               // PH_*: where the member is between and within iterations
    hipEvent_t ev;           // recorded behind its queued iteration start or end
    hipEvent_t ran;          // recorded behind its last queue step (its end waits for it)
    int side;                // side stream of its iteration starts and ends
    int state;               // 0 iterating, 1 done, < 0 failed (status)
    bool begun;              // its start's host half is read; ev covers the device work it queued
    double prev;
    int converged, hit_max;
    Ctx cx;
    std::vector<double> hist;
    std::vector<long long> joins, leaves, comms;
};

#define BATCH_SIDES 2

struct lf_batch {
    int device;
    hipStream_t stream;
    bool own_stream;
    std::vector<BatchMember *> members;      // by member id; nullptr once removed
    std::vector<BatchMember *> live;         // members still iterating (any order)
    // Iteration starts and ends run on side streams, beside the steps: an end waits (on the
    // device) for its member's last step; a start follows an end the host has seen done.
    hipStream_t side[BATCH_SIDES];
    std::deque<BatchMember *> waitq[BATCH_SIDES];   // members whose queued start or end is
                                             // not yet read, in each side stream's order
    Member *hmem[2];
    int *hboff[2];
    hipEvent_t hev[2];
    Member *dmem;
    int *dboff;
    int cap;                                 // members the buffers hold
    int slot;
    bool use_graph;                          // replay the step from a captured graph
    hipGraph_t graph;
    hipGraphExec_t exec;
    hipGraphNode_t node[LF_MULTI_KERNELS];
    int graph_cap;                           // cap the graph was captured for
    long long graph_steps;
    long long steps, member_steps;           // steps that launched, queues they ran
    double wait_ms;                          // host time waiting for the device in steps
    double phase_ms, params_ms, launch_ms;   // host time: iteration starts and ends,
                                             // per-member parameters, upload and launch
    char err[512];
};

static int batch_error(lf_batch *b, int code, const char *msg)
{
    snprintf(b->err, sizeof b->err, "%s", msg);
    return code;
}

// Capture the multi-graph launches of a step once (grids and member counts are set
// per step on the executable graph; descriptors live at fixed device addresses).
static int batch_capture(lf_batch *b)
{
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
    }
    const void *fn[LF_MULTI_KERNELS];
    int grid[LF_MULTI_KERNELS], block[LF_MULTI_KERNELS];
    lf_multi_kernels(fn, grid, block);
    const int zero = 0;
    if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return batch_error(b, LF_EDEVICE, "stream capture failed to start");
    for (int i = 0; i < LF_MULTI_KERNELS; i++) {
        const int *o = b->dboff + grid[i] * (b->cap + 1);
        void *args[3] = {(void *)&b->dmem, (void *)&o, (void *)&zero};
        (void)hipLaunchKernel(fn[i], dim3(1), dim3(block[i]), args, 0, b->stream);
    }
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(b->stream, &g) != hipSuccess || !g)
        return batch_error(b, LF_EDEVICE, "stream capture failed");
    size_t nn = 0;
    (void)hipGraphGetNodes(g, nullptr, &nn);
    std::vector<hipGraphNode_t> nodes(nn);
    if (nn != LF_MULTI_KERNELS || hipGraphGetNodes(g, nodes.data(), &nn) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return batch_error(b, LF_EDEVICE, "unexpected captured graph");
    }
    for (int i = 0; i < LF_MULTI_KERNELS; i++) {   // match the nodes to the kernels
        b->node[i] = nullptr;
        for (size_t k = 0; k < nn; k++) {
            hipKernelNodeParams p;
            if (hipGraphKernelNodeGetParams(nodes[k], &p) == hipSuccess && p.func == fn[i]) b->node[i] = nodes[k];
        }
        if (!b->node[i]) {
            (void)hipGraphDestroy(g);
            return batch_error(b, LF_EDEVICE, "kernel node not found in the captured graph");
        }
    }
    if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        b->exec = nullptr;
        return batch_error(b, LF_EDEVICE, "graph instantiation failed");
    }
    b->graph = g;
    b->graph_cap = b->cap;
    return LF_OK;
}

// one step from the executable graph: grids and member count of every node, then replay
static int batch_replay(lf_batch *b, int nm, const int *total)
{
    if (!b->exec || b->graph_cap != b->cap) LF_TRY(batch_capture(b));
    const void *fn[LF_MULTI_KERNELS];
    int grid[LF_MULTI_KERNELS], block[LF_MULTI_KERNELS];
    lf_multi_kernels(fn, grid, block);
    for (int i = 0; i < LF_MULTI_KERNELS; i++) {
        const int t = grid[i];
        const int *o = b->dboff + t * (b->cap + 1);
        void *args[3] = {(void *)&b->dmem, (void *)&o, (void *)&nm};
        hipKernelNodeParams p;
        memset(&p, 0, sizeof p);
        p.func = (void *)fn[i];
        p.gridDim = dim3(total[t] > 0 ? total[t] : 1);   // blocks past the last member return at once
        p.blockDim = dim3(block[i]);
        p.sharedMemBytes = 0;
        p.kernelParams = args;
        p.extra = nullptr;
        if (hipGraphExecKernelNodeSetParams(b->exec, b->node[i], &p) != hipSuccess)
            return batch_error(b, LF_EDEVICE, "graph node update failed");
    }
    if (hipGraphLaunch(b->exec, b->stream) != hipSuccess) return batch_error(b, LF_EDEVICE, "graph launch failed");
    b->graph_steps++;
    return LF_OK;
}

static int batch_reserve(lf_batch *b, int nm)
{
    if (nm <= b->cap) return LF_OK;
    int cap = b->cap ? b->cap : 64;
    while (cap < nm) cap *= 2;
    for (int s = 0; s < 2; s++) {
        if (b->hmem[s]) {
            (void)hipEventSynchronize(b->hev[s]);
            (void)hipHostFree(b->hmem[s]);
            (void)hipHostFree(b->hboff[s]);
        }
        if (hipHostMalloc((void **)&b->hmem[s], sizeof(Member) * cap, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&b->hboff[s], sizeof(int) * LF_MULTI_GRIDS * (cap + 1), hipHostMallocDefault) !=
                hipSuccess)
            return batch_error(b, LF_ENOMEM, "pinned host buffers of the batch");
    }
    (void)hipStreamSynchronize(b->stream);
    if (b->dmem) (void)hipFree(b->dmem);
    if (b->dboff) (void)hipFree(b->dboff);
    if (hipMalloc((void **)&b->dmem, sizeof(Member) * cap) != hipSuccess ||
        hipMalloc((void **)&b->dboff, sizeof(int) * LF_MULTI_GRIDS * (cap + 1)) != hipSuccess)
        return batch_error(b, LF_ENOMEM, "device buffers of the batch");
    b->cap = cap;
    return LF_OK;
}

// A member's iteration start and end are queued on the batch stream like its queue
// kernels, with an event behind them; the host finishes them on a later step once the event
// has completed, so it never waits for the stream and the device never drains.  The member
// sits out the steps in between.
#define PH_BEGIN 0           // an iteration start is to be queued
#define PH_BEGIN_WAIT 1      // queued; waiting for its event
#define PH_RUN 2             // launching queues
#define PH_END_WAIT 3        // the iteration end is queued; waiting for its event

// record the result of a finished iteration (its end has completed on the device) and
// decide whether the member goes on
static int member_iteration_done(BatchMember *m)
{
    lf_handle *h = m->h;
    long long joins = 0, leaves = 0, live = 0;
    int rc = lf_iter_finish_complete(h, &joins, &leaves, &live);
    if (rc != LF_OK) return rc;
    m->it++;
    m->hist.push_back(h->Wt);
    m->joins.push_back(joins);
    m->leaves.push_back(leaves);
    m->comms.push_back(live);
    bool stop = (m->prev == 0.0) || ((h->Wt - m->prev) / m->prev < m->theta);
    m->prev = h->Wt;
    m->phase = PH_BEGIN;
    if (stop) {
        m->converged = 1;
        m->state = 1;
    } else if (m->it >= m->max_iters) {
        m->hit_max = 1;
        m->state = 1;
    }
    return LF_OK;
}

extern "C" {

int lf_batch_create(lf_batch **out, int device, void *hip_stream)
{
    if (!out) return LF_EINVAL;
    *out = nullptr;
    if (hipSetDevice(device) != hipSuccess) return LF_EDEVICE;
    lf_batch *b = new lf_batch();
    b->device = device;
    b->cap = 0;
    b->slot = 0;
    b->dmem = nullptr;
    b->dboff = nullptr;
    b->use_graph = true;
    b->graph = nullptr;
    b->exec = nullptr;
    b->graph_cap = 0;
    b->graph_steps = 0;
    b->steps = 0;
    b->member_steps = 0;
    b->wait_ms = 0.0;
    b->phase_ms = 0.0;
    b->params_ms = 0.0;
    b->launch_ms = 0.0;
    b->err[0] = 0;
    for (int s = 0; s < 2; s++) {
        b->hmem[s] = nullptr;
        b->hboff[s] = nullptr;
        b->hev[s] = nullptr;
    }
    bool ok = hipEventCreateWithFlags(&b->hev[0], hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&b->hev[1], hipEventDisableTiming) == hipSuccess;
    b->own_stream = false;
    for (int k = 0; k < BATCH_SIDES; k++) b->side[k] = nullptr;
    for (int k = 0; k < BATCH_SIDES && ok; k++)
        ok = hipStreamCreateWithFlags(&b->side[k], hipStreamNonBlocking) == hipSuccess;
    if (ok && hip_stream) {
        b->stream = (hipStream_t)hip_stream;
    } else if (ok) {
        ok = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) == hipSuccess;
        b->own_stream = ok;
    }
    if (!ok) {
        for (int s = 0; s < 2; s++)
            if (b->hev[s]) (void)hipEventDestroy(b->hev[s]);
        for (int k = 0; k < BATCH_SIDES; k++)
            if (b->side[k]) (void)hipStreamDestroy(b->side[k]);
        delete b;
        return LF_EDEVICE;
    }
    *out = b;
    return LF_OK;
}

const char *lf_batch_last_error(lf_batch *b) { return b ? b->err : "null batch"; }

int lf_batch_set_graph(lf_batch *b, int32_t on)
{
    if (!b) return LF_EINVAL;
    b->use_graph = on != 0;
    return LF_OK;
}

int lf_batch_add(lf_batch *b, lf_handle *h, int32_t queue_size, double threshold, int32_t max_iters,
                 int32_t *member_id)
{
    if (!b || !h || !member_id) return LF_EINVAL;
    if (queue_size < 1 || !(threshold >= 0.0) || max_iters < 0)
        return batch_error(b, LF_EINVAL, "queue_size >= 1, threshold >= 0 and max_iters >= 0 required");
    if (h->state < 2) return batch_error(b, LF_ESTATE, "lf_batch_add: communities not initialised");
    if (h->device != b->device) return batch_error(b, LF_EINVAL, "lf_batch_add: handle on another device");
    if (hipStreamSynchronize(h->stream) != hipSuccess) return batch_error(b, LF_EDEVICE, "stream sync failed");
    BatchMember *m = new BatchMember();
    if (hipEventCreateWithFlags(&m->ev, hipEventDisableTiming) != hipSuccess) {
        delete m;
        return batch_error(b, LF_EDEVICE, "event creation failed");
    }
    if (hipEventCreateWithFlags(&m->ran, hipEventDisableTiming) != hipSuccess) {
        (void)hipEventDestroy(m->ev);
        delete m;
        return batch_error(b, LF_EDEVICE, "event creation failed");
    }
    m->h = h;
    m->saved_stream = h->stream;
    h->stream = b->stream;
    h->phase_graphs = 1;          // iteration starts and ends replayed from graphs
    long long n = h->n;
    m->qq = queue_size < n ? queue_size : (n > 0 ? n : 1);
    m->nq = 0;
    m->k = 0;
    m->max_iters = max_iters;
    m->theta = threshold;
    m->it = 0;
    m->phase = PH_BEGIN;
    m->begun = false;
    m->state = (h->cc == 0.0 || max_iters == 0) ? 1 : 0;
    m->converged = h->cc == 0.0 ? 1 : 0;
    m->hit_max = 0;
    m->prev = h->Wt;
    m->hist.push_back(h->Wt);
    *member_id = (int32_t)b->members.size();
    m->side = *member_id % BATCH_SIDES;
    b->members.push_back(m);
    if (m->state == 0) b->live.push_back(m);
    return LF_OK;
}

// A member's queued start or end has completed: read its report and move it on.  The
// host halves run with the member's side stream current, so device work they queue (a
// grown buffer refilled) stays in order with its starts and ends; a start whose host
// half queued some is waited for once more (*requeue) before the member steps.
static int member_phase_done(lf_batch *b, BatchMember *m, bool *requeue)
{
    *requeue = false;
    lf_handle *h = m->h;
    hipStream_t sd = b->side[m->side];
    h->stream = sd;
    int rc = LF_OK;
    if (m->phase == PH_END_WAIT) {
        rc = member_iteration_done(m);          // PH_BEGIN, or done
    } else if (m->begun) {
        m->begun = false;
        m->phase = PH_RUN;
    } else {
        rc = lf_iter_begin_complete(h, m->qq, &m->nq);
        if (rc == LF_OK) {
            m->cx = lf_ctx(h);
            m->k = 0;
            if (h->second_half_work) {
                rc = hipEventRecord(m->ev, sd) == hipSuccess ? LF_OK : LF_EDEVICE;
                m->begun = true;
                *requeue = true;
            } else {
                m->phase = PH_RUN;
            }
        }
    }
    h->stream = b->stream;
    return rc;
}

static void drop_member(lf_batch *b, BatchMember *m)
{
    std::deque<BatchMember *> &q = b->waitq[m->side];
    auto w = std::find(q.begin(), q.end(), m);
    if (w != q.end()) q.erase(w);
    auto l = std::find(b->live.begin(), b->live.end(), m);
    if (l != b->live.end()) {
        *l = b->live.back();
        b->live.pop_back();
    }
}

int lf_batch_step(lf_batch *b, int32_t *running)
{
    if (!b) return LF_EINVAL;
    std::vector<BatchMember *> act;
    auto tp = std::chrono::steady_clock::now();
    // queued starts and ends that have completed, oldest first: a side stream runs them in
    // queue order, so its first one not done ends its scan
    for (int k = 0; k < BATCH_SIDES; k++) {
        std::deque<BatchMember *> &wq = b->waitq[k];
        while (!wq.empty()) {
            BatchMember *m = wq.front();
            hipError_t q = hipEventQuery(m->ev);
            if (q == hipErrorNotReady) break;
            wq.pop_front();
            bool requeue = false;
            int rc = q == hipSuccess ? member_phase_done(b, m, &requeue) : LF_EDEVICE;
            if (rc != LF_OK) m->state = rc;
            else if (requeue) wq.push_back(m);
        }
    }
    for (size_t i = 0; i < b->live.size();) {
        BatchMember *m = b->live[i];
        if (m->state != 0) {                  // done or failed: no longer stepped
            b->live[i] = b->live.back();
            b->live.pop_back();
            continue;
        }
        i++;
        if (m->phase == PH_BEGIN) {
            hipStream_t sd = b->side[m->side];
            m->h->stream = sd;
            int rc = lf_iter_begin_enqueue(m->h, m->qq);
            if (rc == LF_OK && hipEventRecord(m->ev, sd) != hipSuccess) rc = LF_EDEVICE;
            m->h->stream = b->stream;
            if (rc != LF_OK) {
                m->state = rc;
                continue;
            }
            m->phase = PH_BEGIN_WAIT;
            b->waitq[m->side].push_back(m);
        } else if (m->phase == PH_RUN) {
            act.push_back(m);
        }
    }
    b->phase_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tp).count();
    if (act.empty()) {
        // nothing to launch: wait for a queued start or end instead of spinning
        for (int k = 0; k < BATCH_SIDES; k++) {
            if (b->waitq[k].empty()) continue;
            auto t0 = std::chrono::steady_clock::now();
            if (hipEventSynchronize(b->waitq[k].front()->ev) != hipSuccess)
                return batch_error(b, LF_EDEVICE, "event sync failed");
            b->wait_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            break;
        }
    }
    const int nm = (int)act.size();
    if (nm > 0) {
        LF_TRY(batch_reserve(b, nm));
        const int s = b->slot;
        b->slot ^= 1;
        auto t0 = std::chrono::steady_clock::now();
        if (hipEventSynchronize(b->hev[s]) != hipSuccess) return batch_error(b, LF_EDEVICE, "event sync failed");
        b->wait_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        b->steps++;
        b->member_steps += nm;
        auto t1 = std::chrono::steady_clock::now();
        Member *hm = b->hmem[s];
        int *hb = b->hboff[s];
        int total[LF_MULTI_GRIDS] = {0, 0, 0, 0};
        for (int i = 0; i < nm; i++) {
            BatchMember *m = act[i];
            QGrids g;
            lf_queue_params(m->h, m->k, m->nq, m->qq, true, &hm[i].qs, &g);
            m->cx.qtag = m->h->qtag++;
            hm[i].cx = m->cx;
            const int blocks[LF_MULTI_GRIDS] = {g.big, g.fin, g.apply, g.refresh};
            for (int t = 0; t < LF_MULTI_GRIDS; t++) {
                hb[t * (b->cap + 1) + i] = total[t];
                total[t] += blocks[t];
            }
        }
        for (int t = 0; t < LF_MULTI_GRIDS; t++) hb[t * (b->cap + 1) + nm] = total[t];
        auto t2 = std::chrono::steady_clock::now();
        b->params_ms += std::chrono::duration<double, std::milli>(t2 - t1).count();
        if (hipMemcpyAsync(b->dmem, hm, sizeof(Member) * nm, hipMemcpyHostToDevice, b->stream) != hipSuccess ||
            hipMemcpyAsync(b->dboff, hb, sizeof(int) * LF_MULTI_GRIDS * (b->cap + 1), hipMemcpyHostToDevice, b->stream) !=
                hipSuccess ||
            hipEventRecord(b->hev[s], b->stream) != hipSuccess)
            return batch_error(b, LF_EDEVICE, "descriptor upload failed");
        if (b->use_graph) {
            LF_TRY(batch_replay(b, nm, total));
        } else if (lf_launch_multi(b->stream, b->dmem, b->dboff, b->cap, nm, total) != LF_OK) {
            return batch_error(b, LF_EDEVICE, "multi-graph launch failed");
        }
        auto t3 = std::chrono::steady_clock::now();
        b->launch_ms += std::chrono::duration<double, std::milli>(t3 - t2).count();
        for (BatchMember *m : act) {
            m->k++;
            if (m->k == m->nq) {
                // the end runs on the member's side stream once this step is done
                hipStream_t sd = b->side[m->side];
                int rc = LF_OK;
                if (hipEventRecord(m->ran, b->stream) != hipSuccess || hipStreamWaitEvent(sd, m->ran, 0) != hipSuccess)
                    rc = LF_EDEVICE;
                m->h->stream = sd;
                if (rc == LF_OK) rc = lf_iter_finish_enqueue(m->h);
                if (rc == LF_OK && hipEventRecord(m->ev, sd) != hipSuccess) rc = LF_EDEVICE;
                m->h->stream = b->stream;
                if (rc != LF_OK) {
                    m->state = rc;
                } else {
                    m->phase = PH_END_WAIT;
                    b->waitq[m->side].push_back(m);
                }
            }
        }
        b->phase_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t3).count();
    }
    int live = 0;
    for (BatchMember *m : b->live)
        if (m->state == 0) live++;
    if (running) *running = live;
    return LF_OK;
}

// LF_OK and the results when the member is done; LF_EAGAIN while it still iterates; the
// member's error status if it failed.  The arrays of `out` are sized as for
// lf_run_iterations (any may be NULL).
int lf_batch_member_info(lf_batch *b, int32_t member_id, lf_run_info *out)
{
    if (!b || member_id < 0 || member_id >= (int32_t)b->members.size() || !b->members[member_id])
        return LF_EINVAL;
    BatchMember *m = b->members[member_id];
    if (m->state == 0) return LF_EAGAIN;
    if (m->state < 0) return m->state;
    if (out) {
        lf_handle *h = m->h;
        out->iterations = m->it;
        out->converged = m->converged;
        out->hit_max = m->hit_max;
        out->wtilde = h->Wt;
        out->wcc_hat = h->cc != 0.0 ? h->Wt / h->cc : 0.0;
        for (int i = 0; i <= m->it; i++)
            if (out->wtilde_hist) out->wtilde_hist[i] = m->hist[i];
        for (int i = 0; i < m->it; i++) {
            if (out->joins) out->joins[i] = m->joins[i];
            if (out->leaves) out->leaves[i] = m->leaves[i];
            if (out->communities) out->communities[i] = m->comms[i];
        }
    }
    return LF_OK;
}

// Take a member out of the batch (done or not); its handle goes back to its own stream.
int lf_batch_remove(lf_batch *b, int32_t member_id)
{
    if (!b || member_id < 0 || member_id >= (int32_t)b->members.size() || !b->members[member_id])
        return LF_EINVAL;
    BatchMember *m = b->members[member_id];
    drop_member(b, m);
    // mid-iteration the memberships live in the handle's lines: back to its slot layout
    if (m->state == 0 && m->phase == PH_RUN) (void)lf_lines_back(m->h);
    (void)hipStreamSynchronize(b->stream);
    for (int k = 0; k < BATCH_SIDES; k++) (void)hipStreamSynchronize(b->side[k]);
    m->h->stream = m->saved_stream;
    m->h->phase_graphs = 0;
    lf_phase_graphs_drop(m->h);
    (void)hipEventDestroy(m->ev);
    (void)hipEventDestroy(m->ran);
    delete m;
    b->members[member_id] = nullptr;
    return LF_OK;
}

// Take a finished member out of the batch without waiting: *left is recorded behind its
// last work on the batch stream and its side stream, and the caller waits for it before
// using the handle (which is back on its own stream) and destroys it afterwards.
int lf_batch_detach(lf_batch *b, int32_t member_id, hipEvent_t *left)
{
    *left = nullptr;
    if (!b || member_id < 0 || member_id >= (int32_t)b->members.size() || !b->members[member_id])
        return LF_EINVAL;
    BatchMember *m = b->members[member_id];
    drop_member(b, m);
    if (m->state == 0 && m->phase == PH_RUN) (void)lf_lines_back(m->h);
    hipStream_t sd = b->side[m->side];
    int rc = hipEventRecord(m->ran, b->stream) == hipSuccess && hipStreamWaitEvent(sd, m->ran, 0) == hipSuccess &&
                     hipEventRecord(m->ev, sd) == hipSuccess
                 ? LF_OK
                 : LF_EDEVICE;
    (void)hipEventDestroy(m->ran);          // released once the wait on it has passed
    *left = m->ev;
    m->h->stream = m->saved_stream;
    m->h->phase_graphs = 0;         // its graphs go with the handle, after the wait
    delete m;
    b->members[member_id] = nullptr;
    return rc;
}

int lf_batch_destroy(lf_batch *b)
{
    if (!b) return LF_OK;
    (void)hipSetDevice(b->device);
    (void)hipStreamSynchronize(b->stream);
    for (size_t i = 0; i < b->members.size(); i++)
        if (b->members[i]) lf_batch_remove(b, (int32_t)i);
    for (int s = 0; s < 2; s++) {
        if (b->hmem[s]) (void)hipHostFree(b->hmem[s]);
        if (b->hboff[s]) (void)hipHostFree(b->hboff[s]);
        (void)hipEventDestroy(b->hev[s]);
    }
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->dmem) (void)hipFree(b->dmem);
    if (b->dboff) (void)hipFree(b->dboff);
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    for (int k = 0; k < BATCH_SIDES; k++) (void)hipStreamDestroy(b->side[k]);
    delete b;
    return LF_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------------------
// serving runtime
// ------------------------------------------------------------------------------------
// The thread that ticks the server only steps the batch and moves jobs in and out of it.
// Worker threads, each with a stream of its own, load and initialise admitted jobs and
// retire finished ones (memberships copied back, device state released to the allocation
// cache), so neither waits in the stepping thread.
#define SERVER_WORKERS 4

struct Job {
    long long id;
    int state;               // 0 queued, 1 running, 2 done, < 0 failed (status)
    long long n;
    std::vector<int64_t> src, dst;
    int q;
    double theta;
    int max_iters;
    size_t footprint;
    lf_handle *h;
    int member;              // batch member id while in the batch, else -1
    int rc;                  // status of the worker's step (load or retirement)
    hipEvent_t left;         // recorded behind the job's last work in the batch
    std::vector<int64_t> off;
    std::vector<int32_t> ids;
    lf_run_info info;
    std::vector<double> hist;
    std::vector<long long> joins, leaves, comms;
};

struct lf_server {
    int device;
    hipStream_t stream;      // the batch's work
    bool own_stream;
    lf_batch *batch;
    size_t budget, used;
    int max_batch, running;
    std::deque<Job *> queue;          // submitted, not yet admitted (arrival order)
    std::deque<long long> done;       // finished or failed, not yet taken
    std::map<long long, Job *> jobs;
    std::vector<Job *> active;        // jobs in the batch
    long long next_id;
    double ms[5];            // admission and retirement (worker time), batch steps, hand-over, ticks
    char err[512];
    // workers
    std::vector<std::thread> workers;
    std::vector<hipStream_t> wstream;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Job *> to_load, to_retire;     // work for the workers
    std::deque<Job *> loaded, retired;        // their results, taken by the next tick
    bool stop;
    double wms[2];                            // worker time: loading, retiring
    long long phase_runs[3];                  // retired jobs' iteration starts and ends:
                                              // plain, captured, replayed
};

static double ms_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// Device bytes a job may hold at most: graph build scratch, CSR, node arrays, membership
// slots, community records and member lists (grown faster in a batch), and the per-queue
// work lists; blocks are rounded up to their allocation class (at most one eighth more).
static size_t job_footprint(long long n, long long npairs, int q)
{
    long long nn = n > 0 ? n : 1;
    long long qq = q < nn ? q : nn;
    size_t b = (size_t)(48ll << 20) + (size_t)nn * 768 + (size_t)npairs * 64 + (size_t)qq * 256;
    return b + b / 8;
}

static int server_error(lf_server *s, int code, const char *msg)
{
    snprintf(s->err, sizeof s->err, "%s", msg);
    return code;
}

// worker: load the graph and the initial clustering of a job on the worker's stream
static int job_load(lf_server *s, Job *j, hipStream_t st)
{
    int rc = lf_create(&j->h, s->device, (void *)st, 0);
    if (rc == LF_OK) rc = lf_load_graph(j->h, j->n, (int64_t)j->src.size(), j->src.data(), j->dst.data(), 0);
    if (rc == LF_OK) rc = lf_init_communities(j->h);
    if (rc == LF_OK && hipStreamSynchronize(st) != hipSuccess) rc = LF_EDEVICE;
    std::vector<int64_t>().swap(j->src);
    std::vector<int64_t>().swap(j->dst);
    return rc;
}

// worker: once the job's work in the batch has completed, copy its memberships to host
// memory and release its device state
static int job_collect(Job *j)
{
    int rc = LF_OK;
    if (j->left) {
        if (hipEventSynchronize(j->left) != hipSuccess) rc = LF_EDEVICE;
        (void)hipEventDestroy(j->left);
        j->left = nullptr;
    }
    int64_t total = 0;
    if (rc == LF_OK) rc = lf_get_memberships(j->h, nullptr, nullptr, 0, &total);
    if (rc == LF_OK) {
        j->off.resize(j->n + 1);
        j->ids.resize(total > 0 ? total : 1);
        rc = lf_get_memberships(j->h, j->off.data(), j->ids.data(), (int64_t)j->ids.size(), &total);
        j->ids.resize(total);
    }
    lf_destroy(j->h);
    j->h = nullptr;
    return rc;
}

static void worker_main(lf_server *s, int w)
{
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        s->cv.wait(lk, [&] { return s->stop || !s->to_load.empty() || !s->to_retire.empty(); });
        if (s->stop) return;
        const bool retire = !s->to_retire.empty();   // retiring frees memory: first
        Job *j = retire ? s->to_retire.front() : s->to_load.front();
        if (retire) s->to_retire.pop_front();
        else s->to_load.pop_front();
        lk.unlock();
        auto t0 = std::chrono::steady_clock::now();
        j->rc = retire ? job_collect(j) : job_load(s, j, s->wstream[w]);
        const double ms = ms_since(t0);
        lk.lock();
        s->wms[retire ? 1 : 0] += ms;
        (retire ? s->retired : s->loaded).push_back(j);
    }
}

// the job has left the server's device memory (done or failed)
static void job_gone(lf_server *s, Job *j)
{
    s->used -= j->footprint;
    s->running--;
    s->done.push_back(j->id);
}

extern "C" {

int lf_server_create(lf_server **out, int device, void *hip_stream, uint64_t hbm_budget, int32_t max_batch)
{
    if (!out || max_batch < 1 || hbm_budget == 0) return LF_EINVAL;
    *out = nullptr;
    if (hipSetDevice(device) != hipSuccess) return LF_EDEVICE;
    lf_server *s = new lf_server();
    s->device = device;
    s->budget = hbm_budget;
    s->used = 0;
    s->max_batch = max_batch;
    s->running = 0;
    s->next_id = 0;
    s->err[0] = 0;
    s->stop = false;
    for (int k = 0; k < 5; k++) s->ms[k] = 0.0;
    s->wms[0] = s->wms[1] = 0.0;
    for (int k = 0; k < 3; k++) s->phase_runs[k] = 0;
    bool ok = true;
    for (int w = 0; w < SERVER_WORKERS && ok; w++) {
        hipStream_t st = nullptr;
        ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
        if (ok) s->wstream.push_back(st);
    }
    if (ok && hip_stream) {
        s->stream = (hipStream_t)hip_stream;
        s->own_stream = false;
    } else if (ok) {
        ok = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) == hipSuccess;
        s->own_stream = ok;
    }
    int rc = ok ? lf_batch_create(&s->batch, device, (void *)s->stream) : LF_EDEVICE;
    if (rc != LF_OK) {
        if (ok && s->own_stream) (void)hipStreamDestroy(s->stream);
        for (hipStream_t st : s->wstream) (void)hipStreamDestroy(st);
        delete s;
        return rc;
    }
    for (int w = 0; w < SERVER_WORKERS; w++) s->workers.emplace_back(worker_main, s, w);
    *out = s;
    return LF_OK;
}

const char *lf_server_last_error(lf_server *s) { return s ? s->err : "null server"; }

int lf_server_submit(lf_server *s, int64_t n, int64_t n_pairs, const int64_t *src, const int64_t *dst,
                     int32_t queue_size, double threshold, int32_t max_iters, int64_t *job_id)
{
    if (!s || !job_id || n < 0 || n_pairs < 0 || (n_pairs > 0 && (!src || !dst)) || queue_size < 1 ||
        !(threshold >= 0.0) || max_iters < 0)
        return LF_EINVAL;
    size_t fp = job_footprint(n, n_pairs, queue_size);
    if (fp > s->budget) return server_error(s, LF_ENOMEM, "job footprint exceeds the whole device budget");
    Job *j = new Job();
    j->id = s->next_id++;
    j->state = 0;
    j->n = n;
    j->src.assign(src, src + n_pairs);
    j->dst.assign(dst, dst + n_pairs);
    j->q = queue_size;
    j->theta = threshold;
    j->max_iters = max_iters;
    j->footprint = fp;
    j->h = nullptr;
    j->member = -1;
    j->rc = LF_OK;
    j->left = nullptr;
    s->queue.push_back(j);
    s->jobs[j->id] = j;
    *job_id = j->id;
    return LF_OK;
}

// Take the workers' results (loaded jobs join the batch, retired jobs are done), admit
// queued jobs that fit, run one step of the batch, hand finished jobs to the workers.
// *pending = jobs queued or running afterwards.
int lf_server_tick(lf_server *s, int32_t *pending)
{
    if (!s) return LF_EINVAL;
    auto t_tick = std::chrono::steady_clock::now();
    std::deque<Job *> loaded, retired;
    {
        std::lock_guard<std::mutex> g(s->mu);
        loaded.swap(s->loaded);
        retired.swap(s->retired);
        s->ms[0] = s->wms[0];
        s->ms[2] = s->wms[1];
    }
    for (Job *j : retired) {
        j->state = j->rc == LF_OK ? 2 : j->rc;
        job_gone(s, j);
    }
    bool more = false;
    for (Job *j : loaded) {
        int rc = j->rc;
        if (rc == LF_OK) rc = lf_batch_add(s->batch, j->h, j->q, j->theta, j->max_iters, &j->member);
        if (rc == LF_OK) {
            s->active.push_back(j);
            continue;
        }
        j->state = rc;
        if (j->h) lf_destroy(j->h);
        j->h = nullptr;
        j->member = -1;
        job_gone(s, j);
    }
    // admission in arrival order while the job fits the budget (its memory is reserved
    // from now until its retirement has completed)
    while (!s->queue.empty() && s->running < s->max_batch) {
        Job *j = s->queue.front();
        if (s->used + j->footprint > s->budget) break;
        s->queue.pop_front();
        s->used += j->footprint;
        s->running++;
        j->state = 1;
        std::lock_guard<std::mutex> g(s->mu);
        s->to_load.push_back(j);
        more = true;
    }
    if (more) s->cv.notify_all();
    s->ms[3] += ms_since(t_tick);
    auto t0 = std::chrono::steady_clock::now();
    int32_t live = 0;
    LF_TRY(lf_batch_step(s->batch, &live));
    s->ms[1] += ms_since(t0);
    t0 = std::chrono::steady_clock::now();
    more = false;
    for (size_t k = 0; k < s->active.size();) {
        Job *j = s->active[k];
        int rc = lf_batch_member_info(s->batch, j->member, nullptr);
        if (rc == LF_EAGAIN) {
            k++;
            continue;
        }
        j->hist.assign(j->max_iters + 1, 0.0);
        j->joins.assign(j->max_iters > 0 ? j->max_iters : 1, 0);
        j->leaves.assign(j->joins.size(), 0);
        j->comms.assign(j->joins.size(), 0);
        memset(&j->info, 0, sizeof j->info);
        j->info.wtilde_hist = j->hist.data();
        j->info.joins = (int64_t *)j->joins.data();
        j->info.leaves = (int64_t *)j->leaves.data();
        j->info.communities = (int64_t *)j->comms.data();
        if (rc == LF_OK) rc = lf_batch_member_info(s->batch, j->member, &j->info);
        for (int k = 0; k < 3; k++) s->phase_runs[k] += j->h->phase_runs[k];
        int drc = lf_batch_detach(s->batch, j->member, &j->left);
        j->member = -1;
        s->active[k] = s->active.back();
        s->active.pop_back();
        if (rc != LF_OK || drc != LF_OK) {        // failed in the batch: release at once
            (void)hipStreamSynchronize(s->stream);
            if (j->left) (void)hipEventDestroy(j->left);
            j->left = nullptr;
            lf_destroy(j->h);
            j->h = nullptr;
            j->state = rc != LF_OK ? rc : drc;
            job_gone(s, j);
            continue;
        }
        std::lock_guard<std::mutex> g(s->mu);
        s->to_retire.push_back(j);
        more = true;
    }
    if (more) s->cv.notify_all();
    s->ms[3] += ms_since(t0);
    if (pending) *pending = (int32_t)s->queue.size() + s->running;
    s->ms[4] += ms_since(t_tick);
    return LF_OK;
}

int lf_server_set_graph(lf_server *s, int32_t on)
{
    if (!s) return LF_EINVAL;
    return lf_batch_set_graph(s->batch, on);
}

// host milliseconds: admission and retirement (summed over the worker threads), batch
// steps, handing jobs to and from the workers, whole ticks; the part of the steps spent
// waiting for the device; steps that launched and the queues they ran; host time of the
// steps in iteration starts and ends, per-member parameters, upload and launch; the
// iteration starts and ends of retired jobs run plainly, captured and replayed (counts)
int lf_server_timing(lf_server *s, double *ms)
{
    if (!s || !ms) return LF_EINVAL;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->ms[0] = s->wms[0];
        s->ms[2] = s->wms[1];
    }
    for (int k = 0; k < 5; k++) ms[k] = s->ms[k];
    ms[5] = s->batch->wait_ms;
    ms[6] = (double)s->batch->steps;
    ms[7] = (double)s->batch->member_steps;
    ms[8] = s->batch->phase_ms;
    ms[9] = s->batch->params_ms;
    ms[10] = s->batch->launch_ms;
    for (int k = 0; k < 3; k++) ms[11 + k] = (double)s->phase_runs[k];
    return LF_OK;
}

// 0 queued, 1 running, 2 done (results waiting), < 0 failed with that status
// ids of jobs that finished (or failed) since the last call, in completion order, at
// most capacity of them; *count = how many were written
int lf_server_take_done(lf_server *s, int64_t *ids, int32_t capacity, int32_t *count)
{
    if (!s || !count || capacity < 0 || (capacity > 0 && !ids)) return LF_EINVAL;
    int32_t k = 0;
    while (k < capacity && !s->done.empty()) {
        ids[k++] = s->done.front();
        s->done.pop_front();
    }
    *count = k;
    return LF_OK;
}

int lf_server_poll(lf_server *s, int64_t job_id, int32_t *state)
{
    if (!s || !state) return LF_EINVAL;
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return LF_EINVAL;
    *state = it->second->state;
    return LF_OK;
}

// Results of a done job, in the two-call pattern of lf_get_memberships; info as from
// lf_run_iterations (its arrays sized max_iters + 1 / max_iters, any may be NULL).  The job
// is forgotten once its memberships have been copied out.
int lf_server_fetch(lf_server *s, int64_t job_id, int64_t *offsets, int32_t *comm_ids, int64_t capacity,
                    int64_t *total, lf_run_info *info)
{
    if (!s || !total) return LF_EINVAL;
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return LF_EINVAL;
    Job *j = it->second;
    if (j->state < 0) return j->state;
    if (j->state != 2) return LF_EAGAIN;
    *total = (int64_t)j->ids.size();
    if (info) {
        info->iterations = j->info.iterations;
        info->converged = j->info.converged;
        info->hit_max = j->info.hit_max;
        info->wcc_hat = j->info.wcc_hat;
        info->wtilde = j->info.wtilde;
        for (int i = 0; i <= j->info.iterations; i++)
            if (info->wtilde_hist) info->wtilde_hist[i] = j->hist[i];
        for (int i = 0; i < j->info.iterations; i++) {
            if (info->joins) info->joins[i] = j->joins[i];
            if (info->leaves) info->leaves[i] = j->leaves[i];
            if (info->communities) info->communities[i] = j->comms[i];
        }
    }
    if (!offsets && !comm_ids) return LF_OK;
    if (!offsets || !comm_ids || capacity < *total) return server_error(s, LF_ERANGE, "buffers too small");
    memcpy(offsets, j->off.data(), sizeof(int64_t) * (j->n + 1));
    if (*total > 0) memcpy(comm_ids, j->ids.data(), sizeof(int32_t) * *total);
    delete j;
    s->jobs.erase(it);
    return LF_OK;
}

int lf_server_stats(lf_server *s, uint64_t *used, uint64_t *budget, int32_t *running, int32_t *queued)
{
    if (!s) return LF_EINVAL;
    if (used) *used = s->used;
    if (budget) *budget = s->budget;
    if (running) *running = s->running;
    if (queued) *queued = (int32_t)s->queue.size();
    return LF_OK;
}

int lf_server_destroy(lf_server *s)
{
    if (!s) return LF_OK;
    (void)hipSetDevice(s->device);
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;                      // workers finish the job in hand and leave
    }
    s->cv.notify_all();
    for (std::thread &t : s->workers) t.join();
    (void)hipStreamSynchronize(s->stream);
    for (auto &kv : s->jobs) {
        Job *j = kv.second;
        if (j->member >= 0) lf_batch_remove(s->batch, j->member);
        if (j->left) (void)hipEventDestroy(j->left);
        if (j->h) lf_destroy(j->h);
        delete j;
    }
    lf_batch_destroy(s->batch);
    if (s->own_stream) (void)hipStreamDestroy(s->stream);
    for (hipStream_t st : s->wstream) (void)hipStreamDestroy(st);
    delete s;
    return LF_OK;
}

int lf_get_memory(lf_handle *h, uint64_t *bytes, uint64_t *peak)
{
    if (!h) return LF_EINVAL;
    if (bytes) *bytes = h->dev_bytes;
    if (peak) *peak = h->dev_bytes_peak;
    return LF_OK;
}

}  // extern "C"
