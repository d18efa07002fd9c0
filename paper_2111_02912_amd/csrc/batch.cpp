// Batch executor: many independent operator calls of different plans,
// issued concurrently on a few streams, optionally recorded into one HIP
// graph and replayed with a single launch.
#include <algorithm>
#include <new>
#include <numeric>
#include <vector>

#include "kbn_internal.h"
#include "kbnufft.h"

struct kbn_batch_s {
    std::vector<kbn_task> tasks;
    std::vector<std::vector<int>> per_stream;  // task indices in issue order
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> joins;
    hipEvent_t fork = nullptr;
    hipStream_t origin = nullptr;  // capture origin (never the caller's stream)
    std::vector<kbn_plan> plans;   // distinct plans, first-use order
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

#define KBN_BHIP(expr, what)                                                        \
    do {                                                                            \
        hipError_t e_ = (expr);                                                     \
        if (e_ != hipSuccess)                                                       \
            return kbn_internal_fail(KBN_ERR_HIP, what);                            \
    } while (0)

int run_task(const kbn_task &t, hipStream_t s) {
    switch (t.op) {
    case KBN_TASK_FORWARD:
        return kbn_forward(t.plan, t.B, t.C, t.a, t.smaps, t.out, s);
    case KBN_TASK_ADJOINT:
        return kbn_adjoint(t.plan, t.B, t.C, t.a, t.smaps, t.out, s);
    case KBN_TASK_JAC_OMEGA_FWD:
        return kbn_jac_omega_fwd(t.plan, t.B, t.C, t.a, t.smaps, t.g, (float *)t.out, t.accumulate, s);
    case KBN_TASK_JAC_OMEGA_ADJ:
        return kbn_jac_omega_adj(t.plan, t.B, t.C, t.a, t.smaps, t.g, (float *)t.out, t.accumulate, s);
    case KBN_TASK_JAC_X_FWD:
        return kbn_jac_x(t.plan, KBN_OP_FORWARD, t.B, t.C, t.a, t.smaps, t.out, s);
    case KBN_TASK_JAC_X_ADJ:
        return kbn_jac_x(t.plan, KBN_OP_ADJOINT, t.B, t.C, t.a, t.smaps, t.out, s);
    default:
        return kbn_internal_fail(KBN_ERR_INVALID_ARG, "unknown task op");
    }
}

double task_cost(const kbn_task &t) {
    switch (t.op) {
    case KBN_TASK_FORWARD:
    case KBN_TASK_JAC_X_ADJ:
        return kbn_internal_cost(t.plan, t.B, t.C, 0, 0);
    case KBN_TASK_JAC_OMEGA_FWD:
    case KBN_TASK_JAC_OMEGA_ADJ:
        return kbn_internal_cost(t.plan, t.B, t.C, 1, 0);
    default:
        return kbn_internal_cost(t.plan, t.B, t.C, 0, 1);
    }
}

// Fork the batch's streams off `from`, issue every stream's tasks, join.
int issue(kbn_batch b, hipStream_t from) {
    KBN_BHIP(hipEventRecord(b->fork, from), "hipEventRecord (fork)");
    int rc = KBN_OK;
    for (size_t i = 0; i < b->per_stream.size(); ++i) {
        hipStream_t s = b->streams[i];
        KBN_BHIP(hipStreamWaitEvent(s, b->fork, 0), "hipStreamWaitEvent (fork)");
        for (int ti : b->per_stream[i]) {
            if (rc != KBN_OK) break;
            rc = run_task(b->tasks[ti], s);
        }
        // join even after a failure so that `from` still orders after
        // whatever was issued
        KBN_BHIP(hipEventRecord(b->joins[i], s), "hipEventRecord (join)");
        KBN_BHIP(hipStreamWaitEvent(from, b->joins[i], 0), "hipStreamWaitEvent (join)");
    }
    return rc;
}

void release_graph(kbn_batch b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->exec)
        for (kbn_plan p : b->plans) kbn_internal_graph_ref(p, -1);
    b->exec = nullptr;
    b->graph = nullptr;
}

void free_batch(kbn_batch b) {
    release_graph(b);
    for (auto s : b->streams) (void)hipStreamDestroy(s);
    for (auto e : b->joins) (void)hipEventDestroy(e);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->origin) (void)hipStreamDestroy(b->origin);
    delete b;
}

}  // namespace

extern "C" {

int kbn_batch_create(kbn_batch *out, int ntasks, const kbn_task *tasks, int nstreams) {
    if (!out) return kbn_internal_fail(KBN_ERR_INVALID_ARG, "null output pointer");
    *out = nullptr;
    if (ntasks < 1 || !tasks) return kbn_internal_fail(KBN_ERR_INVALID_ARG, "empty task list");
    if (nstreams == 0) nstreams = 4;
    if (nstreams < 1 || nstreams > 16) return kbn_internal_fail(KBN_ERR_INVALID_ARG, "nstreams must be 0..16");
    for (int i = 0; i < ntasks; ++i) {
        if (!tasks[i].plan) return kbn_internal_fail(KBN_ERR_INVALID_ARG, "task with a null plan");
        if (tasks[i].op < KBN_TASK_FORWARD || tasks[i].op > KBN_TASK_JAC_X_ADJ)
            return kbn_internal_fail(KBN_ERR_INVALID_ARG, "unknown task op");
    }
    kbn_batch b = new (std::nothrow) kbn_batch_s();
    if (!b) return kbn_internal_fail(KBN_ERR_OOM, "host allocation failed");
    b->tasks.assign(tasks, tasks + ntasks);

    // chains: the tasks of one plan, in list order
    std::vector<std::vector<int>> chains;
    std::vector<double> cost;
    for (int i = 0; i < ntasks; ++i) {
        kbn_plan p = tasks[i].plan;
        size_t c = std::find(b->plans.begin(), b->plans.end(), p) - b->plans.begin();
        if (c == b->plans.size()) {
            b->plans.push_back(p);
            chains.emplace_back();
            cost.push_back(0.0);
        }
        chains[c].push_back(i);
        cost[c] += task_cost(tasks[i]);
    }
    // largest chains first, each onto the least loaded stream
    const int ns = std::min<int>(nstreams, (int)chains.size());
    std::vector<int> idx(chains.size());
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    std::vector<double> load(ns, 0.0);
    b->per_stream.resize(ns);
    for (int c : idx) {
        int s = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[s] += cost[c];
        b->per_stream[s].insert(b->per_stream[s].end(), chains[c].begin(), chains[c].end());
    }
    b->streams.assign(ns, nullptr);
    b->joins.assign(ns, nullptr);
    int rc = KBN_OK;
    for (int i = 0; i < ns && rc == KBN_OK; ++i) {
        if (hipStreamCreateWithFlags(&b->streams[i], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&b->joins[i], hipEventDisableTiming) != hipSuccess)
            rc = kbn_internal_fail(KBN_ERR_HIP, "stream/event creation");
    }
    if (rc == KBN_OK && (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
                         hipStreamCreateWithFlags(&b->origin, hipStreamNonBlocking) != hipSuccess))
        rc = kbn_internal_fail(KBN_ERR_HIP, "stream/event creation");
    if (rc != KBN_OK) {
        free_batch(b);
        return rc;
    }
    *out = b;
    return KBN_OK;
}

int kbn_batch_run(kbn_batch b, void *stream) {
    if (!b) return kbn_internal_fail(KBN_ERR_INVALID_ARG, "null batch");
    return issue(b, (hipStream_t)stream);
}

int kbn_batch_capture(kbn_batch b, void *stream) {
    if (!b) return kbn_internal_fail(KBN_ERR_INVALID_ARG, "null batch");
    for (kbn_plan p : b->plans)
        if (kbn_internal_timing_on(p))
            return kbn_internal_fail(KBN_ERR_INVALID_ARG, "a plan of the batch has timing enabled");
    release_graph(b);
    hipStream_t s = (hipStream_t)stream;
    // one eager pass sizes every workspace, so the capture allocates nothing
    int rc = issue(b, s);
    if (rc != KBN_OK) return rc;
    KBN_BHIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    KBN_BHIP(hipStreamBeginCapture(b->origin, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    rc = issue(b, b->origin);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->origin, &g);
    if (rc != KBN_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess || !g) return kbn_internal_fail(KBN_ERR_HIP, "hipStreamEndCapture");
    hipGraphExec_t x = nullptr;
    if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return kbn_internal_fail(KBN_ERR_HIP, "hipGraphInstantiate");
    }
    b->graph = g;
    b->exec = x;
    for (kbn_plan p : b->plans) kbn_internal_graph_ref(p, +1);
    return KBN_OK;
}

int kbn_batch_launch(kbn_batch b, void *stream) {
    if (!b) return kbn_internal_fail(KBN_ERR_INVALID_ARG, "null batch");
    if (!b->exec) return kbn_internal_fail(KBN_ERR_INVALID_ARG, "batch has not been captured");
    KBN_BHIP(hipGraphLaunch(b->exec, (hipStream_t)stream), "hipGraphLaunch");
    return KBN_OK;
}

int kbn_batch_destroy(kbn_batch b) {
    if (!b) return kbn_internal_fail(KBN_ERR_INVALID_ARG, "null batch");
    (void)hipDeviceSynchronize();
    free_batch(b);
    return KBN_OK;
}

}  // extern "C"
