// Batch executor: many independent operator calls of different plans,
// issued concurrently on a few streams, optionally recorded into one HIP
// graph and replayed with a single launch.  In fused mode the tasks run in
// phases: their FFT passes on the streams, then one interpolation launch per
// phase and kernel shape for all tasks (staged gathers of all forward-type
// tasks of one dimension and window width, of all omega-Jacobian tasks, and
// output-stationary spreads of all adjoint-type tasks with one owner-tile
// shape), then each task's epilogue on its stream.
#include <algorithm>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "kbn_internal.h"
#include "kbnufft.h"

namespace {

// Tasks interpolated by one launch, and that launch's device job list.
struct FuseGroup {
    int kind = 0;  // 0, 1: gather modes; 2: spread
    int D = 0, J = 0;
    KbnSpreadSel sel;
    int To[KBN_MAX_D] = {0, 0, 0};
    std::vector<int> members;  // task indices
    kbn_plan mem = nullptr;    // plan whose allocator holds the job list
    char *dev = nullptr;       // jobs, then the int64 (gather) or int (spread) start offsets
    int64_t total = 0;         // gather workgroups / spread rows
    size_t lds = 0;
    int maxngr = 0;
    hipEvent_t done = nullptr;
};

}  // namespace

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
    // fused mode
    bool fuse = false;
    bool prepared = false;
    std::vector<uint64_t> epochs;  // per plan, when the phases were prepared
    std::vector<KbnPhased> ph;     // per task
    std::vector<hipEvent_t> pre_done;  // per task: its FFT passes are issued
    std::vector<FuseGroup> groups;
    hipStream_t gstream = nullptr, sstream = nullptr;  // gather and spread launches
    hipEvent_t gjoin = nullptr, sjoin = nullptr;
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

int issue_fused(kbn_batch b, hipStream_t from);

// Fork the batch's streams off `from`, issue every stream's tasks, join.
int issue(kbn_batch b, hipStream_t from) {
    if (b->fuse) return issue_fused(b, from);
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

// Free the phases' workspaces and job lists once the batch's work is done.
void release_phases(kbn_batch b) {
    if (!b->prepared && b->ph.empty()) return;
    for (auto st : b->streams) (void)hipStreamSynchronize(st);
    if (b->gstream) (void)hipStreamSynchronize(b->gstream);
    if (b->sstream) (void)hipStreamSynchronize(b->sstream);
    for (auto &ph : b->ph) kbn_internal_phase_release(&ph, nullptr);
    for (auto &g : b->groups) {
        if (g.dev) kbn_internal_free(g.mem, g.dev, nullptr);
        if (g.done) (void)hipEventDestroy(g.done);
    }
    for (auto e : b->pre_done)
        if (e) (void)hipEventDestroy(e);
    b->ph.clear();
    b->groups.clear();
    b->pre_done.clear();
    b->prepared = false;
}

bool same_group(const FuseGroup &g, const KbnPhased &ph) {
    const KbnGeom &x = ph.kind == 2 ? ph.sj.g : ph.gj.g;
    if (g.kind != ph.kind || g.D != x.D || g.J != x.J) return false;
    if (ph.kind != 2) return true;
    if (g.sel.cpt != ph.sel.cpt || g.sel.ebv != ph.sel.ebv || g.sel.tcells != ph.sel.tcells) return false;
    for (int d = 0; d < x.D; ++d)
        if (g.To[d] != x.To[d]) return false;
    return true;
}

// Split every task into phases, group the interpolations by launch shape and
// upload each group's job list (waits for `s`).
int prepare_phases(kbn_batch b, hipStream_t s) {
    release_phases(b);
    const int n = (int)b->tasks.size();
    b->ph.assign(n, KbnPhased());
    b->pre_done.assign(n, nullptr);
    int rc = KBN_OK;
    for (int i = 0; i < n && rc == KBN_OK; ++i) rc = kbn_internal_phase_prepare(b->tasks[i], &b->ph[i], s);
    if (rc != KBN_OK) {
        b->prepared = true;  // so that release_phases frees what was allocated
        release_phases(b);
        return rc;
    }
    for (int i = 0; i < n; ++i) {
        const KbnPhased &ph = b->ph[i];
        if (ph.kind < 0) continue;
        size_t k = 0;
        while (k < b->groups.size() && !same_group(b->groups[k], ph)) ++k;
        if (k == b->groups.size()) {
            FuseGroup g;
            const KbnGeom &x = ph.kind == 2 ? ph.sj.g : ph.gj.g;
            g.kind = ph.kind;
            g.D = x.D;
            g.J = x.J;
            g.sel = ph.sel;
            for (int d = 0; d < KBN_MAX_D; ++d) g.To[d] = x.To[d];
            g.mem = ph.p;
            b->groups.push_back(g);
        }
        b->groups[k].members.push_back(i);
        if (ph.kind <= 1 && hipEventCreateWithFlags(&b->pre_done[i], hipEventDisableTiming) != hipSuccess)
            rc = kbn_internal_fail(KBN_ERR_HIP, "hipEventCreate");
    }
    std::vector<char> host;
    for (auto &g : b->groups) {
        if (rc != KBN_OK) break;
        const int nm = (int)g.members.size();
        host.clear();
        if (g.kind <= 1) {
            std::vector<KbnGatherJob> jobs(nm);
            std::vector<int64_t> start(nm + 1, 0);
            for (int k = 0; k < nm; ++k) {
                const KbnPhased &ph = b->ph[g.members[k]];
                jobs[k] = ph.gj;
                start[k + 1] = start[k] + (int64_t)ph.gj.blocks * ph.groups;
                g.lds = std::max(g.lds, ph.lds);
            }
            g.total = start[nm];
            host.resize(sizeof(KbnGatherJob) * nm + sizeof(int64_t) * (nm + 1));
            std::memcpy(host.data(), jobs.data(), sizeof(KbnGatherJob) * nm);
            std::memcpy(host.data() + sizeof(KbnGatherJob) * nm, start.data(), sizeof(int64_t) * (nm + 1));
        } else {
            std::vector<KbnSpreadJob> jobs(nm);
            int64_t rows = 0;
            for (int k = 0; k < nm; ++k) {
                jobs[k] = b->ph[g.members[k]].sj;
                rows += jobs[k].ny;
                g.maxngr = std::max(g.maxngr, jobs[k].ngr);
            }
            // the launch's rows fit the grid limit: each job strides over its
            // work items with its share of them
            if (rows > KBN_GRID_Y_MAX)
                for (auto &j : jobs) j.ny = std::max<int64_t>(1, (int64_t)j.ny * KBN_GRID_Y_MAX / rows - 1);
            std::vector<int> start(nm + 1, 0);
            for (int k = 0; k < nm; ++k) start[k + 1] = start[k] + jobs[k].ny;
            g.total = start[nm];
            g.lds = g.sel.lds;
            host.resize(sizeof(KbnSpreadJob) * nm + sizeof(int) * (nm + 1));
            std::memcpy(host.data(), jobs.data(), sizeof(KbnSpreadJob) * nm);
            std::memcpy(host.data() + sizeof(KbnSpreadJob) * nm, start.data(), sizeof(int) * (nm + 1));
        }
        rc = kbn_internal_alloc(g.mem, (void **)&g.dev, (int64_t)host.size(), s);
        if (rc == KBN_OK && (hipMemcpyAsync(g.dev, host.data(), host.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
                             hipStreamSynchronize(s) != hipSuccess))
            rc = kbn_internal_fail(KBN_ERR_HIP, "job list upload");
        if (rc == KBN_OK && hipEventCreateWithFlags(&g.done, hipEventDisableTiming) != hipSuccess)
            rc = kbn_internal_fail(KBN_ERR_HIP, "hipEventCreate");
    }
    b->prepared = true;
    if (rc != KBN_OK) {
        release_phases(b);
        return rc;
    }
    b->epochs.resize(b->plans.size());
    for (size_t i = 0; i < b->plans.size(); ++i) b->epochs[i] = kbn_internal_epoch(b->plans[i]);
    return KBN_OK;
}

bool phases_stale(kbn_batch b) {
    if (!b->prepared) return true;
    for (size_t i = 0; i < b->plans.size(); ++i)
        if (b->epochs[i] != kbn_internal_epoch(b->plans[i])) return true;
    return false;
}

int launch_group(const FuseGroup &g, hipStream_t s) {
    const int nm = (int)g.members.size();
    hipError_t e;
    if (g.kind <= 1) {
        const KbnGatherJob *jobs = (const KbnGatherJob *)g.dev;
        const int64_t *start = (const int64_t *)(g.dev + sizeof(KbnGatherJob) * nm);
        e = kbn_launch_gather_multi(g.D, g.J, g.kind, jobs, start, nm, g.total, g.lds, s);
    } else {
        const KbnSpreadJob *jobs = (const KbnSpreadJob *)g.dev;
        const int *start = (const int *)(g.dev + sizeof(KbnSpreadJob) * nm);
        e = kbn_launch_spread_os_multi(g.sel, g.D, g.J, g.maxngr, jobs, start, nm, (int)g.total, s);
    }
    if (e != hipSuccess) return kbn_internal_fail(KBN_ERR_HIP, hipGetErrorString(e));
    return KBN_OK;
}

// Fused issue: FFT passes (and whole tasks) on the streams, the spreads on
// their own stream from the start, each gather group once its tasks' passes
// are issued, then the epilogues on the tasks' streams.
int issue_fused(kbn_batch b, hipStream_t from) {
    if (phases_stale(b)) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(from, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
            return kbn_internal_fail(KBN_ERR_UNSUPPORTED, "fused batch phases changed during capture");
        const int rc = prepare_phases(b, from);
        if (rc != KBN_OK) return rc;
    }
    KBN_BHIP(hipEventRecord(b->fork, from), "hipEventRecord (fork)");
    int rc = KBN_OK;
    const size_t ns = b->per_stream.size();
    for (size_t i = 0; i < ns; ++i) {
        hipStream_t s = b->streams[i];
        KBN_BHIP(hipStreamWaitEvent(s, b->fork, 0), "hipStreamWaitEvent (fork)");
        for (int ti : b->per_stream[i]) {
            if (rc != KBN_OK) break;
            KbnPhased &ph = b->ph[ti];
            if (ph.kind < 0) {
                rc = run_task(b->tasks[ti], s);
            } else if (ph.kind <= 1) {
                rc = kbn_internal_phase_pre(&ph, s);
                if (rc == KBN_OK && hipEventRecord(b->pre_done[ti], s) != hipSuccess)
                    rc = kbn_internal_fail(KBN_ERR_HIP, "hipEventRecord");
            }
        }
    }
    KBN_BHIP(hipStreamWaitEvent(b->sstream, b->fork, 0), "hipStreamWaitEvent (fork)");
    KBN_BHIP(hipStreamWaitEvent(b->gstream, b->fork, 0), "hipStreamWaitEvent (fork)");
    for (auto &g : b->groups) {
        if (rc != KBN_OK) break;
        hipStream_t s = g.kind == 2 ? b->sstream : b->gstream;
        if (g.kind <= 1)
            for (int ti : g.members) KBN_BHIP(hipStreamWaitEvent(s, b->pre_done[ti], 0), "hipStreamWaitEvent");
        for (int ti : g.members) {
            if (rc == KBN_OK) rc = kbn_internal_points_wait(b->tasks[ti].plan, s);
        }
        if (rc != KBN_OK) break;
        rc = launch_group(g, s);
        if (rc == KBN_OK && hipEventRecord(g.done, s) != hipSuccess)
            rc = kbn_internal_fail(KBN_ERR_HIP, "hipEventRecord");
    }
    for (size_t i = 0; i < ns; ++i) {
        hipStream_t s = b->streams[i];
        for (int ti : b->per_stream[i]) {
            if (rc != KBN_OK) break;
            KbnPhased &ph = b->ph[ti];
            if (ph.kind < 1) continue;
            for (auto &g : b->groups)
                if (std::find(g.members.begin(), g.members.end(), ti) != g.members.end())
                    KBN_BHIP(hipStreamWaitEvent(s, g.done, 0), "hipStreamWaitEvent");
            rc = kbn_internal_phase_post(&ph, s);
        }
        // join even after a failure so that `from` still orders after
        // whatever was issued
        KBN_BHIP(hipEventRecord(b->joins[i], s), "hipEventRecord (join)");
        KBN_BHIP(hipStreamWaitEvent(from, b->joins[i], 0), "hipStreamWaitEvent (join)");
    }
    KBN_BHIP(hipEventRecord(b->gjoin, b->gstream), "hipEventRecord (join)");
    KBN_BHIP(hipStreamWaitEvent(from, b->gjoin, 0), "hipStreamWaitEvent (join)");
    KBN_BHIP(hipEventRecord(b->sjoin, b->sstream), "hipEventRecord (join)");
    KBN_BHIP(hipStreamWaitEvent(from, b->sjoin, 0), "hipStreamWaitEvent (join)");
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
    release_phases(b);
    if (b->gstream) (void)hipStreamDestroy(b->gstream);
    if (b->sstream) (void)hipStreamDestroy(b->sstream);
    if (b->gjoin) (void)hipEventDestroy(b->gjoin);
    if (b->sjoin) (void)hipEventDestroy(b->sjoin);
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
    if (nstreams == 0) nstreams = 8;  // 8 measured 6% faster than 4 on the 33-instance bundle
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
    // the captured fused issue ended the process in the HIP graph runtime
    // (host segmentation fault, cause not found): fused batches run eagerly
    if (b->fuse) return kbn_internal_fail(KBN_ERR_UNSUPPORTED, "a fused batch cannot be captured");
    for (kbn_plan p : b->plans)
        if (kbn_internal_timing_on(p))
            return kbn_internal_fail(KBN_ERR_INVALID_ARG, "a plan of the batch has timing enabled");
    release_graph(b);
    hipStream_t s = (hipStream_t)stream;
    // one eager pass sizes every workspace, so the capture allocates nothing
    int rc = issue(b, s);
    if (rc != KBN_OK) return rc;
    KBN_BHIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    // the eager pass waited for every plan's index pass: note it, so that the
    // captured calls need not wait on events from outside the capture
    for (kbn_plan p : b->plans) kbn_internal_points_settle(p);
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

int kbn_batch_fuse(kbn_batch b, int on) {
    if (!b) return kbn_internal_fail(KBN_ERR_INVALID_ARG, "null batch");
    if (b->exec) return kbn_internal_fail(KBN_ERR_INVALID_ARG, "batch has been captured");
    if (on && !b->gstream) {
        if (hipStreamCreateWithFlags(&b->gstream, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&b->sstream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&b->gjoin, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&b->sjoin, hipEventDisableTiming) != hipSuccess)
            return kbn_internal_fail(KBN_ERR_HIP, "stream/event creation");
    }
    if (!on) release_phases(b);
    b->fuse = on != 0;
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
