// Continuous-batching query server over the graphs of a context.
//
// A query asks for Algorithm 1 (PercIS) on one resident graph with its own
// (eps, delta, seed). Queries wait in arrival order until their hit buffer
// (4 bytes per node) fits in the server's memory pool, one device block of
// the budget's size allocated when the server is created and sub-allocated
// per query (first fit); admitted queries run their two sampling phases in
// chunks. A launch carries the first phase of every query that is in it and
// then second phases in arrival order, filled up to the step's sample
// budget, so queries of different graphs and sizes share the device and a
// query that arrives while others run joins the next launch.
//
// Two launches are in flight on the context's stream: while the device runs
// one, the host reads the statistics of the one before, and the per-query
// work between phases (the bounds of Algorithm 1, the estimates) runs on a
// second stream, so the device does not wait for the host. A query's
// samples are indices of its own (seed, phase) stream, so its result is the
// same alone or in any mix, and equals percis_graph_estimate for the same
// arguments.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <unordered_map>
#include <vector>

#include "percis.h"
#include "percis_host.h"
#include "percis_internal.h"

using namespace percis;

namespace {

enum QState { QUEUED = 0, PHASE1 = 1, PHASE2 = 2, DONE = 3, FAILED = 4 };

struct Query {
    int64_t id = 0;
    int32_t graph = 0;
    double eps = 0, delta = 0;
    uint64_t seed = 0;
    QState state = QUEUED;
    int status = PERCIS_OK;
    uint32_t* d_hits = nullptr;    // in the server's pool
    int64_t off = -1;              // offset of d_hits in the pool
    int64_t bytes = 0;
    uint64_t planned = 0;          // samples of the current phase handed to launches
    uint64_t done = 0;             // samples of the current phase finished
    uint64_t target = 0;           // samples of the current phase
    uint64_t sum_I = 0, sum_I2 = 0, overflow = 0;
    percis_estimate_info info{};
    std::vector<double> p;
    std::chrono::steady_clock::time_point t_submit, t_admit;
};

constexpr int kMaxLaunchTasks = 4096;  // query chunks one launch carries at most
constexpr int kInFlight = 2;           // launches on the device at a time

// First-fit allocator over the pool: free ranges by offset.
struct Pool {
    int64_t size = 0;
    std::map<int64_t, int64_t> free_;   // offset -> length

    void reset(int64_t n) {
        size = n;
        free_.clear();
        free_[0] = n;
    }
    int64_t alloc(int64_t n) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const int64_t at = it->first, len = it->second;
            free_.erase(it);
            if (len > n) free_[at + n] = len - n;
            return at;
        }
        return -1;
    }
    void release(int64_t at, int64_t n) {
        auto it = free_.emplace(at, n).first;
        auto next = std::next(it);
        if (next != free_.end() && at + n == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == at) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Flight {
    AsyncLaunch launch;
    std::vector<Query*> owners;
    bool busy = false;
};

}  // namespace

struct percis_server {
    percis_ctx* ctx = nullptr;
    int64_t budget = 0;
    int64_t in_use = 0;
    uint64_t chunk = 0;
    uint64_t step_samples = 0;
    int64_t next_id = 1;
    void* pool_mem = nullptr;
    Pool pool;
    hipStream_t post = nullptr;                     // per-query work between phases
    Flight flights[kInFlight];
    int head = 0;                                   // oldest launch in flight
    int inflight = 0;
    std::deque<Query*> queued;
    std::vector<Query*> active;                     // admission order
    std::unordered_map<int64_t, Query*> by_id;
    uint64_t samples_done = 0;
    double kernel_ms = 0;
    int64_t peak_in_use = 0;
};

namespace {

void release(percis_server* s, Query* q) {
    if (q->off >= 0) {
        s->pool.release(q->off, q->bytes);
        q->off = -1;
        q->d_hits = nullptr;
        s->in_use -= q->bytes;
    }
}

// Admits queued queries in arrival order while their buffers fit the pool.
void admit(percis_server* s) {
    while (!s->queued.empty()) {
        Query* q = s->queued.front();
        if (q->bytes > s->budget) {
            q->state = FAILED;
            q->status = PERCIS_E_NOMEM;
            s->queued.pop_front();
            continue;
        }
        const int64_t at = s->pool.alloc(q->bytes);
        if (at < 0) break;
        q->off = at;
        q->d_hits = (uint32_t*)((char*)s->pool_mem + at);
        s->in_use += q->bytes;
        s->peak_in_use = std::max(s->peak_in_use, s->in_use);
        q->state = PHASE1;
        q->info.l1 = (uint64_t)std::ceil(std::max(1000.0, std::log(1.0 / q->delta) / q->eps));
        q->target = q->info.l1;
        q->planned = q->done = 0;
        q->t_admit = std::chrono::steady_clock::now();
        s->queued.pop_front();
        s->active.push_back(q);
    }
}

// Plans one launch of at most step_samples samples: first phase 1 of every
// admitted query in it (short, and it decides the size of phase 2), at most
// `chunk` samples each, then phase 2 in arrival order, each query taking
// what it still needs from what the launch has left. A query is then never
// slowed by queries that arrived after it, beyond their phase 1.
void plan(percis_server* s, std::vector<TaskSpec>& tasks, std::vector<Query*>& owners) {
    uint64_t left = s->step_samples;
    for (int ph = 1; ph <= 2 && left > 0; ph++) {
        for (Query* q : s->active) {
            if (left == 0 || (int)tasks.size() >= kMaxLaunchTasks) break;
            if ((int)q->state != ph || q->planned >= q->target) continue;
            uint64_t take = std::min<uint64_t>(q->target - q->planned, left);
            if (ph == 1) take = std::min<uint64_t>(take, s->chunk);
            tasks.push_back(TaskSpec{q->graph, (uint32_t)ph, q->planned, take, q->seed, q->d_hits, q->planned > 0});
            owners.push_back(q);
            q->planned += take;
            left -= take;
        }
    }
}

// Plans and enqueues launches until kInFlight are on the device or there is
// nothing to hand out.
int fill(percis_server* s) {
    percis_ctx* c = s->ctx;
    while (s->inflight < kInFlight) {
        Flight& f = s->flights[(s->head + s->inflight) % kInFlight];
        std::vector<TaskSpec> tasks;
        f.owners.clear();
        plan(s, tasks, f.owners);
        if (tasks.empty()) break;
        const int rc = launch_tasks_async(c, tasks, &f.launch);
        if (rc) return rc;
        f.busy = true;
        s->inflight++;
    }
    return PERCIS_OK;
}

// A query whose current phase has finished: the bounds of Algorithm 1 after
// phase 1 (phase 2 then starts at the next launch), the estimate after
// phase 2. Device work on the server's second stream, after `after` (the
// launch that finished the phase). Returns 1 if the query is done (or failed).
int finish_phase(percis_server* s, Query* q, hipEvent_t after, int* rc_out) {
    percis_ctx* c = s->ctx;
    *rc_out = PERCIS_OK;
    GraphData& G = *get_graph(c, q->graph);
    if (q->overflow) {
        q->state = FAILED;
        q->status = PERCIS_E_SIGMA_OVERFLOW;
        q->info.overflow = q->overflow;
        return 1;
    }
    if (hipStreamWaitEvent(s->post, after, 0) != hipSuccess) {
        *rc_out = fail(c, PERCIS_E_DEVICE, "cannot order the server's streams");
        return 0;
    }
    if (q->state == PHASE1) {
        if ((*rc_out = phase1_bounds(c, G, q->info.l1, q->sum_I, q->sum_I2, q->d_hits, q->eps, q->delta, &q->info,
                                     s->post)))
            return 0;
        if (q->info.l >= 4294967295ull) {
            q->state = FAILED;
            q->status = PERCIS_E_TOO_LARGE;
            return 1;
        }
        q->state = PHASE2;
        q->target = q->info.l;
        q->planned = q->done = 0;
        return 0;
    }
    q->p.resize(G.n);
    if ((*rc_out = estimates_to_host(c, G, q->d_hits, q->info.l, q->p.data(), s->post))) return 0;
    q->state = DONE;
    q->info.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - q->t_submit).count();
    return 1;
}

}  // namespace

extern "C" {

int percis_server_create(percis_ctx* ctx, int64_t memory_budget_bytes, uint64_t chunk_samples, uint64_t step_samples,
                         percis_server** out) {
    if (!ctx || !out || memory_budget_bytes <= 0 || chunk_samples == 0 || step_samples == 0) return PERCIS_E_INVAL;
    if (ctx->host_only) return fail(ctx, PERCIS_E_STATE, "host-only context cannot serve");
    int rc = set_device(ctx);
    if (rc) return rc;
    percis_server* s = new (std::nothrow) percis_server();
    if (!s) return PERCIS_E_NOMEM;
    s->ctx = ctx;
    s->budget = memory_budget_bytes / 256 * 256;
    s->chunk = chunk_samples;
    s->step_samples = std::max(step_samples, chunk_samples);
    if (hipMalloc(&s->pool_mem, (size_t)std::max<int64_t>(s->budget, 256)) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return fail(ctx, PERCIS_E_NOMEM, "cannot allocate the %lld-byte query pool", (long long)memory_budget_bytes);
    }
    s->pool.reset(s->budget);
    rc = hipStreamCreateWithFlags(&s->post, hipStreamNonBlocking) == hipSuccess ? PERCIS_OK
         : fail(ctx, PERCIS_E_DEVICE, "cannot create the server's stream");
    for (int i = 0; i < kInFlight && rc == PERCIS_OK; i++) rc = async_launch_init(ctx, &s->flights[i].launch, kMaxLaunchTasks);
    if (rc) {
        percis_server_destroy(s);
        return rc;
    }
    *out = s;
    return PERCIS_OK;
}

void percis_server_destroy(percis_server* s) {
    if (!s) return;
    if (s->ctx && !s->ctx->host_only) {
        (void)hipSetDevice(s->ctx->device);
        if (s->ctx->stream) (void)hipStreamSynchronize(s->ctx->stream); else (void)hipDeviceSynchronize();
        if (s->post) (void)hipStreamSynchronize(s->post);
    }
    for (auto& kv : s->by_id) delete kv.second;
    for (Flight& f : s->flights) async_launch_free(&f.launch);
    if (s->post) (void)hipStreamDestroy(s->post);
    if (s->pool_mem) (void)hipFree(s->pool_mem);
    delete s;
}

int percis_server_submit(percis_server* s, int32_t graph, double eps, double delta, uint64_t seed, int64_t* query_id) {
    if (!s || !query_id) return PERCIS_E_INVAL;
    percis_ctx* c = s->ctx;
    GraphData* G = get_graph(c, graph);
    if (!G || !G->has_graph || !G->has_states) return fail(c, PERCIS_E_INVAL, "no graph %d with states", graph);
    if (!(eps > 0 && eps < 1) || !(delta > 0 && delta < 1)) return fail(c, PERCIS_E_INVAL, "need 0 < eps, delta < 1");
    int rc = graph_upload(c, *G, true);
    if (rc) return rc;
    int64_t D = 0;
    if ((rc = vertex_diam_ub(c, *G, &D))) return rc;
    Query* q = new (std::nothrow) Query();
    if (!q) return fail(c, PERCIS_E_NOMEM, "out of host memory");
    q->info.D = D;
    q->id = s->next_id++;
    q->graph = graph;
    q->eps = eps;
    q->delta = delta;
    q->seed = seed;
    q->bytes = ((int64_t)G->n * 4 + 255) / 256 * 256;
    q->t_submit = std::chrono::steady_clock::now();
    s->queued.push_back(q);
    s->by_id[q->id] = q;
    *query_id = q->id;
    return PERCIS_OK;
}

int percis_server_step(percis_server* s, int32_t* completed) {
    if (!s) return PERCIS_E_INVAL;
    percis_ctx* c = s->ctx;
    if (completed) *completed = 0;
    int rc = set_device(c);
    if (rc) return rc;
    admit(s);
    if ((rc = fill(s))) return rc;
    if (s->inflight == 0) return PERCIS_OK;

    // the oldest launch: its statistics, then the queries whose phase it ended
    Flight& f = s->flights[s->head];
    std::vector<percis_stats> ts;
    percis_stats launch{};
    rc = finish_tasks_async(c, &f.launch, &ts, &launch);
    s->head = (s->head + 1) % kInFlight;
    s->inflight--;
    f.busy = false;
    if (rc != PERCIS_OK && rc != PERCIS_E_SIGMA_OVERFLOW) return rc;
    s->samples_done += launch.samples;
    s->kernel_ms += launch.kernel_ms;
    int32_t done = 0;
    for (size_t i = 0; i < f.owners.size(); i++) {
        Query* q = f.owners[i];
        q->done += f.launch.tasks[i].count;
        q->sum_I += ts[i].sum_I;
        q->sum_I2 += ts[i].sum_I2;
        q->overflow += ts[i].overflow;
    }
    for (size_t i = 0; i < f.owners.size(); i++) {
        Query* q = f.owners[i];
        if (q->done < q->target || q->planned > q->done || q->state == DONE || q->state == FAILED) continue;
        int err = PERCIS_OK;
        done += finish_phase(s, q, f.launch.done, &err);
        if (err) return err;
    }
    // retire finished queries; their pool space admits the next ones
    std::vector<Query*> still;
    for (Query* q : s->active) {
        if (q->state == DONE || q->state == FAILED) release(s, q);
        else still.push_back(q);
    }
    s->active.swap(still);
    admit(s);
    if ((rc = fill(s))) return rc;
    if (completed) *completed = done;
    return PERCIS_OK;
}

int percis_server_result(percis_server* s, int64_t query_id, int32_t* done, double* p_out, int32_t n_cap,
                         percis_estimate_info* info) {
    if (!s || !done) return PERCIS_E_INVAL;
    auto it = s->by_id.find(query_id);
    if (it == s->by_id.end()) return fail(s->ctx, PERCIS_E_INVAL, "unknown query %lld", (long long)query_id);
    Query* q = it->second;
    *done = (q->state == DONE || q->state == FAILED) ? 1 : 0;
    if (!*done) return PERCIS_OK;
    const int status = q->status;
    if (q->state == DONE) {
        if (p_out) {
            if (n_cap < (int32_t)q->p.size()) return fail(s->ctx, PERCIS_E_INVAL, "output holds %d of %zu values", n_cap, q->p.size());
            std::memcpy(p_out, q->p.data(), sizeof(double) * q->p.size());
        }
    }
    if (info) *info = q->info;
    release(s, q);
    delete q;
    s->by_id.erase(it);
    return status;
}

int percis_server_status(percis_server* s, int32_t* queued, int32_t* active, int64_t* bytes_in_use,
                         int64_t* peak_bytes, uint64_t* samples_done) {
    if (!s) return PERCIS_E_INVAL;
    if (queued) *queued = (int32_t)s->queued.size();
    if (active) *active = (int32_t)s->active.size();
    if (bytes_in_use) *bytes_in_use = s->in_use;
    if (peak_bytes) *peak_bytes = s->peak_in_use;
    if (samples_done) *samples_done = s->samples_done;
    return PERCIS_OK;
}

}  // extern "C"
