// Continuous-batching query server over the graphs of a context.
//
// A query asks for Algorithm 1 (PercIS) on one resident graph with its own
// (eps, delta, seed). Queries wait in arrival order until their hit buffer
// (4 bytes per node) fits in the server's device-memory budget; admitted
// queries run their two sampling phases in chunks. Every step is one task
// launch that carries one chunk of every active query (in admission order,
// up to the step's sample budget), so queries of different graphs and sizes
// overlap on the device and a query that arrives while others run starts at
// the next step. A query's samples are indices of its own (seed, phase)
// stream, so its result is the same alone or in any mix, and equals
// percis_graph_estimate for the same arguments.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
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
    uint32_t* d_hits = nullptr;
    int64_t bytes = 0;
    uint64_t next = 0;             // next sample index of the current phase
    uint64_t target = 0;           // samples of the current phase
    uint64_t sum_I = 0, sum_I2 = 0, overflow = 0;
    percis_estimate_info info{};
    std::vector<double> p;
    std::chrono::steady_clock::time_point t_submit, t_admit;
};

}  // namespace

struct percis_server {
    percis_ctx* ctx = nullptr;
    int64_t budget = 0;
    int64_t in_use = 0;
    uint64_t chunk = 0;
    uint64_t step_samples = 0;
    int64_t next_id = 1;
    std::deque<Query*> queued;
    std::vector<Query*> active;                     // admission order
    std::unordered_map<int64_t, Query*> by_id;
    uint64_t samples_done = 0;
    double kernel_ms = 0;
    int64_t peak_in_use = 0;
};

namespace {

void release(percis_server* s, Query* q) {
    if (q->d_hits) {
        (void)hipFree(q->d_hits);
        q->d_hits = nullptr;
        s->in_use -= q->bytes;
    }
}

// Admits queued queries in arrival order while their buffers fit.
int admit(percis_server* s) {
    while (!s->queued.empty()) {
        Query* q = s->queued.front();
        if (s->in_use + q->bytes > s->budget && !s->active.empty()) break;
        if (s->in_use + q->bytes > s->budget && q->bytes > s->budget) {
            q->state = FAILED;
            q->status = PERCIS_E_NOMEM;
            s->queued.pop_front();
            continue;
        }
        void* p = nullptr;
        if (hipMalloc(&p, (size_t)q->bytes) != hipSuccess) {
            (void)hipGetLastError();
            if (s->active.empty()) {
                q->state = FAILED;
                q->status = PERCIS_E_NOMEM;
                s->queued.pop_front();
                continue;
            }
            break;
        }
        q->d_hits = (uint32_t*)p;
        s->in_use += q->bytes;
        s->peak_in_use = std::max(s->peak_in_use, s->in_use);
        q->state = PHASE1;
        q->info.l1 = (uint64_t)std::ceil(std::max(1000.0, std::log(1.0 / q->delta) / q->eps));
        q->target = q->info.l1;
        q->next = 0;
        q->t_admit = std::chrono::steady_clock::now();
        s->queued.pop_front();
        s->active.push_back(q);
    }
    return PERCIS_OK;
}

}  // namespace

extern "C" {

int percis_server_create(percis_ctx* ctx, int64_t memory_budget_bytes, uint64_t chunk_samples, uint64_t step_samples,
                         percis_server** out) {
    if (!ctx || !out || memory_budget_bytes <= 0 || chunk_samples == 0 || step_samples == 0) return PERCIS_E_INVAL;
    if (ctx->host_only) return fail(ctx, PERCIS_E_STATE, "host-only context cannot serve");
    percis_server* s = new (std::nothrow) percis_server();
    if (!s) return PERCIS_E_NOMEM;
    s->ctx = ctx;
    s->budget = memory_budget_bytes;
    s->chunk = chunk_samples;
    s->step_samples = std::max(step_samples, chunk_samples);
    *out = s;
    return PERCIS_OK;
}

void percis_server_destroy(percis_server* s) {
    if (!s) return;
    if (s->ctx && !s->ctx->host_only) {
        (void)hipSetDevice(s->ctx->device);
        (void)hipDeviceSynchronize();
    }
    for (auto& kv : s->by_id) {
        release(s, kv.second);
        delete kv.second;
    }
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
    if (s->active.empty()) return PERCIS_OK;

    // one chunk of every active query, in admission order, within the step budget
    std::vector<TaskSpec> tasks;
    std::vector<Query*> owners;
    uint64_t planned = 0;
    for (Query* q : s->active) {
        if (planned >= s->step_samples) break;
        const uint64_t left = q->target - q->next;
        const uint64_t take = std::min<uint64_t>(left, std::min<uint64_t>(s->chunk, s->step_samples - planned));
        if (take == 0) continue;
        const uint32_t phase = q->state == PHASE1 ? 1u : 2u;
        tasks.push_back(TaskSpec{q->graph, phase, q->next, take, q->seed, q->d_hits, q->next > 0});
        owners.push_back(q);
        planned += take;
    }
    if (tasks.empty()) return PERCIS_OK;
    std::vector<percis_stats> ts;
    percis_stats launch{};
    rc = run_tasks(c, tasks, &ts, &launch);
    if (rc != PERCIS_OK && rc != PERCIS_E_SIGMA_OVERFLOW) return rc;
    s->samples_done += launch.samples;
    s->kernel_ms += launch.kernel_ms + launch.pair_ms;

    int32_t done = 0;
    for (size_t i = 0; i < owners.size(); i++) {
        Query* q = owners[i];
        q->next += tasks[i].count;
        q->sum_I += ts[i].sum_I;
        q->sum_I2 += ts[i].sum_I2;
        q->overflow += ts[i].overflow;
        if (q->next < q->target) continue;
        GraphData& G = *get_graph(c, q->graph);
        if (q->overflow) {
            q->state = FAILED;
            q->status = PERCIS_E_SIGMA_OVERFLOW;
            q->info.overflow = q->overflow;
        } else if (q->state == PHASE1) {
            if ((rc = phase1_bounds(c, G, q->info.l1, q->sum_I, q->sum_I2, q->d_hits, q->eps, q->delta, &q->info)))
                return rc;
            if (q->info.l >= 4294967295ull) {
                q->state = FAILED;
                q->status = PERCIS_E_TOO_LARGE;
            } else {
                q->state = PHASE2;
                q->target = q->info.l;
                q->next = 0;
                continue;
            }
        } else {
            q->p.resize(G.n);
            if ((rc = estimates_to_host(c, G, q->d_hits, q->info.l, q->p.data()))) return rc;
            q->state = DONE;
            q->info.total_ms =
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - q->t_submit).count();
        }
        done++;
    }
    // retire finished queries and free their buffers for the next admissions
    std::vector<Query*> still;
    for (Query* q : s->active) {
        if (q->state == DONE || q->state == FAILED) release(s, q);
        else still.push_back(q);
    }
    s->active.swap(still);
    admit(s);
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
