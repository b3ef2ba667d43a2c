// Library-internal host-side state of the PercIS library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "percis.h"
#include "percis_internal.h"

namespace percis {

// One graph with its states: the graph's host copy in internal ids (nodes
// with arcs first, caller order kept) and its device copy; the states and
// everything derived from them live on the device only.
struct GraphData {
    bool has_graph = false, directed = false;
    int32_t n = 0, n_act = 0;
    int64_t m = 0;
    std::vector<int32_t> h_rp, h_col;      // out-adjacency, rows sorted
    std::vector<int32_t> h_irp, h_icol;    // in-adjacency (directed graphs only)
    std::vector<int32_t> h_ccol;           // in-rows with entries in caller id order (the canonical walk)
    std::vector<int32_t> h_orig, h_newid;  // internal id -> caller id, and back
    bool graph_on_device = false;
    int32_t *d_rp = nullptr, *d_col = nullptr, *d_irp = nullptr, *d_icol = nullptr, *d_orig = nullptr;
    int32_t* d_ccol = nullptr;
    uint32_t* d_hits = nullptr;            // hits buffer owned by the library

    int32_t* d_newid = nullptr;            // caller id -> internal id (device)

    // States and the pair distribution, device-resident (built on the device
    // from k; a host-only context only validates states).
    bool has_states = false;
    uint64_t C = 0;                        // total pair weight (units of 1/65535)
    double d_hat = 1.0;                    // max(1, max_v C / S_v)
    bool states_on_device = false;
    uint16_t* d_k = nullptr;               // states by caller id
    int32_t* d_perm = nullptr;             // rank -> internal id
    uint32_t* d_kr = nullptr;
    uint64_t *d_W = nullptr, *d_P = nullptr;
    double *d_dv = nullptr, *d_Sv = nullptr;  // C / S_v and S_v by caller id
    void* build_mem = nullptr;             // scratch of the state build
    double* d_p = nullptr;                 // staging of the estimates, by caller id
    unsigned long long* d_red = nullptr;   // reduction word

    int64_t D_override = -1;
    int64_t D_cached = -1;                 // VertexDiamUB (the graph never changes after loading)
};

// A task as the host sees it: a sample range of one graph into device hits.
struct TaskSpec {
    int32_t graph;
    uint32_t phase;
    uint64_t first, count, seed;
    uint32_t* d_hits;
    bool accumulate;
};

}  // namespace percis

struct percis_ctx {
    int device = 0;
    bool host_only = false;                // created with PERCIS_HOST_ONLY: input validation only
    hipStream_t stream = nullptr;
    std::string err;
    int cu_count = 0;
    double wall_hz = 0.0;                  // device wall-clock rate

    std::vector<percis::GraphData*> graphs;  // [0] is the graph of percis_load_csr

    void* slot_mem = nullptr;
    int nslots = 0;
    int64_t slot_act = 0;                  // largest graph (nodes with arcs) the slots fit
    percis::DevSlots slots{};
    percis::SamplerShape shape{};

    percis::DevStats* d_stats = nullptr;   // launch-wide counters
    unsigned long long* d_work = nullptr;  // [6]: next list entry (or source), listed pairs, listed wide samples,
                                           //      next wide entry, listed handed-on samples, next handed-on entry
    percis::PairRec* d_pairs = nullptr;    // pair list of one chunk
    percis::PairRec* d_wide = nullptr;     // samples of one chunk with sigma_st >= 2^64
    percis::PairRec* d_big = nullptr;      // samples of one chunk that outgrew a compact slot
    void* cslot_mem = nullptr;             // compact slots (none when ncslots = 0)
    int ncslots = 0;
    percis::DevSlots cslots{};
    percis::SamplerShape cshape{};
    void* wide_mem = nullptr;              // scratch of the 128-bit path
    int wide_slots = 0;
    percis::WideSlots wslots{};
    percis::WideDebug* d_wdbg = nullptr;   // debug request of the 128-bit path, followed by its path
    int32_t wdbg_cap = 0;
    uint64_t pair_cap = 0;
    std::vector<hipEvent_t> chunk_ev;      // 3 per chunk: pairs, sampler, end
    percis::DevTask* d_tasks = nullptr;
    percis::DevStats* d_task_stats = nullptr;
    int task_cap = 0;
    percis::DebugOut* d_dbg = nullptr;
    int32_t dbg_cap = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipStream_t cap_stream = nullptr;      // private stream for capturing and replaying batches
    uint64_t generation = 0;               // bumped whenever a captured launch's buffers or inputs change

    int64_t opt_slots = 0, opt_scratch_mb = 0, opt_block = 0, opt_bitmaps = 0, opt_compact = 0, opt_defer_block = 0;
    int64_t opt_pair_chunk = 0, opt_balance = 0;
    void* noalloc = nullptr;               // this device's copy of the no-allocation scratch
};

namespace percis {

int fail(percis_ctx* c, int code, const char* fmt, ...);

// Size of the static device scratch of percis_sample_range_noalloc (one copy
// per GPU the library runs on, held until the process ends).
constexpr int64_t kNoAllocScratchBytes = 256ll << 20;
// Device address of the context's device's copy of that scratch, looked up
// once per device (percis_create does it).
int noalloc_scratch(percis_ctx* c, void** out);

#define HIPCHK(c, expr)                                                                            \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return ::percis::fail((c), e_ == hipErrorOutOfMemory ? PERCIS_E_NOMEM : PERCIS_E_DEVICE, \
                                  "%s: %s", #expr, hipGetErrorString(e_));                         \
    } while (0)

template <class T>
void dfree(T*& p) {
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

template <class T>
int dalloc(percis_ctx* c, T*& p, size_t count) {
    dfree(p);
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, sizeof(T) * (count ? count : 1));
    if (e != hipSuccess)
        return fail(c, PERCIS_E_NOMEM, "hipMalloc(%zu bytes): %s", sizeof(T) * count, hipGetErrorString(e));
    p = (T*)q;
    return PERCIS_OK;
}

// A task launch that the caller keeps in flight (the query server runs two
// at a time on the context's stream): device task table and statistics,
// their pinned host copies, and events.
struct AsyncLaunch {
    int cap = 0;                       // tasks the buffers hold
    std::vector<TaskSpec> tasks;       // the launch's tasks
    std::vector<DevTask> table;        // host task table (read by the upload until the launch ends)
    DevTask* d_tasks = nullptr;
    DevStats* d_tstats = nullptr;      // per task
    DevStats* d_lstats = nullptr;      // launch-wide
    DevStats* h_tstats = nullptr;      // pinned copies
    DevStats* h_lstats = nullptr;
    hipEvent_t start = nullptr, end = nullptr, done = nullptr;
};
int async_launch_init(percis_ctx* c, AsyncLaunch* a, int cap);
void async_launch_free(AsyncLaunch* a);
int launch_tasks_async(percis_ctx* c, const std::vector<TaskSpec>& tasks, AsyncLaunch* a);
int finish_tasks_async(percis_ctx* c, AsyncLaunch* a, std::vector<percis_stats>* out, percis_stats* launch);

int set_device(percis_ctx* c);
int graph_upload(percis_ctx* c, GraphData& G, bool states);
GraphData* get_graph(percis_ctx* c, int32_t id);
int run_tasks(percis_ctx* c, const std::vector<TaskSpec>& tasks, std::vector<percis_stats>* out, percis_stats* launch);
// The bounds of Algorithm 1 from phase 1 (the device reduction of the hits
// runs on `stream`, which is synchronised).
int phase1_bounds(percis_ctx* c, const GraphData& G, uint64_t l1, uint64_t sum_I, uint64_t sum_I2,
                  const uint32_t* d_hits1, double eps, double delta, percis_estimate_info* I, hipStream_t stream);
int vertex_diam_ub(percis_ctx* c, GraphData& G, int64_t* D);
// p_out[v] = d_v h_v / l through the graph's staging array, on `stream` (synchronised).
int estimates_to_host(percis_ctx* c, const GraphData& G, const uint32_t* d_hits, uint64_t l, double* p_out,
                      hipStream_t stream);

}  // namespace percis
