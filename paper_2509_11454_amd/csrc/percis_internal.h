// Library-internal declarations shared by the host side (percis_api.cpp) and
// the device side (percis_kernels.hip). Nothing here is part of the ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace percis {

// Device view of the graph in internal node ids: nodes with at least one
// arc get ids 0..n_act-1 by degree (out + in), largest first, ties in caller
// order; nodes without arcs follow. Rows and in-rows are sorted by internal
// id, so the lanes that share a row touch neighbouring records. The
// canonical path takes predecessors in ascending caller id: ccol holds the
// in-rows again with their entries in that order.
struct DevGraph {
    int32_t n;
    int32_t n_act;
    const int32_t* rp;    // [n+1] out-adjacency
    const int32_t* col;   // [m]
    const int32_t* irp;   // [n+1] in-adjacency (same arrays if undirected)
    const int32_t* icol;  // [m]
    const int32_t* ccol;  // [m] in-rows (bounds irp), entries in ascending caller id; = icol + m
    const int32_t* orig;  // [n] internal id -> caller's id
};

// Device view of the exact integer pair distribution (Algorithm 2 in units
// of 1/65535): ranks i = 1..n sorted by (k non-increasing, caller id
// increasing).
struct DevCdf {
    int32_t n;
    uint64_t C;            // total weight, sum over ordered pairs of R(k_u - k_w)
    const int32_t* perm;   // [n+1]  perm[i] = internal id of rank i
    const uint32_t* kr;    // [n+2]  k of rank i
    const uint64_t* W;     // [n+2]  W[i] = sum_{j >= i} kr[j], W[n+1] = 0
    const uint64_t* P;     // [n+1]  P[i] = sum_{j <= i} c_j, c_j = (n-j+1) kr[j] - W[j]
};

// Per-node scratch of a slot: levels (value = level + 1, 0 = unreached, plus
// flag bits) and shortest-path counts from both ends, in one 32-byte record so
// that a visited node touches one memory sector.
struct NodeRec {
    uint32_t lv_s;
    uint32_t lv_t;
    uint64_t sg_s;
    uint64_t sg_t;
    uint64_t pad;
};

// Record of a compact slot, indexed by the node's position in its side's LDS
// visited table (one array of table size per side): level (+1, 0 =
// unreached, plus flag bits), then on the s side sigma_s, on the t side the
// sigma_s pulled through the t-ball (a meeting node's is copied from its s
// record) and sigma_t.
struct CRec {
    uint32_t lv;
    uint32_t pad;
    uint64_t ws;
    uint64_t wt;
    uint64_t pad2;
};

// One arc u -> v of a sample's shortest-path DAG with the count sigma_s(u)
// that weighs u among v's predecessors in the canonical walk.
struct DagArc {
    int32_t tail, head;
    uint64_t w;
};

// Per-slot scratch; the node arrays are [slots][stride] (stride >= n_act) and
// all-zero between samples (each sample clears what it touched). A compact
// slot set (crec != nullptr) has no per-node arrays: records are crec
// [slots][2][table size], the queues hold table positions with stride = table
// size (q_d: [slots][2][stride], s positions then t positions), and there
// are no bitmaps.
struct DevSlots {
    NodeRec* rec;     // per-node records
    int32_t* q_s;     // s-side BFS queue (levels are contiguous segments)
    int32_t* q_t;     // t-side BFS queue
    int32_t* q_d;     // meeting layer
    int32_t* tls;     // [slots][stride + 2] start of each t-level in q_t
    int64_t stride;   // elements per slot
    uint32_t* bm;     // visited bitmaps (device mode, or a spilled side in LDS mode): [slots][2][words]
    int64_t words;    // 32-bit words per bitmap
    DagArc* arcs;     // [slots][acap] arcs of the sample's shortest-path DAG, for the walk
    int32_t acap;     // arcs per slot
    CRec* crec;       // compact slot set: [slots][2][stride] records
    uint32_t* mlx;    // [slots][mlxcap][2] arcs into the other ball past the LDS list (head, staged tail | position)
    int32_t mlxcap;   // entries per slot
};

// Device-side accumulators of one sampling call.
struct DevStats {
    unsigned long long samples, reachable, sum_I, sum_I2, overflow, first_overflow;
    unsigned long long edges, sigma_adds, vexp, vdisc;
    unsigned long long spills;           // samples whose visited set outgrew an LDS table
    unsigned long long deferred;         // samples a compact slot handed to the per-node slots
    unsigned long long phase_ticks[5];   // summed over workgroups, wall-clock ticks
    unsigned long long walk_errors;      // samples whose walk found no predecessor (launch-wide only)
};

// One task of a launch: samples first .. first+count-1 of stream
// (seed, phase) on one graph. A launch runs many tasks (possibly on different
// graphs) through one persistent grid; the launch's sample index space is the
// concatenation of the tasks' ranges.
struct DevTask {
    DevGraph g;
    DevCdf cdf;
    uint64_t first, count, seed, phase;
    uint32_t* hits;                  // [g.n] by caller id
    DevStats* stats;                 // this task's sample statistics
    unsigned long long offset;       // launch index of the task's first sample
    uint32_t clear_hits;             // zero hits before sampling
    uint32_t pad;
};

// A sample whose pair needs a search: its launch index (minus the chunk's
// first), its pair (internal ids) and its task.
struct PairRec {
    uint32_t q;
    int32_t s, t, task;
};

// One chunk of a launch: launch indices base .. base+count-1. The pair kernel
// draws every pair of the chunk, counts the samples whose pair has an end
// without arcs (unreachable) and lists the others in pairs[0 .. *npairs);
// the sampler then claims list entries through *work.
struct SampleLaunch {
    const DevTask* tasks;            // device array
    int ntasks;
    uint32_t balance;                // the s side grows while its frontier degree sum is at most
                                     // balance % of the t side's (100: the balanced rule)
    unsigned long long base, count;  // the chunk
    PairRec* pairs;                  // [count] capacity
    unsigned long long* npairs;      // entries listed (written by the pair kernel)
    unsigned long long* work;        // next unclaimed list entry
    DevStats* stats;                 // launch-wide work counters and phase times
    int slots;                       // sampler grid size
    PairRec* wide;                   // [count] capacity: samples with sigma_st >= 2^64
    unsigned long long* nwide;       // entries listed (written by the sampler)
    PairRec* big;                    // [count] capacity: samples whose ball outgrew a compact slot
    unsigned long long* nbig;        // entries listed (written by the compact sampler)
    unsigned long long* big_work;    // next unclaimed entry of big (zeroed with the chunk)
};

// Scratch of the 128-bit path (samples with sigma_st >= 2^64): per slot, a
// distance (-1 = unreached), a 128-bit count and a queue entry per active node.
struct WideSlots {
    int32_t* dist;               // [slots][stride], all -1 between samples
    unsigned __int128* sigma;    // [slots][stride], all 0 between samples
    int32_t* queue;              // [slots][stride]
    int64_t stride;
    unsigned long long* work;    // next unclaimed wide-list entry
};

// Debug request of the 128-bit path.
struct WideDebug {
    int32_t s, t;
    unsigned __int128 r;
    int32_t L, overflow;         // overflow: sigma_st saturated (>= 2^128 - 1)
    unsigned __int128 sigma;
    int32_t cap;
    int32_t* path;               // device, cap entries
};

// Debug request: one (s, t, r) path; output written to `out`.
struct DebugOut {
    int32_t L;
    int32_t overflow;
    uint64_t sigma;
    int32_t path[1];   // flexible: L+1 entries (internal ids)
};

// Launch shape of the sampler: threads per workgroup and whether the
// visited sets are LDS tables (else device bitmaps).
struct SamplerShape {
    int block;        // 64, 128, 256, 512 or 1024 (compact: 64, 128 or 256)
    bool lds_sets;
    bool compact;     // compact slots (requires lds_sets)
    int64_t lds_bytes;  // dynamic LDS per workgroup (the visited-set tables) when lds_sets
};

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t count, hipStream_t stream);
hipError_t launch_fill_u8(void* p, int64_t bytes, hipStream_t stream);
hipError_t launch_init_stats(DevStats* st, unsigned long long* work, hipStream_t stream);
// Zeroes every task's statistics and, where asked, its hits (one launch).
hipError_t launch_clear_tasks(const DevTask* tasks, int ntasks, int64_t max_n, hipStream_t stream);
// Zeroes *work, *npairs and *nwide, then draws the chunk's pairs (one lane per sample).
hipError_t launch_pairs(const SampleLaunch& a, hipStream_t stream);
// The chunk's listed wide samples (a.wide[0 .. *a.nwide)) on `slots`
// workgroups (an empty list costs one short launch).
hipError_t launch_wide(const SampleLaunch& a, const WideSlots& w, int slots, hipStream_t stream);
// One (s, t, r) through the 128-bit path, on graph g, using slot 0 of w.
hipError_t launch_wide_debug(const DevGraph& g, const WideSlots& w, WideDebug* dbg, hipStream_t stream);
// The chunk's pairs on `slots` (per-node slots, or compact slots when
// slots.crec is set; these defer samples that outgrow them to a.big).
hipError_t launch_sampler(const DevSlots& slots, const SampleLaunch& a, const SamplerShape& shape,
                          hipStream_t stream);
hipError_t launch_debug_path(const DevGraph& g, const DevSlots& slots, int32_t s, int32_t t, uint64_t r,
                             DebugOut* out, int32_t cap, const SamplerShape& shape, hipStream_t stream);
// Exact percolation centrality: per-slot scratch of exact_scratch_bytes
// (all-zero on entry), sum over sources of the dependencies into out[n_act].
hipError_t launch_exact(const DevGraph& g, const uint16_t* k, void* scratch, int64_t stride, int slots,
                        unsigned long long* work, double* out, hipStream_t stream);
int64_t exact_scratch_bytes(int64_t stride, int slots);

// Resident workgroups per CU for a shape (0 if it cannot launch).
int sampler_occupancy(const SamplerShape& shape);
int64_t sampler_static_lds();
// Dynamic LDS of the visited-set tables (LDS mode) of a sampler with `block`
// threads per sample (per-node slots of 512 threads or more have larger
// tables), and the entries per side of a table (the records per side of a
// compact slot).
int64_t sampler_table_lds(bool compact, int block);
int sampler_table_cap(bool compact);

}  // namespace percis
