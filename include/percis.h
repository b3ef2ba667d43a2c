/*
 * percis.h -- C ABI of the MI355X (gfx950) PercIS hot path.
 *
 * PercIS (Cruciani & Pellegrina, "Fast Percolation Centrality Approximation
 * with Importance Sampling") estimates the percolation centrality p(v) of
 * every node (Definition 1, Eq. 1) by importance sampling: each sample draws
 * an ordered pair (s,t) with probability kappa~(s,t) proportional to
 * R(x_s - x_t) = max(0, x_s - x_t) (Section III-A), picks one shortest s-t
 * path uniformly at random (RandomSP, Section III-B) and credits every
 * internal node of that path. Because kappa(s,t,v)/kappa~(s,t) equals the
 * per-node constant d_v = C / S_v for every sampled pair (proof of
 * Proposition 5), the per-sample output reduces to integer hit counts h_v and
 * the estimate is p~(v) = d_v h_v / l.
 *
 * Conventions
 *  - Every call returns an int status: PERCIS_OK (0) or a negative error
 *    code. No C++ exception crosses this boundary. percis_last_error() gives
 *    a human-readable message for the last failing call on a context.
 *  - A context owns every device buffer it allocates. Outputs are written
 *    only into caller-owned buffers; the library never hands an allocation
 *    to the caller. One context is used by one host thread at a time;
 *    distinct contexts may be used concurrently.
 *  - Pointers are host pointers unless the call's flags contain
 *    PERCIS_DEVICE_PTRS, in which case they are device pointers on the
 *    context's device (for instance the data of torch tensors).
 *  - All device work is enqueued on the context's HIP stream (the null
 *    stream unless one was given); calls that return host results
 *    synchronise that stream before returning. Captured batches
 *    (percis_batch_*) replay on a private stream of the context, after its
 *    stream has drained, and return when they have finished.
 *  - Percolation states are quantised: x_v = k_v / 65535 with k_v in
 *    0..65535; all sampling arithmetic is exact integer arithmetic.
 *  - Graphs are unweighted, given as CSR with int32 node ids; undirected
 *    graphs store both arcs of every edge. Limits: 1 <= n <= 2^25 nodes
 *    (so that the integer pair weights fit in 64 bits), m <= 2^31 - 1 arcs.
 */
#ifndef PERCIS_H
#define PERCIS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define PERCIS_OK                 0
#define PERCIS_E_INVAL           -1  /* bad argument or malformed graph */
#define PERCIS_E_STATE           -2  /* call out of order (no graph / no states) */
#define PERCIS_E_NOMEM           -3  /* device or host allocation failed */
#define PERCIS_E_DEVICE          -4  /* HIP runtime error */
#define PERCIS_E_DEGENERATE      -5  /* all states equal: kappa~ undefined */
#define PERCIS_E_TOO_LARGE       -6  /* n > 2^25, or 2^32 or more samples in one call */
#define PERCIS_E_SIGMA_OVERFLOW  -7  /* a sampled pair has 2^128 - 1 or more shortest paths */

/* ---- flags ---- */
#define PERCIS_DIRECTED     0x1u  /* load_csr: arcs are directed */
#define PERCIS_DEVICE_PTRS  0x2u  /* pointer arguments are device memory */
#define PERCIS_ACCUMULATE   0x4u  /* sample_range: add to hits instead of overwriting */

typedef struct percis_ctx percis_ctx;

/* Per-call statistics of the sampler. |I(tau)| is the number of internal
 * nodes of the sampled path (Section II-A); it is d(s,t) - 1 for a reachable
 * pair and 0 for an unreachable one. The four work counters count, over all
 * samples of the call: adjacency entries examined (edges), shortest-path
 * count accumulations (sigma_adds), vertices whose adjacency was scanned
 * (vertices_expanded) and vertices first reached (vertices_discovered).
 * Results (hits, samples, reachable, sum_I, sum_I2, overflow) never depend
 * on timing; the work counters may vary slightly between runs, because
 * arcs of a search's last level that do not reach the other ball are skipped
 * as soon as any thread has seen one that does, and because a sample near a
 * compact slot's table limit may or may not be handed on and redone. */
typedef struct {
    uint64_t samples;
    uint64_t reachable;
    uint64_t sum_I;
    uint64_t sum_I2;
    uint64_t overflow;          /* samples with sigma_st >= 2^128 - 1 (their counts saturate) */
    uint64_t first_overflow;    /* smallest such sample index, or UINT64_MAX */
    uint64_t edges;
    uint64_t sigma_adds;
    uint64_t vertices_expanded;
    uint64_t vertices_discovered;
    double   kernel_ms;         /* device time of the sampling kernel (searches and walks) */
    /* Time spent per sample phase, summed over the concurrently running
     * samples (slot-milliseconds): starting the two balls, the bidirectional
     * BFS, the meeting layer and the sigma_s sweep, the path walk (during
     * which one wave claims the next sample), and clearing the slot. */
    double   phase_ms[5];
    double   pair_ms;           /* device time of the pair kernel (Algorithm 2 draws) */
    uint64_t spilled;           /* samples whose visited set on a side outgrew its LDS table */
    uint64_t deferred;          /* samples a compact slot handed to the per-node slots (PERCIS_OPT_COMPACT) */
    /* kernel_ms split by sampler pass: [0] the first pass (the compact slots
     * when they are on, else the only pass), [1] the per-node slots' pass over
     * the samples handed on, with the 128-bit path's launch. Captured replays
     * report 0 for both. */
    double   pass_ms[2];
} percis_stats;

/* Result summary of percis_estimate (Algorithm 1). */
typedef struct {
    uint64_t l1;          /* phase-1 sample size, ceil(max(1000, ln(1/delta)/eps)) */
    uint64_t l;           /* phase-2 sample size (Theorem 1 with Alg. 1's constants) */
    int64_t  D;           /* vertex-diameter bound used */
    double   d_hat;       /* likelihood ratio max_v C / S_v */
    double   rho_tilde;   /* phase-1 mean of |I| */
    double   Lambda;      /* phase-1 unbiased sample variance of |I| */
    double   rho_hat;     /* Proposition 2 bound, at delta/4 */
    double   v_hat;       /* Proposition 3 bound, at delta/4 */
    double   x_hat;       /* d/2 - sqrt(d^2/4 - min(d^2/4, v_hat)) */
    double   phase1_ms, bounds_ms, phase2_ms, total_ms;
    uint64_t overflow;    /* overflowed samples over both phases */
} percis_estimate_info;

/* Creates a context on HIP device `device`. `hip_stream` is a hipStream_t
 * (NULL = null stream) that every later call enqueues on; it must outlive the
 * context or be replaced with percis_set_stream. device = PERCIS_HOST_ONLY
 * creates a context that makes no HIP call at all: it validates graphs and
 * states, and every call that needs the device returns PERCIS_E_STATE. The
 * device copy of the graph is uploaded by the first call that needs it
 * (percis_set_states does). */
#define PERCIS_HOST_ONLY (-1)
int percis_create(int device, void* hip_stream, percis_ctx** out);
void percis_destroy(percis_ctx* ctx);
int percis_set_stream(percis_ctx* ctx, void* hip_stream);

/* Loads the graph G = (V, E) of Section II-A: row_ptr[n+1], col[m]
 * (row_ptr[0] = 0, non-decreasing, row_ptr[n] = m, 0 <= col < n). Rejected
 * with PERCIS_E_INVAL: self-loops, duplicate arcs (E is a set), and for an
 * undirected graph an arc whose reverse is missing. Rows need not be sorted;
 * the library keeps its own sorted copy. For a directed graph the library
 * also builds the in-adjacency. Discards previously set states.
 * flags: PERCIS_DIRECTED, PERCIS_DEVICE_PTRS. */
int percis_load_csr(percis_ctx* ctx, int32_t n, int64_t m, const int32_t* row_ptr,
                    const int32_t* col, uint32_t flags);

/* Sets the percolation states x_v = k[v] / 65535 (k[n] uint16) and builds the
 * exact integer pair distribution on the device: ranks sorted by
 * (k non-increasing, node id increasing) (Section II-A, "up to a
 * relabelling"), then the preprocessing of Algorithm 2 (appendix) in units of
 * 1/65535, and the weights d_v = C / S_v. The graph stays on the device: a
 * state-only update moves k (2n bytes) and nothing else, and with
 * PERCIS_DEVICE_PTRS k is device memory and never leaves the device. Only C
 * and d_hat come back to the host. Returns PERCIS_E_DEGENERATE if all states
 * are equal (the total weight C is 0, Definition 1 undefined); the graph then
 * has no states until the next successful call. Synchronises the context's
 * stream. flags: PERCIS_DEVICE_PTRS. */
int percis_set_states(percis_ctx* ctx, const uint16_t* k, uint32_t flags);

/* Draws samples first .. first+count-1 of the stream (seed, phase): for each,
 * the pair (s,t) of Algorithm 2, a shortest-path-counting BFS (balanced
 * bidirectional, Section III-B), the r-th shortest path in canonical order
 * (r uniform in [0, sigma_st); walking back from t, the predecessors of a node
 * are taken in ascending caller id, each covering sigma_s of the indices),
 * and one hit to each internal node.
 * hits[n] (uint32) receives the per-node hit counts; hit counts over disjoint
 * index ranges add up. The random stream is Philox4x64-10 with key
 * (seed, phase) and counter (sample index, variate, attempt, 0), so results do
 * not depend on launch configuration. Requires count < 2^32. Returns
 * PERCIS_E_SIGMA_OVERFLOW if any sampled pair has sigma_st >= 2^128 - 1
 * (such samples add no hits; st reports the count and first index). Pairs
 * with 2^64 <= sigma_st < 2^128 - 1 take a 128-bit path (r drawn at 128 bits,
 * the same stream) and count like any other.
 * st may be NULL. flags: PERCIS_DEVICE_PTRS (hits is device memory),
 * PERCIS_ACCUMULATE. */
int percis_sample_range(percis_ctx* ctx, uint64_t first, uint64_t count, uint64_t seed, uint32_t phase,
                        uint32_t* hits, uint32_t flags, percis_stats* st);

/* percis_sample_range(ctx, 0, n_samples, seed, 0, hits, flags, st). */
int percis_sample(percis_ctx* ctx, uint64_t n_samples, uint64_t seed, uint32_t* hits, uint32_t flags,
                  percis_stats* st);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * samples, hits and statistics as percis_sample_range on the context's graph
 * 0, with no hipMalloc, hipFree or other allocation in the call. Every
 * scratch buffer of the launch lies in a static device array of the library,
 * 256 MiB per GPU (allocated once when the library is first used on a GPU,
 * held until the process ends): the pair lists of chunks of at most 2^16
 * samples, the visited-set slots and one slot of the 128-bit path, laid out
 * anew for each call and cleared by kernels first. Requirements: the graph
 * and its states were set with percis_load_csr and percis_set_states (those
 * calls allocate); hits is device memory (flags must contain
 * PERCIS_DEVICE_PTRS; PERCIS_ACCUMULATE is allowed). Returns
 * PERCIS_E_TOO_LARGE when the graph has more nodes with arcs than one
 * per-node slot and one 128-bit slot can hold in the array (about 3.6
 * million), PERCIS_E_INVAL without PERCIS_DEVICE_PTRS, PERCIS_E_STATE before
 * a graph with states. All calls on one GPU share the array, whatever their
 * context: calls that overlap on one GPU (other host threads, other streams)
 * race and give wrong results. kernel_ms covers the whole call (pair draws
 * included); pair_ms and pass_ms are 0. */
int percis_sample_range_noalloc(percis_ctx* ctx, uint64_t first, uint64_t count, uint64_t seed, uint32_t phase,
                                uint32_t* hits, uint32_t flags, percis_stats* st);

/* Algorithm 1 (PercIS): VertexDiamUB, l1 samples in phase 1, the bounds of
 * Propositions 2 and 3 and the sample size of Theorem 1 (with the constants
 * of Alg. 1), l samples in phase 2, and p_out[v] = d_v h_v / l (host array of
 * n doubles; p := 0 where S_v = 0). Requires 0 < eps < 1, 0 < delta < 1.
 * info may be NULL. */
int percis_estimate(percis_ctx* ctx, double eps, double delta, uint64_t seed, double* p_out,
                    percis_estimate_info* info);

/* ---- many graphs in one launch ----
 * A context holds graph 0 (set by percis_load_csr / percis_set_states) and
 * any number of further graphs added with percis_add_graph. A task is a
 * sample range of one graph; percis_sample_tasks runs any set of tasks, on
 * any mix of graphs, through one persistent launch (the samples of all tasks
 * share the device's workgroups). Each task's hits and statistics equal what
 * percis_sample_range would give for the same graph, range, seed and phase. */

/* Adds a graph with its states (arguments as for percis_load_csr followed by
 * percis_set_states; flags: PERCIS_DIRECTED, PERCIS_DEVICE_PTRS) and returns
 * its id (>= 1) in *graph_id. */
int percis_add_graph(percis_ctx* ctx, int32_t n, int64_t m, const int32_t* row_ptr, const int32_t* col,
                     const uint16_t* k, uint32_t flags, int32_t* graph_id);

/* Size of graph `graph`: nodes, arcs, and nodes with at least one arc. */
int percis_graph_info(percis_ctx* ctx, int32_t graph, int32_t* n, int64_t* m, int32_t* n_active);

typedef struct {
    int32_t graph;        /* graph id (0 = the graph of percis_load_csr) */
    uint32_t phase;       /* stream phase */
    uint64_t first;       /* first sample index */
    uint64_t count;       /* number of samples, < 2^32 */
    uint64_t seed;
    uint32_t* hits;       /* device memory, n entries of that graph, caller-owned */
    uint32_t flags;       /* PERCIS_ACCUMULATE or 0 */
    percis_stats* stats;  /* host, receives this task's sample statistics; may be NULL */
} percis_task;

/* Runs ntasks tasks in one launch on the context's stream and waits for it.
 * Each task's stats receive its sample counts (samples, reachable, sum_I,
 * sum_I2, overflow, first_overflow) and the kernel time; launch_stats (may be
 * NULL) receives the sums over all tasks plus the launch-wide work counters
 * and phase times. Returns PERCIS_E_SIGMA_OVERFLOW if any task overflowed. */
int percis_sample_tasks(percis_ctx* ctx, int32_t ntasks, const percis_task* tasks, percis_stats* launch_stats);

/* The same launch as a HIP graph, for callers that run one task set again and
 * again (a batch step): percis_batch_capture uploads the task table, makes
 * sure the device copies, slots and list buffers exist, and captures the
 * launch's kernels (task clearing, then per chunk (PERCIS_OPT_PAIR_CHUNK) the
 * pair kernel, the sampler and the 128-bit path) on a private stream into a
 * graph owned by *batch. percis_batch_replay launches the graph, waits, and
 * fills each task's stats (the pointers given at capture) and launch_stats
 * (may be NULL) as percis_sample_tasks does; kernel_ms is the graph's device
 * time and pair_ms 0. A replay gives exactly the hits and statistics of
 * percis_sample_tasks on the same tasks. The capture holds device addresses
 * and each graph's total weight: after percis_load_csr, percis_set_states
 * (successful or not), percis_set_option (other than PERCIS_OPT_BALANCE, whose
 * rule a capture keeps), or a launch with a larger chunk than any before on
 * this context, a replay returns PERCIS_E_STATE (capture again). Destroy batches
 * before their context. Replays of one context run one at a time. */
typedef struct percis_batch percis_batch;
int percis_batch_capture(percis_ctx* ctx, int32_t ntasks, const percis_task* tasks, percis_batch** batch);
int percis_batch_replay(percis_batch* batch, percis_stats* launch_stats);
void percis_batch_destroy(percis_batch* batch);

/* Algorithm 1 on graph `graph` (percis_estimate is this with graph 0). */
int percis_graph_estimate(percis_ctx* ctx, int32_t graph, double eps, double delta, uint64_t seed, double* p_out,
                          percis_estimate_info* info);

/* PercIS-DI, the data-independent variant of Section IV (sample size bound
 * experiment): no first phase; rho_hat = D (the vertex-diameter bound) and
 * v_hat = d_hat^2 / 4 (its largest possible value) in Theorem 1's sample size
 * (Alg. 1's constants), then l samples of stream phase 2 and
 * p_out[v] = d_v h_v / l as in percis_estimate. info->l1 = 0. */
int percis_graph_estimate_di(percis_ctx* ctx, int32_t graph, double eps, double delta, uint64_t seed,
                             double* p_out, percis_estimate_info* info);
int percis_graph_set_vertex_diameter(percis_ctx* ctx, int32_t graph, int64_t D);

/* Overrides VertexDiamUB with a caller-known bound D >= the maximum number of
 * internal nodes of any shortest path (D < 0 restores the default: a BFS per
 * connected component for undirected graphs, the largest weakly connected
 * component's size minus 2 for directed ones). */
int percis_set_vertex_diameter(percis_ctx* ctx, int64_t D);

/* VertexDiamUB of Algorithm 1 (Section III-B) for graph `graph` into *D: the
 * override if one is set, else computed on the device once per loaded graph
 * (connected components by min-label hooking; for an undirected graph, per
 * component, a BFS from its node u of smallest caller id gives min(|comp| - 2,
 * 2 ecc(u) - 1); for a directed graph the largest weakly connected
 * component's size minus 2; components of one node give 0). Synchronises the
 * context's stream. */
int percis_graph_vertex_diameter(percis_ctx* ctx, int32_t graph, int64_t* D);

/* Test hook: runs RandomSP on the device for a given pair (s, t) and path
 * index r < 2^64, with 64-bit counts. Writes L = d(s,t) (-1 if unreachable)
 * and sigma_st (2^64 - 1 with *overflow = 1 when sigma_st >= 2^64: then see
 * percis_debug_path_wide); if reachable, not overflowed, r < sigma_st and
 * cap >= L + 1, writes the path s, ..., t into path[] (host). */
int percis_debug_path(percis_ctx* ctx, int32_t s, int32_t t, uint64_t r, int32_t* path, int32_t cap,
                      int32_t* L, uint64_t* sigma, int32_t* overflow);

/* Test hook of the 128-bit path that sampling calls take for pairs with
 * sigma_st >= 2^64: RandomSP for (s, t) and r = r_lo + 2^64 r_hi with exact
 * 128-bit counts. Writes L (-1 if unreachable), sigma_st as two halves
 * (2^128 - 1 and *overflow = 1 when it saturates) and, if reachable, not
 * overflowed, r < sigma_st and cap >= L + 1, the path s, ..., t. */
int percis_debug_path_wide(percis_ctx* ctx, int32_t s, int32_t t, uint64_t r_lo, uint64_t r_hi, int32_t* path,
                           int32_t cap, int32_t* L, uint64_t* sigma_lo, uint64_t* sigma_hi, int32_t* overflow);

/* Test hook: copies the device-built pair distribution of graph `graph`
 * (Algorithm 2's preprocessing in units of 1/65535) to host arrays, each may
 * be NULL: perm[n+1] (rank -> caller's node id, ranks sorted by k
 * non-increasing then id increasing; perm[0] = -1), kr[n+2] (k of rank i;
 * kr[0] = kr[n+1] = 0), W[n+2] (W[i] = sum_{j >= i} kr[j]), P[n+1]
 * (P[i] = sum_{j <= i} ((n-j+1) kr[j] - W[j]), so P[n] = C), d_v[n] and
 * S_v[n] by node id (S_v = the weight of the pairs that avoid v,
 * d_v = C / S_v or 0), and the scalars C and d_hat = max(1, max_v d_v).
 * Synchronises the context's stream. */
int percis_debug_states(percis_ctx* ctx, int32_t graph, int32_t* perm, uint32_t* kr, uint64_t* W, uint64_t* P,
                        double* d_v, double* S_v, uint64_t* C, double* d_hat);

/* Exact percolation centrality of graph `graph` (Definition 1, Eq. 1) on the
 * device, by Brandes-style dependency accumulation from every source (the
 * paper's exact baseline, Section IV-A): p_out[n] (host), p := 0 where S_v =
 * 0; *kernel_ms (may be NULL) gets the device time. O(n m) work; the sums are
 * in double, so results agree with a serial computation to rounding. */
int percis_exact(percis_ctx* ctx, int32_t graph, double* p_out, double* kernel_ms);

/* Tuning knobs (launch shape only; results never depend on them).
 * PERCIS_OPT_SLOTS: concurrent samples (resident workgroups), 0 = auto.
 * PERCIS_OPT_COMPACT: compact slots, whose node records are indexed by the
 * node's place in the side's LDS table (about 300 KB per slot instead of
 * ~48 bytes per node of the graph): 1 = off; 2 = on, with the per-node slots
 * redoing every sample that a side's table cannot hold (more than 1536 nodes);
 * 0 = auto (on when LDS tables are used and the per-node slots are too few,
 * for lack of memory, to fill the device). Reads 1 or 2 once a graph is
 * loaded. PERCIS_OPT_SLOTS reads the compact slots' count when they are on.
 * PERCIS_OPT_SCRATCH_MB: cap on the sampler's scratch memory, 0 = auto (up to
 * 80 % of the free device memory when a graph is large enough to need it).
 * PERCIS_OPT_BLOCK: threads per sample (64, 128, 256, 512 or 1024), 0 = auto
 * (auto also runs a launch of at most 16 samples per slot with 512 threads
 * per sample on fewer slots: such a launch is bound by its slowest samples).
 * PERCIS_OPT_BITMAPS: how a sample's visited sets are kept: 1 = one bitmap
 * per side in device memory; 2 = an exact hash table per side in LDS (8 KB
 * per sample, 64 KB at 512 threads or more), moved to the device bitmap if a
 * side grows past 3/4 of it (768 nodes; 6144 at 512 threads or more);
 * 0 = auto (2 unless it lowers the number of resident samples).
 * Reading PERCIS_OPT_SLOTS, _BLOCK or _BITMAPS after a graph is loaded gives
 * the shape in use (BITMAPS then reads 1 or 2). */
#define PERCIS_OPT_SLOTS       1
#define PERCIS_OPT_SCRATCH_MB  2
#define PERCIS_OPT_BLOCK       3
#define PERCIS_OPT_BITMAPS     4
#define PERCIS_OPT_COMPACT     5
/* PERCIS_OPT_DEFER_BLOCK: threads per sample of the per-node slots while
 * compact slots are on (they then only run the samples with large balls):
 * 64 .. 1024, 0 = auto. */
#define PERCIS_OPT_DEFER_BLOCK 6
/* PERCIS_OPT_PAIR_CHUNK: samples per chunk of a launch, 1 .. 2^30, 0 = auto
 * (2^24). The pair kernel draws and lists one chunk's pairs before the
 * sampler runs them; the lists take 48 bytes of device memory per sample of a
 * chunk. Results do not depend on it. Reading it gives the chunk in use. */
#define PERCIS_OPT_PAIR_CHUNK  7
/* PERCIS_OPT_BALANCE: the side rule of the balanced bidirectional search
 * (Section III-B): the s ball grows the next level while the degree sum of
 * its frontier is at most BALANCE % of the t ball's, else the t ball grows.
 * 25 .. 400, 0 = auto (100: the ball with the smaller frontier degree sum).
 * The shortest-path counts, the canonical walk and so every result are the
 * same under any rule; only the work per sample changes. A captured launch
 * keeps the rule in force when it was captured. Reading it gives the rule in
 * use. */
#define PERCIS_OPT_BALANCE     8
int percis_set_option(percis_ctx* ctx, int option, int64_t value);
int percis_get_option(percis_ctx* ctx, int option, int64_t* value);

/* Autotuner: times one launch of probe_samples samples (stream phase 3, seed
 * `seed`) of graph `graph`, or split evenly over every graph with states when
 * `graph` is -1, under a staged search, and keeps the fastest knobs as the
 * context's options (PERCIS_OPT_BLOCK, _BITMAPS, _COMPACT, _SLOTS, _BALANCE):
 *   1. the automatic shape (every option 0), then threads per sample 128, 256,
 *      512, 1024 x visited sets in device bitmaps, in LDS tables, in LDS
 *      tables on compact slots (the work granularity and the frontier layout);
 *   2. the best shape on 3/4 and 1/2 of its slots (the batch width);
 *   3. the best so far under the side rules 50 and 200 (PERCIS_OPT_BALANCE).
 * Each candidate runs one untimed launch, then two timed ones; the faster
 * counts. A candidate that cannot run (memory, occupancy) is passed over.
 * The choice is reported in *result (may be NULL). Results of sampling calls
 * never depend on any of these knobs. Errors: E_INVAL (no graph, probe size
 * outside 1 .. 2^32 - 1), E_STATE (no states; no graph with states for -1;
 * host-only context), E_DEVICE (no candidate could run); the options are
 * restored to their values before the call on error. */
typedef struct {
    int32_t block;          /* threads per sample of the first pass (the compact slots' when compact is 2) */
    int32_t bitmaps;        /* visited sets: 1 = device bitmaps, 2 = LDS tables */
    int32_t slots;          /* concurrent samples of the first pass */
    int32_t candidates;     /* candidates timed */
    double samples_per_s;   /* probe throughput of the choice */
    int32_t compact;        /* 1 = per-node slots only, 2 = compact slots first */
    int32_t balance;        /* side rule (PERCIS_OPT_BALANCE) */
    int32_t defer_block;    /* threads per sample of the pass over the samples handed on (compact 2), else 0 */
    double auto_samples_per_s; /* probe throughput with every option 0 */
} percis_tuning;
int percis_autotune(percis_ctx* ctx, int32_t graph, uint64_t probe_samples, uint64_t seed, percis_tuning* result);

/* ---- serving: continuous batching of centrality queries ----
 * A server runs Algorithm 1 queries (graph, eps, delta, seed) over the graphs
 * resident in its context. percis_server_create allocates one device pool of
 * memory_budget_bytes (rounded down to 256 bytes); queries wait in arrival
 * order until their hit buffer (4 bytes per node, rounded up to 256) fits in
 * it (first fit, no further allocation per query). A launch of at most
 * step_samples samples carries phase 1 of every admitted query in that
 * phase (at most chunk_samples samples of each per launch), then phase 2 of
 * the others in arrival order, each taking what it still needs from what is
 * left. Two launches are kept in flight on the
 * context's stream; each percis_server_step waits for the older one, reads
 * its statistics, finishes the phases it completed (the bounds of Algorithm
 * 1, the estimates; on a second stream of the server), retires and admits
 * queries and enqueues the next launch. Queries of different graphs share
 * the device, and a query submitted while others run joins a launch at the
 * next step. A query's result is the same alone or in any mix, and equals
 * percis_graph_estimate with the same arguments. The server is used from one
 * host thread at a time; no other work may use the context while queries are
 * in flight. */
typedef struct percis_server percis_server;
int percis_server_create(percis_ctx* ctx, int64_t memory_budget_bytes, uint64_t chunk_samples,
                         uint64_t step_samples, percis_server** out);
void percis_server_destroy(percis_server* server);
/* Queues a query; returns its id. */
int percis_server_submit(percis_server* server, int32_t graph, double eps, double delta, uint64_t seed,
                         int64_t* query_id);
/* Admits what fits, keeps two launches in flight, waits for the older one
 * and advances and retires the queries it served; *completed (may be NULL)
 * counts queries that finished or failed in this step. Returns at once if
 * no query is active or queued. */
int percis_server_step(percis_server* server, int32_t* completed);
/* *done = 1 once the query has finished: its estimate is copied to p_out
 * (host, n_cap >= n of its graph; may be NULL), its summary to info (may be
 * NULL), the query is forgotten, and the query's own status is returned
 * (PERCIS_OK, or the error that stopped it). *done = 0 while it runs. */
int percis_server_result(percis_server* server, int64_t query_id, int32_t* done, double* p_out, int32_t n_cap,
                         percis_estimate_info* info);
/* Queue lengths, device bytes held by admitted queries (now and at peak),
 * and samples drawn so far. Any pointer may be NULL. */
int percis_server_status(percis_server* server, int32_t* queued, int32_t* active, int64_t* bytes_in_use,
                         int64_t* peak_bytes, uint64_t* samples_done);

const char* percis_status_str(int status);
const char* percis_last_error(const percis_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* PERCIS_H */
