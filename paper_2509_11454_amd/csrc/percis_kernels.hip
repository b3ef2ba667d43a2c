// PercIS sampler kernels for gfx950 (MI355X).
//
// One persistent workgroup per slot claims launch indices from a global
// counter; a launch is a table of tasks (sample ranges of possibly different
// graphs). Results never depend on the launch shape: every sample's
// randomness is keyed on its index (Philox4x64-10, counter (index, variate,
// attempt, 0), key (seed, phase)), and all accumulation is integer.
//
// Slots come in two kinds. A per-node slot owns one 32-byte record per node
// (levels and shortest-path counts from both ends), three queues, two device
// bitmap planes and a DAG-arc list. A compact slot indexes its records by the
// node's position in its side's LDS visited table instead, so it costs a
// fixed few hundred KB whatever the graph; a sample whose side outgrows the
// table is handed on to the per-node slots and redone there. Visited sets
// are exact LDS hash tables; a per-node side that outgrows its table moves to
// its device bitmap plane. Every slot is all-zero between samples: each
// sample clears exactly what it touched.
//
// Per sample (Algorithm 2 of the paper's appendix, then RandomSP of
// Section III-B):
//   1. pair (pair_kernel, one lane per sample, ahead of the sampler): U_s
//      uniform in [0, C) picks rank s = min{d : U_s < P[d]}; U_t uniform in
//      [0, c_s) picks t = min{d > s : U_t < F_s(d)} with
//      F_s(d) = (d - s + 1) k_s - (W_s - W_{d+1}); both bounded draws use
//      Lemire's multiply-and-reject, both searches are per-lane bisections.
//      Pairs whose s has no out-arcs or whose t has no in-arcs are counted as
//      unreachable there.
//   2. balanced bidirectional BFS with shortest-path counting: the side whose
//      frontier has the smaller degree sum expands one full level, edge-
//      balanced across the workgroup; the first level that reaches the other
//      ball fixes d(s,t) = L and the meeting layer M, and
//      sigma_st = sum_{w in M} sigma_s(w) sigma_t(w). That last level keeps
//      only its arcs into the other ball (listed by a barrier-free first
//      pass).
//   3. shortest-path counts from s are pulled level by level from M down to
//      t through the t-ball, so that every node of the shortest-path DAG knows
//      sigma_s; every sigma_s add records its DAG arc, in one list segment per
//      distance from s.
//   4. r uniform in [0, sigma_st); the canonical backward walk from t takes,
//      among the predecessors one level closer to s in ascending caller id,
//      the first whose cumulative sigma_s exceeds r (from the step's segment
//      of the arc list, else from the in-row in caller order); once the walk
//      reaches s, every internal node of the path gets one hit.
// Counts are exact: a sample whose sigma_st reaches 2^64 is listed and redone
// by wide_kernel with 128-bit counts; only a count that saturates 128 bits is
// an overflow (no hits).
#include "percis_internal.h"

namespace percis {

constexpr int CH = 128;  // capacity of the LDS chunk arrays
// Frontier nodes staged per chunk: one per thread, at most CH.
template <int BSZ>
constexpr int chunk_len() { return BSZ < CH ? BSZ : CH; }
constexpr uint32_t LVMASK = 0x0FFFFFFFu;
constexpr uint32_t OVFBIT = 0x40000000u;
#ifndef PERCIS_UNROLL
#define PERCIS_UNROLL 6
#endif
constexpr int UNROLL = PERCIS_UNROLL;  // adjacency entries per thread per batch
#ifndef PERCIS_SCAN_UNROLL
#define PERCIS_SCAN_UNROLL 4
#endif
constexpr int SCAN_UNROLL = PERCIS_SCAN_UNROLL;  // entries per thread per step of a long chunk's first pass
// In-row chunks of 64 loaded together by the walk's row scan. One: the scan
// is rare since walk steps with up to 4096 predecessors select from the arc
// list, and the sampler's searches are sensitive to its code size (the
// 512-thread kernel at 57.6 KB ran its handed-on pass of directed R-MAT 24 in
// 245 ms, at 55.8 KB in 230 ms).
constexpr int WALK_UNROLL = 1;
constexpr int ARC_UNROLL = 4;   // DAG-arc chunks of 64 loaded together by the walk
constexpr int KCAP = 64;        // predecessors a walk step gathers from the arc list
constexpr int SEGCAP = 64;      // path positions whose arc-list segment a sample keeps
constexpr int MLCAP = 128;      // arcs into the other ball that a chunk's first pass lists in LDS
                                // (more go to the slot's device list, sl.mlxcap of them)

// Slot scratch is private to one workgroup (one CU), so every access to it is
// a workgroup-scope atomic: coherent among the workgroup's waves without the
// device-wide cache maintenance that agent scope costs on a multi-XCD part.
#define WGS __HIP_MEMORY_SCOPE_WORKGROUP

// Device memory through typed global pointers. A pointer loaded from a struct
// in memory is generic to the compiler, and a generic (flat) access counts
// against the LDS counter as well, so that every wait for an LDS result would
// also wait for the outstanding global loads. The sampler converts its graph
// and slot pointers into these views once.
template <class T>
using G = __attribute__((address_space(1))) T;
template <class T>
__device__ __forceinline__ G<T>* gptr(T* p) { return (G<T>*)p; }
// 16-byte records move as one vector access (a class type cannot be copied
// through an address-space-qualified pointer).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
template <class T>
__device__ __forceinline__ const G<T>* gptr(const T* p) { return (const G<T>*)p; }

__device__ __forceinline__ uint32_t ld32(G<uint32_t>* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, WGS); }
__device__ __forceinline__ uint64_t ld64(G<uint64_t>* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, WGS); }
__device__ __forceinline__ int32_t ldq(G<int32_t>* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, WGS); }
__device__ __forceinline__ uint32_t or32(G<uint32_t>* p, uint32_t v) {
    return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, WGS);
}
__device__ __forceinline__ uint64_t add64(G<uint64_t>* p, uint64_t v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, WGS);
}

// Field access by side: 0 = s side, 1 = t side.
template <int SIDE>
__device__ __forceinline__ G<uint32_t>* LV(G<NodeRec>* R, int32_t w) { return SIDE ? &R[w].lv_t : &R[w].lv_s; }
template <int SIDE>
__device__ __forceinline__ G<uint64_t>* SG(G<NodeRec>* R, int32_t w) { return SIDE ? &R[w].sg_t : &R[w].sg_s; }

// The graph and a slot's scratch as typed global views.
struct GGraph {
    int32_t n, n_act;
    const G<int32_t>* rp;
    const G<int32_t>* col;
    const G<int32_t>* irp;
    const G<int32_t>* icol;  // the caller-ordered in-rows follow at icol + m (m = irp[n])
    const G<int32_t>* orig;
};
__device__ __forceinline__ GGraph gview(const DevGraph& g) {
    return GGraph{g.n, g.n_act, gptr(g.rp), gptr(g.col), gptr(g.irp), gptr(g.icol), gptr(g.orig)};
}
struct GSlots {
    G<NodeRec>* rec;
    G<int32_t>* q_s;
    G<int32_t>* q_t;
    G<int32_t>* q_d;
    G<int32_t>* tls;
    int64_t stride;
    G<uint32_t>* bm;
    int64_t words;
    G<DagArc>* arcs;
    int32_t acap;
    G<CRec>* crec;
    G<uint32_t>* mlx;
    int32_t mlxcap;
};
__device__ __forceinline__ GSlots sview(const DevSlots& s) {
    return GSlots{gptr(s.rec), gptr(s.q_s), gptr(s.q_t), gptr(s.q_d), gptr(s.tls), s.stride,
                  gptr(s.bm),  s.words,     gptr(s.arcs), s.acap,       gptr(s.crec), gptr(s.mlx), s.mlxcap};
}

// Bitmap operations on one plane of a slot's device bitmaps.
struct Bits {
    __device__ __forceinline__ static uint32_t rd(G<uint32_t>* p, int32_t w) {
        return __hip_atomic_load(p + (w >> 5), __ATOMIC_RELAXED, WGS);
    }
    __device__ __forceinline__ static uint32_t set(G<uint32_t>* p, int32_t w) {
        return __hip_atomic_fetch_or(p + (w >> 5), 1u << (w & 31), __ATOMIC_RELAXED, WGS);
    }
    __device__ __forceinline__ static bool test(uint32_t word, int32_t w) { return (word >> (w & 31)) & 1u; }
    __device__ __forceinline__ static void clear_word(G<uint32_t>* p, int32_t w) {
        __hip_atomic_store(p + (w >> 5), 0u, __ATOMIC_RELAXED, WGS);
    }
};

// A slot's node records. Per-node slots (CMP = false) index them by node id;
// compact slots (CMP = true) by the node's position p in its side's LDS
// table, one record per side. Every accessor takes both; the unused one is
// dropped by the compiler.
template <bool CMP>
struct Recs {
    G<NodeRec>* R;   // per-node slots: this slot's records
    G<CRec>* C;      // compact slots: this slot's [2][table size] records (sizes are defined below)
    template <int SIDE>
    __device__ __forceinline__ G<uint32_t>* lv(int32_t x, int p) const;
    template <int SIDE>
    __device__ __forceinline__ G<uint64_t>* sg(int32_t x, int p) const;
    __device__ __forceinline__ G<uint64_t>* ws(int side, int32_t x, int p) const;
    __device__ __forceinline__ void lv_ws(int side, int32_t x, int p, uint32_t& lv, uint64_t& w) const;
    __device__ __forceinline__ void clear(int side, int32_t x, int p) const;
};

// Visited sets of a sample's two balls.
// LDS = false: one bitmap plane per side in the slot's device memory.
// LDS = true: an exact open-addressing hash table per side in LDS (node id + 1,
// 0 = empty, linear probing), small because a sample's balls are small once
// the last level keeps only its meeting layer. A side whose table would fill
// up is spilled to its device bitmap plane (every node of the side is in its
// queue) and uses the bitmap from then on.
#ifndef PERCIS_HBITS
#define PERCIS_HBITS 10
#endif
// Compact slots may use larger tables: a larger table hands fewer samples
// on to the per-node slots, but costs resident samples. R-MAT 24 directed:
// 10 bits 7.2M (10.5 % handed on), 11 bits 7.7M (6.3 %), 12 bits 6.6M
// samples/s (4.5 %).
#ifndef PERCIS_HBITS_COMPACT
#define PERCIS_HBITS_COMPACT 11
#endif
// Per-node slots of 512 threads or more run few workgroups per CU (the
// samples compact slots hand on, and small launches), so their tables can be
// larger: a side then stays in LDS up to 3/4 of 2^HBITS_WIDE nodes.
#ifndef PERCIS_HBITS_WIDE
#define PERCIS_HBITS_WIDE 13
#endif
constexpr int HBITS = PERCIS_HBITS;           // per-node slots
constexpr int HBITS_C = PERCIS_HBITS_COMPACT; // compact slots
constexpr int HBITS_W = PERCIS_HBITS_WIDE;    // per-node slots of 512 threads or more
template <int TB>
struct Tab {
    static constexpr int CAP = 1 << TB;          // table slots per side
    static constexpr int LIMIT = 3 * CAP / 4;    // most entries a table takes
    static constexpr int ADMIT = 5 * CAP / 8;    // a level decides first visits by the table if it cannot add more
};
// Table bits of a sampler build (threads per sample, compact slots or not).
template <int BSZ, bool CMP>
constexpr int tbits() { return CMP ? HBITS_C : (BSZ >= 512 ? HBITS_W : HBITS); }
constexpr int table_bits(int block, bool compact) { return compact ? HBITS_C : (block >= 512 ? HBITS_W : HBITS); }
constexpr int HCAP = Tab<HBITS>::CAP;         // per-node slots' table
constexpr int CCAP = Tab<HBITS_C>::CAP;       // compact slots' table (records per side)

// Level word of x on side SIDE.
template <bool CMP>
template <int SIDE>
__device__ __forceinline__ G<uint32_t>* Recs<CMP>::lv(int32_t x, int p) const {
    if constexpr (CMP) return &C[SIDE * CCAP + p].lv;
    else return SIDE ? &R[x].lv_t : &R[x].lv_s;
}
// The side's own shortest-path count of x (sigma_s on the s side, sigma_t on
// the t side).
template <bool CMP>
template <int SIDE>
__device__ __forceinline__ G<uint64_t>* Recs<CMP>::sg(int32_t x, int p) const {
    if constexpr (CMP) return SIDE ? &C[CCAP + p].wt : &C[p].ws;
    else return SIDE ? &R[x].sg_t : &R[x].sg_s;
}
// sigma_s of x as the sweep and the walk read it, from side `side`'s record
// (per-node slots have one field for both).
template <bool CMP>
__device__ __forceinline__ G<uint64_t>* Recs<CMP>::ws(int side, int32_t x, int p) const {
    if constexpr (CMP) return &C[side * CCAP + p].ws;
    else return &R[x].sg_s;
}
// Level on side `side` and sigma_s of x in one 16-byte load.
template <bool CMP>
__device__ __forceinline__ void Recs<CMP>::lv_ws(int side, int32_t x, int p, uint32_t& lvw, uint64_t& w) const {
    if constexpr (CMP) {
        const u32x4 v = *reinterpret_cast<const G<u32x4>*>(&C[side * CCAP + p]);
        lvw = v.x;
        w = ((uint64_t)v.w << 32) | v.z;
    } else {
        const u32x4 v = *reinterpret_cast<const G<u32x4>*>(&R[x]);
        lvw = side ? v.y : v.x;
        w = ((uint64_t)v.w << 32) | v.z;
    }
}
// Zeroes x's record (per-node slots: both sides at once).
template <bool CMP>
__device__ __forceinline__ void Recs<CMP>::clear(int side, int32_t x, int p) const {
    G<u32x4>* z = CMP ? reinterpret_cast<G<u32x4>*>(&C[side * CCAP + p]) : reinterpret_cast<G<u32x4>*>(&R[x]);
    z[0] = u32x4{0u, 0u, 0u, 0u};
    z[1] = u32x4{0u, 0u, 0u, 0u};
}
template <bool LDS>
struct Vis {
    G<uint32_t>* bm[2];   // device bitmap planes
};

// The two LDS tables (LDS = true) lie in the workgroup's dynamic LDS, side 0
// first; they are addressed from the array itself so that the compiler keeps
// their accesses in LDS.
extern __shared__ uint32_t dyn_lds[];
template <int TB>
__device__ __forceinline__ uint32_t* tab(int side) { return dyn_lds + side * Tab<TB>::CAP; }

template <int TB>
__device__ __forceinline__ uint32_t hslot(int32_t x) { return ((uint32_t)x * 0x9E3779B1u) >> (32 - TB); }

// Position of x in table T, or -1.
template <int TB>
__device__ __forceinline__ int table_find(uint32_t* T, int32_t x) {
    const uint32_t key = (uint32_t)x + 1;
    for (uint32_t i = hslot<TB>(x);; i = (i + 1) & (Tab<TB>::CAP - 1)) {
        const uint32_t v = __hip_atomic_load(T + i, __ATOMIC_RELAXED, WGS);
        if (v == key) return (int)i;
        if (v == 0) return -1;
    }
}
template <int TB>
__device__ __forceinline__ bool table_has(uint32_t* T, int32_t x) { return table_find<TB>(T, x) >= 0; }

// Inserts x, known to be absent and inserted by this thread only; returns
// its position, or -1 if the table is full (it then stays without x).
template <int TB>
__device__ __forceinline__ int table_put(uint32_t* T, int32_t* cnt, int32_t x) {
    if (atomicAdd(cnt, 1) >= Tab<TB>::LIMIT) return -1;
    const uint32_t key = (uint32_t)x + 1;
    for (uint32_t i = hslot<TB>(x);; i = (i + 1) & (Tab<TB>::CAP - 1)) {
        uint32_t expect = 0;
        if (__hip_atomic_compare_exchange_strong(T + i, &expect, key, __ATOMIC_RELAXED, __ATOMIC_RELAXED, WGS))
            return (int)i;
    }
}

// Finds or inserts x with a bounded table: returns x's position, *fresh
// telling whether this call inserted it, or -1 when an insert would take the
// table past its entry limit (a reservation is taken before each insert
// try, so the table never holds more). The caller gives the sample up on -1.
template <int TB>
__device__ __forceinline__ int table_visit_bounded(uint32_t* T, int32_t* cnt, int32_t x, bool* fresh) {
    const uint32_t key = (uint32_t)x + 1;
    *fresh = false;
    for (uint32_t i = hslot<TB>(x);; i = (i + 1) & (Tab<TB>::CAP - 1)) {
        uint32_t v = __hip_atomic_load(T + i, __ATOMIC_RELAXED, WGS);
        if (v == 0) {
            if (atomicAdd(cnt, 1) >= Tab<TB>::LIMIT) return -1;
            uint32_t expect = 0;
            if (__hip_atomic_compare_exchange_strong(T + i, &expect, key, __ATOMIC_RELAXED, __ATOMIC_RELAXED, WGS)) {
                *fresh = true;
                return (int)i;
            }
            v = expect;
        }
        if (v == key) return (int)i;
    }
}

// Finds or inserts x; true iff this call inserted it. The caller guarantees
// room (fewer than Tab<TB>::CAP entries after every possible insert).
// Per-node slots.
template <int TB>
__device__ __forceinline__ bool table_visit(uint32_t* T, int32_t* cnt, int32_t x) {
    const uint32_t key = (uint32_t)x + 1;
    for (uint32_t i = hslot<TB>(x);; i = (i + 1) & (Tab<TB>::CAP - 1)) {
        uint32_t v = __hip_atomic_load(T + i, __ATOMIC_RELAXED, WGS);
        if (v == 0) {
            uint32_t expect = 0;
            if (__hip_atomic_compare_exchange_strong(T + i, &expect, key, __ATOMIC_RELAXED, __ATOMIC_RELAXED, WGS)) {
                atomicAdd(cnt, 1);
                return true;
            }
            v = expect;
        }
        if (v == key) return false;
    }
}

// Lane l's value as a wave-uniform (scalar) value; l must be wave-uniform.
// Values that steer a wave's control flow are taken this way rather than by
// a shuffle: the compiler cannot see that a shuffled value is the same in
// every lane, and may then split a loop so that lanes run different
// iterations (one lane leaving to do its own work while the others wait in
// an inner copy of the loop).
__device__ __forceinline__ int32_t lane_i32(int32_t v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ uint64_t lane_u64(uint64_t v, int l) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

// ---------------------------------------------------------------- Philox
__device__ __forceinline__ uint64_t philox_word0(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                                 uint64_t k0, uint64_t k1) {
#pragma unroll
    for (int i = 0; i < 10; i++) {
        const uint64_t m0 = 0xD2E7470EE14C6C93ull, m1 = 0xCA5A826395121157ull;
        uint64_t hi0 = __umul64hi(m0, c0), lo0 = m0 * c0;
        uint64_t hi1 = __umul64hi(m1, c2), lo1 = m1 * c2;
        uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
    return c0;
}

// Uniform integer in [0, N), N >= 1, exactly (Lemire 2019).
__device__ uint64_t draw_bounded(uint64_t seed, uint64_t phase, uint64_t idx, uint64_t variate, uint64_t N) {
    for (uint64_t attempt = 0;; attempt++) {
        uint64_t x = philox_word0(idx, variate, attempt, 0, seed, phase);
        uint64_t lo = x * N;
        if (lo < N) {
            uint64_t thr = (0 - N) % N;
            if (lo < thr) continue;
        }
        return __umul64hi(x, N);
    }
}

// Smallest d in [lo, hi] with pred(d), for a monotone pred with pred(hi)
// true (one lane).
template <class Pred>
__device__ __forceinline__ int32_t lane_search(int32_t lo, int32_t hi, Pred pred) {
    while (lo < hi) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if (pred(mid)) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// ------------------------------------------------------------ workgroup state
struct SampleShared {
    int32_t node[CH];
    int32_t npos[CH];     // compact slots: the staged node's position in its side's table
    int32_t beg[CH];
    int32_t off[CH];
    uint64_t sig[CH];
    uint8_t of[CH];
    int32_t wsum[16];
    int32_t s, t;
    int32_t lo_s, hi_s, lo_t, hi_t;
    int32_t a, b;
    unsigned long long deg_s, deg_t, deg_next;       // frontier degree sums
    unsigned long long deg_t_prev;                   // in-degree sum of t-level b - 1
    unsigned long long push_cost;                    // out-degree sum of the meeting layer
    unsigned long long mass_next;                    // sum of the counts of the level being built
    uint32_t wide_s, wide_t, wide_next;              // a frontier's counts may sum to 2^64 or more
    int32_t tail, tail_s, tail_t;
    int32_t nmeet;
    int32_t level_meets;  // the level being built has an arc into the other ball
    int32_t mcnt;         // arcs into the other ball found by a chunk's first pass
    int32_t ml_w[MLCAP];  // those arcs: head node, and staged tail | (head's position in the other table + 1) << 8
    int32_t ml_m[MLCAP];
    int32_t narcs;        // DAG arcs recorded by this sample (may exceed the slot's capacity)
    // The arcs into the nodes at distance q from s are recorded by one stage
    // of the search (the s-side level q, or the t-side step into that
    // distance), so they lie in arcs[seg_lo[q], seg_hi[q]) (seg_hi = -1:
    // not kept, q >= SEGCAP or no such stage yet).
    int32_t seg_lo[SEGCAP], seg_hi[SEGCAP];
    int32_t wk_u[KCAP];   // predecessors of the walk's current node, and their sigma_s
    uint64_t wk_w[KCAP];
    int32_t level_table;  // the level being built decides first visits by its side's table
    int32_t hcnt[2];      // entries reserved in each side's table
    int32_t spilled[2];   // the side's visited set lives in its device bitmap
    int32_t spill_req[2]; // the side's table overflowed in the level being built
    int32_t status;   // 0 running, 1 met, 2 unreachable, 3 given up (outgrew a compact slot)
    int32_t abort;    // a table of a compact slot is full
    int32_t side;     // side of the level being built
    int32_t ovf;
    int32_t walk_err;
    uint64_t sigma;
    // the next sample, claimed and drawn by one wave ahead of time
    unsigned long long nx_idx;
    int32_t nx_ok, nx_task, nx_s, nx_t;
    unsigned long long phase_ticks[5];  // start, BFS, meeting + DAG, walk (+ next pair), clearing
    unsigned long long spills;          // samples of this workgroup that spilled a side
    unsigned long long deferred;        // samples this compact workgroup handed on
    unsigned long long walk_errs;       // samples whose walk found no predecessor at some step
    // per-sample statistics of one task, summed here by thread 0 and added to
    // the task's counters when the workgroup moves to another task
    unsigned long long acc_samples, acc_reach, acc_sum_I, acc_sum_I2, acc_ovf, acc_first;
    int32_t acc_task;
    uint32_t balance;     // side rule of plan_level (SampleLaunch::balance)
};

// Is x in side `side`'s ball? Exact.
template <bool LDS, int TB>
__device__ __forceinline__ bool member(const Vis<LDS>& V, const SampleShared& sh, int side, int32_t x) {
    if (!LDS || sh.spilled[side]) return Bits::test(Bits::rd(V.bm[side], x), x);
    return table_has<TB>(tab<TB>(side), x);
}

// Records the DAG arc tail -> head weighed by sigma_s(tail) = w; arcs past the
// slot's capacity are dropped (the walk then scans in-rows instead).
__device__ __forceinline__ void record_arc(G<DagArc>* arcs, int32_t acap, SampleShared& sh, int32_t tail, int32_t head,
                                           uint64_t w) {
    const int i = atomicAdd(&sh.narcs, 1);
    if (i < acap)
        *reinterpret_cast<G<u32x4>*>(arcs + i) = u32x4{(uint32_t)tail, (uint32_t)head, (uint32_t)w, (uint32_t)(w >> 32)};
}

// Thread 0 only.
__device__ void flush_task_stats(SampleShared& sh, const SampleLaunch& L) {
    if (sh.acc_task >= 0) {
        DevStats* st = L.tasks[sh.acc_task].stats;
        atomicAdd(&st->samples, sh.acc_samples);
        if (sh.acc_reach) atomicAdd(&st->reachable, sh.acc_reach);
        if (sh.acc_sum_I) {
            atomicAdd(&st->sum_I, sh.acc_sum_I);
            atomicAdd(&st->sum_I2, sh.acc_sum_I2);
        }
        if (sh.acc_ovf) {
            atomicAdd(&st->overflow, sh.acc_ovf);
            atomicMin(&st->first_overflow, sh.acc_first);
        }
    }
    sh.acc_samples = sh.acc_reach = sh.acc_sum_I = sh.acc_sum_I2 = sh.acc_ovf = 0;
    sh.acc_first = ~0ull;
}

struct Counters {
    unsigned long long E, A, V, Vd;
};

// Exclusive scan over the first chunk_len<BSZ>() threads (the chunk); every
// thread of the block must call it.
template <int BSZ>
__device__ __forceinline__ int chunk_excl_scan(int v, int32_t* wsum, int& total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    constexpr int NW = chunk_len<BSZ>() / 64;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63 && wid < NW) wsum[wid] = x;
    __syncthreads();
    int pre = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NW; i++) {
        int s = wsum[i];
        if (i < wid) pre += s;
        tot += s;
    }
    total = tot;
    return pre + x - v;
}

__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint64_t y = __shfl_up(v, o, 64);
        if (lane >= o) v += y;
    }
    return v;
}

// Stages up to chunk_len<BSZ>() frontier nodes q[base, base+cnt) of side SIDE in LDS: row
// start, degree prefix sum, shortest-path count and overflow flag of each;
// returns the number of adjacency entries of the chunk. Every thread must
// call it.
template <int BSZ, int SIDE, bool CMP>
__device__ __forceinline__ int stage_chunk(G<int32_t>* q, int base, int cnt, const G<int32_t>* rp,
                                           const Recs<CMP>& rc, bool read_ovf, SampleShared& sh, Counters& cn) {
    const int tid = threadIdx.x;
    int deg = 0, beg = 0;
    int32_t u = 0;
    int p = 0;
    uint64_t su = 0;
    uint32_t of = 0;
    if (tid < cnt) {
        const int32_t e = ldq(q + base + tid);
        if constexpr (CMP) {
            p = e;  // compact slots queue table positions
            u = (int32_t)tab<HBITS_C>(SIDE)[p] - 1;
        } else {
            u = e;
        }
        beg = rp[u];
        deg = rp[u + 1] - beg;
        su = ld64(rc.template sg<SIDE>(u, p));
        if (read_ovf) of = (ld32(rc.template lv<SIDE>(u, p)) & OVFBIT) ? 1 : 0;
        cn.V++;
    }
    int total;
    const int ex = chunk_excl_scan<BSZ>(deg, sh.wsum, total);
    if (tid < chunk_len<BSZ>()) {
        sh.node[tid] = u;
        if constexpr (CMP) sh.npos[tid] = p;
        sh.beg[tid] = beg;
        sh.off[tid] = ex;
        sh.sig[tid] = su;
        sh.of[tid] = (uint8_t)of;
    }
    __syncthreads();
    return total;
}

// Index j of the staged node whose row holds the e-th entry of the chunk.
__device__ __forceinline__ int chunk_owner(const SampleShared& sh, int cnt, int e) {
    int l2 = 0, h2 = cnt - 1;
    while (l2 < h2) {
        const int mid = (l2 + h2 + 1) >> 1;
        if (sh.off[mid] <= e) l2 = mid; else h2 = mid - 1;
    }
    return l2;
}

// chunk_owner searched from `from`, an index whose row starts at or before e
// (the owner of an earlier entry of the same thread: a thread's entries
// increase). A long row keeps its owner for many entries, so the first test
// usually settles it; otherwise a galloping search brackets the owner and a
// bisection finds it. Compact slots use it (measured: their pass 340 ->
// 309 ms on directed R-MAT 24; the per-node slots' 512-thread pass lost more,
// 272 -> 305 ms, so they keep the plain bisection).
__device__ __forceinline__ int chunk_owner_from(const SampleShared& sh, int cnt, int e, int from) {
    int l2 = from, h2 = cnt - 1;
    if (l2 >= h2 || sh.off[l2 + 1] > e) return l2;
    for (int step = 1;; step <<= 1) {
        const int nx = l2 + step;
        if (nx >= h2) break;
        if (sh.off[nx + 1] > e) {
            h2 = nx;
            break;
        }
        l2 = nx + 1;
    }
    while (l2 < h2) {
        const int mid = (l2 + h2 + 1) >> 1;
        if (sh.off[mid] <= e) l2 = mid; else h2 = mid - 1;
    }
    return l2;
}

// The owner of entry e: incrementally (INC, with the thread's last owner in
// hint) or by bisection.
template <bool INC>
__device__ __forceinline__ int owner_of(const SampleShared& sh, int cnt, int e, int& hint) {
    if constexpr (INC) return hint = chunk_owner_from(sh, cnt, e, hint);
    else return chunk_owner(sh, cnt, e);
}

// Sum of a 64-bit value over the wave, with a flag that is set when the sum
// (or any lane's flag) wrapped.
__device__ __forceinline__ void wave_sum_wrap(uint64_t& v, uint32_t& wrap) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t ov = __shfl_xor(v, o, 64);
        const uint32_t ow = __shfl_xor(wrap, o, 64);
        const uint64_t nv = v + ov;
        wrap |= ow | (nv < v ? 1u : 0u);
        v = nv;
    }
}

// The adjacency entries b0 + tid + k * BSZ (k < UNROLL) of a staged chunk
// with `total` entries over `cnt` nodes: the staged tail jj[k] (-1 past the
// end) and the head w[k].
template <int BSZ, bool INC, int U>
__device__ __forceinline__ void fetch_batch(const G<int32_t>* col, const SampleShared& sh, int b0, int total, int cnt,
                                            int32_t (&w)[U], int (&jj)[U], int& hint) {
#pragma unroll
    for (int k = 0; k < U; k++) {
        const int e = b0 + threadIdx.x + k * BSZ;
        jj[k] = -1;
        w[k] = 0;
        if (e < total) {
            jj[k] = owner_of<INC>(sh, cnt, e, hint);
            w[k] = col[sh.beg[jj[k]] + (e - sh.off[jj[k]])];
        }
    }
}

// Member tests of a batch against the other side's ball (side OTHER); bit k
// of the result is set when w[k] is in it, at position po[k] of its table
// (compact slots).
template <int OTHER, bool LDS, bool CMP, int TB, int U>
__device__ __forceinline__ uint32_t probe_batch(const Vis<LDS>& V, const SampleShared& sh, const int32_t (&w)[U],
                                                const int (&jj)[U], int (&po)[U]) {
    uint32_t into = 0;
#pragma unroll
    for (int k = 0; k < U; k++) {
        po[k] = -1;
        if (jj[k] < 0) continue;
        if constexpr (CMP) {
            po[k] = table_find<HBITS_C>(tab<HBITS_C>(OTHER), w[k]);
            if (po[k] >= 0) into |= 1u << k;
        } else if (member<LDS, TB>(V, sh, OTHER, w[k])) {
            into |= 1u << k;
        }
    }
    return into;
}

// One BFS level over the frontier q[lo, hi) of one side (SIDE 0: s, out-arcs;
// SIDE 1: t, in-arcs), edge-balanced: the rows of a chunk of frontier nodes are
// concatenated and the workgroup strides over the concatenation, UNROLL
// entries per thread at a time so that their loads overlap. An arc (u, w)
// adds sigma(u) to w iff w is reached in this level: either its visited bit
// was clear when the arc looked (whoever sets the bit first appends w to the
// queue and writes its level), or w's level field reads 0 (set visited in this
// level, level not written yet) or the new level. Nodes of earlier levels
// carry their own nonzero level, written before the last barrier. New nodes
// that the other side has reached form the meeting layer, written to the
// head of q_d.
// A level with an arc into the other ball is the last one, and of its new
// nodes only the meeting layer is used again, so such a level processes only
// the arcs into the other ball. A chunk of one batch decides this after its
// member tests (one barrier). A longer chunk first scans all its entries for
// such arcs without barriers and lists them in LDS; its second pass then takes
// the list (the last level), or every entry again from the rows just read (a
// level that does not meet), or, past the list's capacity, the entries again,
// keeping those into the other ball.
// Every count of the new level is at most the sum of the frontier's counts
// (no parallel arcs), so the adds are checked for wrapping (`careful`) only
// when that sum reached 2^64. The level's own sum and degree sum (the
// degrees its expansion will scan) are gathered on the way.
template <int SIDE, int BSZ, bool LDS, bool CMP>
__device__ __forceinline__ void expand_bfs(const GGraph& g, const GSlots& sl, int64_t so, const Vis<LDS>& V, const Recs<CMP>& rc,
                           int lo, int hi, uint32_t nl, bool careful, SampleShared& sh, Counters& cn) {
    using B = Bits;
    constexpr int TB = tbits<BSZ, CMP>();
    const int tid = threadIdx.x;
    const bool by_table = LDS && sh.level_table;   // else: bitmap (device mode) or record CAS (LDS mode)
    G<DagArc>* arcs = sl.arcs + (int64_t)blockIdx.x * sl.acap;
    G<uint32_t>* mlx = sl.mlx + (int64_t)blockIdx.x * sl.mlxcap * 2;
    const G<int32_t>* rp = SIDE ? g.irp : g.rp;
    const G<int32_t>* col = SIDE ? g.icol : g.col;
    G<int32_t>* q = (SIDE ? sl.q_t : sl.q_s) + so;
    G<uint32_t>* vis_mine = V.bm[SIDE];
    uint64_t mass = 0, dsum = 0;
    uint32_t wrap = 0;

    constexpr int CHK = chunk_len<BSZ>();
    constexpr int BATCH = BSZ * UNROLL;
    for (int base = lo; base < hi; base += CHK) {
        const int cnt = min(CHK, hi - base);
        if (tid == 0) sh.mcnt = 0;  // ordered before the first pass by stage_chunk's barriers
        const int total = stage_chunk<BSZ, SIDE, CMP>(q, base, cnt, rp, rc, careful, sh, cn);
        const bool single = total <= BATCH;
        bool meets = false, listed = false;
        int n2 = total;  // entries, or listed arcs, of the processing pass
        if (!single) {
            // first pass: list the arcs into the other ball
            int hint = 0;
            for (int b0 = 0; b0 < total; b0 += BSZ * SCAN_UNROLL) {
                int32_t w[SCAN_UNROLL];
                int jj[SCAN_UNROLL], po[SCAN_UNROLL];
                fetch_batch<BSZ, CMP>(col, sh, b0, total, cnt, w, jj, hint);
                const uint32_t in = probe_batch<1 - SIDE, LDS, CMP, TB>(V, sh, w, jj, po);
#pragma unroll
                for (int k = 0; k < SCAN_UNROLL; k++) {
                    if (jj[k] < 0) continue;
                    cn.E++;
                    if ((in >> k) & 1u) {
                        const int i = atomicAdd(&sh.mcnt, 1);
                        const int32_t mk = jj[k] | ((po[k] + 1) << 8);
                        if (i < MLCAP) {
                            sh.ml_w[i] = w[k];
                            sh.ml_m[i] = mk;
                        } else if (i < MLCAP + sl.mlxcap) {
                            *reinterpret_cast<G<u32x2>*>(mlx + 2 * (i - MLCAP)) = u32x2{(uint32_t)w[k], (uint32_t)mk};
                        }
                    }
                }
            }
            __syncthreads();
            // mcnt is final here; level_meets changes only from 0 to 1, and
            // only when mcnt > 0, so every thread makes the same choice
            const int mc = sh.mcnt;
            meets = mc > 0 || sh.level_meets != 0;
            listed = meets && mc <= MLCAP + sl.mlxcap;
            if (listed) n2 = mc;
            if (mc > 0 && tid == 0) sh.level_meets = 1;
        }
        int hint2 = 0;
        for (int b0 = 0; b0 < n2; b0 += BATCH) {
            int32_t w[UNROLL];
            int jj[UNROLL];
            int po[UNROLL];  // compact slots: the arc's head in the other side's table
            uint32_t into_other = 0;  // bit k: arc k ends in the other side's ball
            if (listed) {
#pragma unroll
                for (int k = 0; k < UNROLL; k++) {
                    const int i = b0 + tid + k * BSZ;
                    jj[k] = -1;
                    w[k] = 0;
                    po[k] = -1;
                    if (i < n2) {
                        int32_t m;
                        if (i < MLCAP) {
                            m = sh.ml_m[i];
                            w[k] = sh.ml_w[i];
                        } else {
                            const u32x2 v = *reinterpret_cast<const G<u32x2>*>(mlx + 2 * (i - MLCAP));
                            w[k] = (int32_t)v.x;
                            m = (int32_t)v.y;
                        }
                        jj[k] = m & 255;
                        po[k] = (m >> 8) - 1;
                        into_other |= 1u << k;
                    }
                }
            } else {
                fetch_batch<BSZ, CMP>(col, sh, b0, total, cnt, w, jj, hint2);
                if (single || meets) {
                    into_other = probe_batch<1 - SIDE, LDS, CMP, TB>(V, sh, w, jj, po);
                } else {
#pragma unroll
                    for (int k = 0; k < UNROLL; k++) po[k] = -1;
                }
            }
            if (single) {
                // The flag only goes up within a level, and a later chunk's
                // writers pass this chunk's closing barrier first, so every
                // thread reads the same value.
                if (into_other) sh.level_meets = 1;
                __syncthreads();
                meets = sh.level_meets != 0;
            }
#pragma unroll
            for (int k = 0; k < UNROLL; k++) {
                if (jj[k] < 0) continue;
                if (single) cn.E++;
                if (meets && !((into_other >> k) & 1u)) continue;
                const int32_t x = w[k];
                const int j = jj[k];
                bool add, fresh = false, lv_written = false;
                int p = 0;  // compact slots: x's position in this side's table
                if constexpr (CMP) {
                    // the bounded table decides; a full table gives the sample up
                    p = table_visit_bounded<HBITS_C>(tab<HBITS_C>(SIDE), &sh.hcnt[SIDE], x, &fresh);
                    if (p < 0) {
                        sh.abort = 1;
                        continue;
                    }
                    if (fresh) {
                        add = true;
                    } else {
                        const uint32_t lv = ld32(rc.template lv<SIDE>(x, p)) & LVMASK;
                        add = lv == 0 || lv == nl;
                    }
                } else if (!LDS) {
                    if (!B::test(B::rd(vis_mine, x), x)) {
                        fresh = !B::test(B::set(vis_mine, x), x);
                        add = true;
                    } else {
                        const uint32_t lv = ld32(rc.template lv<SIDE>(x, p)) & LVMASK;
                        add = lv == 0 || lv == nl;
                    }
                } else if (by_table) {
                    fresh = table_visit<TB>(tab<TB>(SIDE), &sh.hcnt[SIDE], x);
                    if (fresh) {
                        add = true;
                    } else {
                        const uint32_t lv = ld32(rc.template lv<SIDE>(x, p)) & LVMASK;
                        add = lv == 0 || lv == nl;
                    }
                } else {
                    // the record's level field decides: 0 = not reached yet
                    uint32_t old = 0;
                    fresh = __hip_atomic_compare_exchange_strong(rc.template lv<SIDE>(x, p), &old, nl,
                                                                 __ATOMIC_RELAXED, __ATOMIC_RELAXED, WGS);
                    add = fresh || (old & LVMASK) == nl;
                    lv_written = true;
                    if (fresh) {
                        if (sh.spilled[SIDE]) (void)B::set(vis_mine, x);
                        else if (table_put<TB>(tab<TB>(SIDE), &sh.hcnt[SIDE], x) < 0) sh.spill_req[SIDE] = 1;
                    }
                }
                if (add) {
                    const uint64_t addv = sh.sig[j];
                    if (careful) {
                        const uint64_t old = add64(rc.template sg<SIDE>(x, p), addv);
                        if (old + addv < old || sh.of[j]) {
                            or32(rc.template lv<SIDE>(x, p), OVFBIT);
                            wrap = 1u;
                        }
                    } else {
                        (void)add64(rc.template sg<SIDE>(x, p), addv);
                    }
                    const uint64_t nm = mass + addv;
                    wrap |= nm < mass ? 1u : 0u;
                    mass = nm;
                    cn.A++;
                    if (SIDE == 0) record_arc(arcs, sl.acap, sh, sh.node[j], x, addv);
                }
                if (SIDE == 1 && ((into_other >> k) & 1u)) {
                    // x is a meeting node (s-level a) and the frontier node, at
                    // t-level b - 1, one of its out-neighbours: this is the
                    // first step of the sigma_s pull, done while the arc is
                    // at hand
                    const uint64_t ss = ld64(rc.ws(0, x, po[k]));
                    (void)add64(rc.ws(1, sh.node[j], CMP ? sh.npos[j] : 0), ss);
                    record_arc(arcs, sl.acap, sh, x, sh.node[j], ss);
                    cn.A++;
                }
                if (fresh) {
                    if (!lv_written) or32(rc.template lv<SIDE>(x, p), nl);
                    const int pos = atomicAdd(&sh.tail, 1);
                    q[pos] = CMP ? p : x;
                    cn.Vd++;
                    dsum += (uint64_t)(rp[x + 1] - rp[x]);
                    if ((into_other >> k) & 1u) {
                        const int mp = atomicAdd(&sh.nmeet, 1);
                        if constexpr (CMP) {
                            // the meeting node's position on each side
                            sl.q_d[2 * so + mp] = SIDE ? po[k] : p;
                            sl.q_d[2 * so + CCAP + mp] = SIDE ? p : po[k];
                        } else {
                            sl.q_d[so + mp] = x;
                        }
                    }
                }
            }
        }
        if (base + CHK < hi) __syncthreads();  // the caller's barrier follows the last chunk
    }
    wave_sum_wrap(mass, wrap);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) dsum += __shfl_xor(dsum, o, 64);
    if ((tid & 63) == 0) {
        const unsigned long long old = atomicAdd(&sh.mass_next, (unsigned long long)mass);
        if (wrap || old + mass < old) sh.wide_next = 1u;
        atomicAdd(&sh.deg_next, (unsigned long long)dsum);
    }
}

// One level of the t-side pull: every node x of q_t[lo, hi) (t-level j - 1)
// adds the sigma_s of its in-neighbours at t-level j (t-level value
// want = j + 1). Counts of nodes off the shortest-path DAG are 0, so only
// DAG arcs add. No count here exceeds sigma_st, known to be below 2^64.
template <int BSZ, bool LDS, bool CMP>
__device__ void pull_level(const GGraph& g, const GSlots& sl, int64_t so, const Vis<LDS>& V, const Recs<CMP>& rc,
                           int lo, int hi, uint32_t want, SampleShared& sh, Counters& cn) {
    const int tid = threadIdx.x;
    G<int32_t>* q = sl.q_t + so;
    G<DagArc>* arcs = sl.arcs + (int64_t)blockIdx.x * sl.acap;
    constexpr int CHK = chunk_len<BSZ>();
    for (int base = lo; base < hi; base += CHK) {
        const int cnt = min(CHK, hi - base);
        int deg = 0, beg = 0;
        int32_t x = 0;
        int px = 0;
        if (tid < cnt) {
            const int32_t e = ldq(q + base + tid);
            if constexpr (CMP) {
                px = e;
                x = (int32_t)tab<HBITS_C>(1)[px] - 1;
            } else {
                x = e;
            }
            beg = g.irp[x];
            deg = g.irp[x + 1] - beg;
            cn.V++;
        }
        int total;
        const int ex = chunk_excl_scan<BSZ>(deg, sh.wsum, total);
        if (tid < CHK) {
            sh.beg[tid] = beg;
            sh.off[tid] = ex;
            sh.sig[tid] = (uint64_t)(uint32_t)x;
            if constexpr (CMP) sh.npos[tid] = px;
        }
        __syncthreads();
        int hint = 0;
        for (int e = tid; e < total; e += BSZ) {
            const int j = owner_of<CMP>(sh, cnt, e, hint);
            const int32_t u = g.icol[sh.beg[j] + (e - sh.off[j])];
            cn.E++;
            int pu = 0;
            if constexpr (CMP) {
                pu = table_find<HBITS_C>(tab<HBITS_C>(1), u);
                if (pu < 0) continue;
            } else if (!member<LDS, tbits<BSZ, CMP>()>(V, sh, 1, u)) {
                continue;
            }
            // levels of this level's nodes are final (set before the last
            // barrier); their sigma_s was completed by the previous pull level
            uint32_t lvu;
            uint64_t su;
            rc.lv_ws(1, u, pu, lvu, su);
            if ((lvu & LVMASK) != want) continue;
            if (su) {
                const int32_t xj = (int32_t)sh.sig[j];
                (void)add64(rc.ws(1, xj, CMP ? sh.npos[j] : 0), su);
                record_arc(arcs, sl.acap, sh, u, xj, su);
                cn.A++;
            }
        }
        if (base + CHK < hi) __syncthreads();
    }
}

// First step of the sigma_s pull done as a push instead (when the s side
// expanded last and the meeting layer's out-rows are shorter than the in-rows
// of t-level b - 1): every meeting node w adds sigma_s(w) to its
// out-neighbours at t-level b - 1 (t-level value want = b).
template <int BSZ, bool LDS, bool CMP>
__device__ void push_meeting(const GGraph& g, const GSlots& sl, int64_t so, const Vis<LDS>& V, const Recs<CMP>& rc,
                             int nmeet, uint32_t want, SampleShared& sh, Counters& cn) {
    const int tid = threadIdx.x;
    G<int32_t>* qd = sl.q_d + (CMP ? 2 * so : so);  // compact: the meeting nodes' s positions
    G<DagArc>* arcs = sl.arcs + (int64_t)blockIdx.x * sl.acap;
    constexpr int CHK = chunk_len<BSZ>();
    for (int base = 0; base < nmeet; base += CHK) {
        const int cnt = min(CHK, nmeet - base);
        const int total = stage_chunk<BSZ, 0, CMP>(qd, base, cnt, g.rp, rc, false, sh, cn);
        int hint = 0;
        for (int e = tid; e < total; e += BSZ) {
            const int j = owner_of<CMP>(sh, cnt, e, hint);
            const int32_t x = g.col[sh.beg[j] + (e - sh.off[j])];
            cn.E++;
            int px = 0;
            if constexpr (CMP) {
                px = table_find<HBITS_C>(tab<HBITS_C>(1), x);
                if (px < 0) continue;
            } else if (!member<LDS, tbits<BSZ, CMP>()>(V, sh, 1, x)) {
                continue;
            }
            if ((ld32(rc.template lv<1>(x, px)) & LVMASK) != want) continue;
            (void)add64(rc.ws(1, x, px), sh.sig[j]);
            record_arc(arcs, sl.acap, sh, sh.node[j], x, sh.sig[j]);
            cn.A++;
        }
        if (base + CHK < nmeet) __syncthreads();
    }
}

// One step of the canonical walk with kc > KCAP predecessors, the arcs into
// w among arcs[a_lo, a_hi): lists them in xb[0, kc) as (internal id, caller
// id, sigma_s low, high), then finds the predecessor of smallest caller id
// whose cumulative sigma_s in caller id order exceeds r by radix selection
// on the caller ids (below 2^25, digits of 7 + 6 + 6 + 6 bits): each round
// sums sigma_s per digit value over the entries with the digits fixed so far
// (histogram in LDS) and fixes the digit where the cumulative sum passes r.
// Subtracts from r the sigma_s of the predecessors passed over. One wave;
// returns -1 if r is not below the total. Kept out of line so that the
// sampler's main body does not carry its registers.
__device__ __noinline__ int32_t walk_select_radix(const G<DagArc>* arcs, int32_t a_lo, int32_t a_hi, int32_t w,
                                                  const G<int32_t>* orig, G<u32x4>* xb, int kc, uint64_t& r,
                                                  uint64_t* hist) {
    const int lane = (int)(threadIdx.x & 63);
    const unsigned long long below = (1ull << lane) - 1;
    int n = 0;
    for (int base = a_lo; base < a_hi; base += 64) {
        const int i = base + lane;
        bool m = false;
        u32x4 av = u32x4{0u, 0u, 0u, 0u};
        if (i < a_hi) {
            av = *reinterpret_cast<const G<u32x4>*>(arcs + i);
            m = (int32_t)av.y == w;
        }
        const unsigned long long bal = __ballot(m);
        const int pos = n + __popcll(bal & below);
        if (m && pos < kc) xb[pos] = u32x4{av.x, (uint32_t)orig[(int32_t)av.x], av.z, av.w};
        n += __popcll(bal);
    }
    if (n != kc) return -1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    uint32_t prefix = 0;
    int hi = 25;
    for (int d = 0; d < 4; d++) {
        const int nb = d == 0 ? 7 : 6, lo = hi - nb, nbk = 1 << nb;
        for (int b = lane; b < nbk; b += 64) hist[b] = 0;
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        for (int i = lane; i < kc; i += 64) {
            const u32x4 e = xb[i];
            if ((e.y >> hi) == prefix)
                atomicAdd((unsigned long long*)&hist[(e.y >> lo) & (nbk - 1)], ((unsigned long long)e.w << 32) | e.z);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        const uint64_t b0 = 2 * lane < nbk ? hist[2 * lane] : 0;
        const uint64_t b1 = 2 * lane + 1 < nbk ? hist[2 * lane + 1] : 0;
        const uint64_t incl = wave_incl_scan_u64(b0 + b1);
        const unsigned long long over = __ballot(incl > r);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        if (!over) return -1;
        const int l = __ffsll((long long)over) - 1;
        const uint64_t before = lane_u64(incl - b0 - b1, l), first = lane_u64(b0, l);
        const bool upper = r >= before + first;
        r -= upper ? before + first : before;
        prefix = (prefix << nb) | (uint32_t)(2 * l + (upper ? 1 : 0));
        hi = lo;
    }
    for (int base = 0; base < kc; base += 64) {
        const int i = base + lane;
        int32_t u = -1;
        if (i < kc) {
            const u32x4 e = xb[i];
            if (e.y == prefix) u = (int32_t)e.x;
        }
        const unsigned long long f = __ballot(u >= 0);
        if (f) return lane_i32(u, __ffsll((long long)f) - 1);
    }
    return -1;
}

// Next BFS level: the side with the smaller frontier degree sum (Section
// III-B's balanced expansion), its queue's append position, fresh
// accumulators. Called by one thread.
template <int TB>
__device__ __forceinline__ void plan_level(SampleShared& sh) {
    sh.side = (sh.deg_s * 100 <= sh.deg_t * sh.balance) ? 0 : 1;
    sh.tail = sh.side == 0 ? sh.hi_s : sh.hi_t;
    // a level adds at most its frontier degree sum of new nodes
    const unsigned long long deg = sh.side == 0 ? sh.deg_s : sh.deg_t;
    sh.level_table =
        !sh.spilled[sh.side] && (unsigned long long)sh.hcnt[sh.side] + deg <= (unsigned long long)Tab<TB>::ADMIT;
    sh.deg_next = 0;
    sh.mass_next = 0;
    sh.wide_next = 0;
    sh.level_meets = 0;
}

// __syncthreads orders the workgroup's scratch accesses (workgroup-scope
// release/acquire around the barrier).
__device__ __forceinline__ void level_barrier() { __syncthreads(); }

// Lane 0 of the calling wave adds v to *p; every lane gets the previous value
// (wave-uniform). Out of line, so that its lane-0 branch stays inside it and
// a caller's loop keeps all lanes in the same iteration.
__device__ __attribute__((noinline)) unsigned long long wave_fetch_add(unsigned long long* p, unsigned long long v) {
    unsigned long long old = 0;
    if ((threadIdx.x & 63) == 0) old = atomicAdd(p, v);
    return lane_u64(old, 0);
}

// Claims the next listed sample into sh.nx_* (sh.nx_ok = 0 past the end of
// the list). Called by one whole wave; no instruction depends on the lane
// except inside the out-of-line claim.
__device__ void claim_next(const SampleLaunch& L, unsigned long long npairs, SampleShared& sh) {
    const int lane = threadIdx.x & 63;
    const unsigned long long q = wave_fetch_add(L.work, 1ull);
    if (q >= npairs) {
        if (lane == 0) sh.nx_ok = 0;
        return;
    }
    const u32x4 pv = *reinterpret_cast<const G<u32x4>*>(gptr(L.pairs) + q);
    const PairRec rec{pv.x, (int32_t)pv.y, (int32_t)pv.z, (int32_t)pv.w};
    if (lane == 0) {
        sh.nx_ok = 1;
        sh.nx_idx = L.base + rec.q;
        sh.nx_task = rec.task;
        sh.nx_s = rec.s;
        sh.nx_t = rec.t;
    }
}

// One sample on this workgroup's slot, for the pair (s, t) already drawn. With
// a launch given, wave 1 claims and draws the next sample during the walk. In
// debug mode (dbg != nullptr) the path index is given instead of drawn, hits
// are not touched and the path is written to dbg (internal ids).
template <int BSZ, bool LDS, bool CMP>
__device__ __forceinline__ void run_sample(const GGraph& g, const GSlots& sl, int64_t so, const Vis<LDS>& V,
                                           uint64_t idx, const DevTask& T, int32_t s, int32_t t,
                                           const SampleLaunch* next, unsigned long long npairs, uint32_t q_rel,
                                           int32_t task, SampleShared& sh, Counters& cn, DebugOut* dbg,
                                           uint64_t dbg_r, int32_t dbg_cap) {
    using B = Bits;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    constexpr int TB = tbits<BSZ, CMP>();
    const Recs<CMP> rc{CMP ? nullptr : sl.rec + so, CMP ? sl.crec + (int64_t)blockIdx.x * 2 * CCAP : nullptr};
    G<int32_t>* q_s = sl.q_s + so;
    G<int32_t>* q_t = sl.q_t + so;
    G<int32_t>* q_d = sl.q_d + (CMP ? 2 * so : so);  // compact: s positions, then t positions at + CCAP
    G<int32_t>* tls = sl.tls + (int64_t)blockIdx.x * (sl.stride + 2);  // start of each t-level in q_t

    // phase timers (thread 0, constant-rate wall clock)
    unsigned long long tm_prev = 0;
    if (tid == 0) tm_prev = wall_clock64();
    auto phase_mark = [&](int ph) {
        if (tid == 0) {
            const unsigned long long now = wall_clock64();
            sh.phase_ticks[ph] += now - tm_prev;
            tm_prev = now;
        }
    };

    // ---- start both balls
    if (wid == 0) {
        if (lane == 0) {
            sh.s = s;
            sh.t = t;
            sh.nmeet = 0; sh.ovf = 0; sh.walk_err = 0; sh.sigma = 0;
            sh.narcs = 0;
            sh.a = 0; sh.b = 0;
            sh.hcnt[0] = sh.hcnt[1] = 0;
            sh.spilled[0] = sh.spilled[1] = 0;
            sh.spill_req[0] = sh.spill_req[1] = 0;
            sh.abort = 0;
            if (s >= g.n_act || t >= g.n_act) {
                // a node without arcs reaches nothing and is reached by nothing
                sh.status = 2;
                sh.tail_s = 0; sh.tail_t = 0;
            } else {
                sh.status = 0;
                int ps = 0, pt = 0;
                if (LDS) {
                    ps = table_put<TB>(tab<TB>(0), &sh.hcnt[0], s);
                    pt = table_put<TB>(tab<TB>(1), &sh.hcnt[1], t);
                } else {
                    B::set(V.bm[0], s);
                    B::set(V.bm[1], t);
                }
                or32(rc.template lv<0>(s, ps), 1u);
                *rc.template sg<0>(s, ps) = 1;
                q_s[0] = CMP ? ps : s;
                or32(rc.template lv<1>(t, pt), 1u);
                *rc.template sg<1>(t, pt) = 1;
                q_t[0] = CMP ? pt : t;
                tls[0] = 0; tls[1] = 1;
                sh.lo_s = 0; sh.hi_s = 1; sh.lo_t = 0; sh.hi_t = 1;
                sh.deg_s = (unsigned long long)(g.rp[s + 1] - g.rp[s]);
                sh.deg_t = (unsigned long long)(g.irp[t + 1] - g.irp[t]);
                sh.wide_s = 0; sh.wide_t = 0;
                sh.deg_t_prev = 0;
                sh.tail_s = 1; sh.tail_t = 1;
                plan_level<TB>(sh);
            }
        }
    }
    if (tid < SEGCAP) sh.seg_hi[tid] = -1;
    level_barrier();
    phase_mark(0);
    // Thread 0's arc-list position at the last stage boundary. It is read only
    // where no stage records arcs: between the two barriers that close a BFS
    // level, and after a sweep step's closing barrier (the next step records
    // nothing before its staging barrier, which thread 0 must reach too).
    int32_t arc_mark = 0;
    auto close_segment = [&](int32_t q) {
        if (tid == 0) {
            const int32_t hi = sh.narcs;
            if (q >= 1 && q < SEGCAP) {
                sh.seg_lo[q] = arc_mark;
                sh.seg_hi[q] = hi;
            }
            arc_mark = hi;
        }
    };

    // ---- balanced bidirectional BFS
    // Thread 0 plans each level (side, append position, fresh accumulators)
    // inside the previous level's last barrier.
    while (sh.status == 0) {
        const int side = sh.side;
        const int nlo = side == 0 ? sh.hi_s : sh.hi_t;
        const bool careful = (side == 0 ? sh.wide_s : sh.wide_t) != 0;
        if (side == 0)
            expand_bfs<0, BSZ, LDS, CMP>(g, sl, so, V, rc, sh.lo_s, sh.hi_s, (uint32_t)sh.a + 2, careful, sh, cn);
        else
            expand_bfs<1, BSZ, LDS, CMP>(g, sl, so, V, rc, sh.lo_t, sh.hi_t, (uint32_t)sh.b + 2, careful, sh, cn);
        level_barrier();
        const int nhi = sh.tail;
        if (!CMP && LDS && sh.spill_req[side]) {
            // the side's table overflowed: its whole ball (its queue) moves to
            // the device bitmap, which answers for the side from now on
            G<int32_t>* qq = side == 0 ? q_s : q_t;
            for (int i = tid; i < nhi; i += BSZ) (void)B::set(V.bm[side], ldq(qq + i));
            __syncthreads();
            if (tid == 0) {
                sh.spilled[side] = 1;
                sh.spill_req[side] = 0;
            }
        }
        // the arcs of this level: into s-level a + 1, or (the t side's meeting
        // level, the first sweep step) into the distance a + 1 from s
        if (side == 0 || sh.nmeet > 0) close_segment(sh.a + 1);
        if (tid == 0) {
            if (side == 0) {
                sh.lo_s = nlo; sh.hi_s = nhi; sh.tail_s = nhi; sh.a++;
                sh.deg_s = sh.deg_next; sh.wide_s = sh.wide_next;
            } else {
                sh.lo_t = nlo; sh.hi_t = nhi; sh.tail_t = nhi; sh.b++;
                sh.deg_t_prev = sh.deg_t;
                sh.deg_t = sh.deg_next; sh.wide_t = sh.wide_next;
                tls[sh.b + 1] = nhi;
            }
            if (CMP && sh.abort) sh.status = 3;
            else if (sh.nmeet > 0) sh.status = 1;
            else if (nhi == nlo) sh.status = 2;
            else plan_level<TB>(sh);
        }
        level_barrier();
    }

    phase_mark(1);

    // ---- meeting layer: sigma_st with overflow detection
    // After the last level, the meeting layer lies at s-level a and t-level b
    // (whichever side moved), so d(s,t) = a + b.
    const int32_t L = sh.a + sh.b;
    if (sh.status == 1) {
        if (wid == 0) {
            uint64_t acc = 0, pc = 0;
            int of = 0;
            for (int i = lane; i < sh.nmeet; i += 64) {
                int32_t w;
                int ps = 0, pt = 0;
                if constexpr (CMP) {
                    ps = ldq(q_d + i);
                    pt = ldq(q_d + CCAP + i);
                    w = (int32_t)tab<HBITS_C>(0)[ps] - 1;
                } else {
                    w = ldq(q_d + i);
                }
                pc += (uint64_t)(g.rp[w + 1] - g.rp[w]);
                const uint32_t ls = ld32(rc.template lv<0>(w, ps)), lt = ld32(rc.template lv<1>(w, pt));
                of |= ((ls | lt) & OVFBIT) ? 1 : 0;
                const uint64_t x = ld64(rc.template sg<0>(w, ps)), y = ld64(rc.template sg<1>(w, pt));
                if constexpr (CMP) *rc.ws(1, w, pt) = x;  // the t record carries sigma_s for the sweep
                if (__umul64hi(x, y) != 0) of = 1;
                const uint64_t p = x * y;
                const uint64_t na = acc + p;
                if (na < acc) of = 1;
                acc = na;
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const uint64_t oa = __shfl_xor(acc, o, 64);
                const int oo = __shfl_xor(of, o, 64);
                const uint64_t na = acc + oa;
                of |= oo | (na < acc ? 1 : 0);
                acc = na;
                pc += __shfl_xor(pc, o, 64);
            }
            if (lane == 0) {
                sh.sigma = acc;
                sh.ovf = of;
                sh.push_cost = pc;
            }
        }
        level_barrier();

        // ---- sigma_s pulled through the t-ball, from t-level b - 1 down to t
        // If the t side expanded last, its meeting level already did the first
        // step; if the s side did, the first step is a push from the meeting
        // layer when that scans fewer arcs.
        if (!sh.ovf) {
            int j = sh.b;
            if (sh.side == 1) {
                j--;
            } else if (j >= 1 && sh.push_cost < sh.deg_t_prev) {
                push_meeting<BSZ, LDS, CMP>(g, sl, so, V, rc, sh.nmeet, (uint32_t)j, sh, cn);
                level_barrier();
                close_segment(sh.a + 1);
                j--;
            }
            for (; j >= 1; j--) {
                pull_level<BSZ, LDS, CMP>(g, sl, so, V, rc, ldq(tls + j - 1), ldq(tls + j), (uint32_t)j + 1, sh, cn);
                level_barrier();
                close_segment(L - j + 1);  // into t-level j - 1
            }
        }
        phase_mark(2);

        // ---- canonical backward walk by wave 0
        // The predecessors of the current node w are the DAG arcs into w that
        // the search recorded (each with sigma_s of its tail); the walk takes
        // the one of smallest caller id whose cumulative sigma_s, in caller id
        // order, exceeds r. Without a complete arc list (or with more than
        // KCAP predecessors) a step scans w's in-row instead, whose entries
        // are in caller id order: the same choice.
        // (a debug call's path index past sigma_st gets L and sigma_st only)
        if (!sh.ovf && wid == 0 && !(dbg && dbg_r >= sh.sigma)) {
            const int32_t aM = sh.a;
            uint64_t r = dbg ? dbg_r : draw_bounded(T.seed, T.phase, idx, 2, sh.sigma);
            const int32_t na = __builtin_amdgcn_readfirstlane(sh.narcs);
            const G<DagArc>* arcs = sl.arcs + (int64_t)blockIdx.x * sl.acap;
            // a step with more than KCAP predecessors lists them in the slot's
            // device list, free after the search
            G<u32x4>* xb = reinterpret_cast<G<u32x4>*>(sl.mlx + (int64_t)blockIdx.x * sl.mlxcap * 2);
            const int xcap = sl.mlxcap / 2;
            const unsigned long long below = (1ull << lane) - 1;  // lanes under this one
            int32_t w = sh.t;
            int err = 0;
            for (int32_t p = L - 1; p >= 1; p--) {
                const bool on_s = p <= aM;
                int32_t sel = -1;
                int kc = INT32_MAX;  // predecessors in the list (INT32_MAX: no complete list)
                // the arcs into w (at distance p + 1): its stage's segment of the
                // list when kept, else the whole list; usable if none was dropped
                int32_t a_lo = 0, a_hi = na;
                if (p + 1 < SEGCAP) {
                    const int32_t h = __builtin_amdgcn_readfirstlane(sh.seg_hi[p + 1]);
                    if (h >= 0) {
                        a_lo = __builtin_amdgcn_readfirstlane(sh.seg_lo[p + 1]);
                        a_hi = h;
                    }
                }
                if (a_hi <= sl.acap) {
                    kc = 0;
                    for (int base = a_lo; base < a_hi; base += 64 * ARC_UNROLL) {
                        DagArc a[ARC_UNROLL];
                        bool m[ARC_UNROLL];
#pragma unroll
                        for (int k = 0; k < ARC_UNROLL; k++) {
                            const int i = base + k * 64 + lane;
                            m[k] = false;
                            if (i < a_hi) {
                                const u32x4 av = *reinterpret_cast<const G<u32x4>*>(arcs + i);
                                a[k] = DagArc{(int32_t)av.x, (int32_t)av.y, ((uint64_t)av.w << 32) | av.z};
                                m[k] = a[k].head == w;
                            }
                        }
#pragma unroll
                        for (int k = 0; k < ARC_UNROLL; k++) {
                            const unsigned long long bal = __ballot(m[k]);
                            const int pos = kc + __popcll(bal & below);
                            if (m[k] && pos < KCAP) {
                                sh.wk_u[pos] = a[k].tail;
                                sh.wk_w[pos] = a[k].w;
                            }
                            kc += __popcll(bal);
                        }
                    }
                    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                    if (kc == 1) {
                        // one predecessor: it covers every index (no order needed)
                        const int32_t u0 = __builtin_amdgcn_readfirstlane(sh.wk_u[0]);
                        if (lane_u64(sh.wk_w[0], 0) > r) sel = u0;
                    } else if (kc <= KCAP) {
                        // order by caller id: each lane swaps its predecessor's
                        // internal id in the list for the caller's
                        int32_t ui = -1, uo = INT32_MAX;
                        uint64_t wi = 0, ci = 0;  // weight, cumulative weight up to and with uo
                        if (lane < kc) {
                            ui = sh.wk_u[lane];
                            wi = sh.wk_w[lane];
                            uo = g.orig[ui];
                        }
                        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                        if (lane < kc) sh.wk_u[lane] = uo;
                        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                        for (int j = 0; j < kc; j++)
                            if (sh.wk_u[j] <= uo) ci += sh.wk_w[j];
                        const bool cand = lane < kc && ci > r;
                        int32_t best = cand ? uo : INT32_MAX;
#pragma unroll
                        for (int o = 32; o > 0; o >>= 1) best = min(best, __shfl_xor(best, o, 64));
                        best = __builtin_amdgcn_readfirstlane(best);
                        if (best != INT32_MAX) {
                            const unsigned long long hit = __ballot(cand && uo == best);
                            const int l = __ffsll((long long)hit) - 1;
                            r -= lane_u64(ci, l) - lane_u64(wi, l);
                            sel = lane_i32(ui, l);
                        }
                    } else if (kc <= xcap) {
                        sel = walk_select_radix(arcs, a_lo, a_hi, w, g.orig, xb, kc, r, sh.sig);
                    }
                    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                }
                if (kc > xcap) {
                    // in-row scan in caller id order: in-neighbours one level closer
                    // to s (s-level p, or t-level L - p past the meeting layer),
                    // weighed by sigma_s
                    const uint32_t want = on_s ? (uint32_t)p + 1 : (uint32_t)(L - p) + 1;
                    const int32_t beg = lane_i32(g.irp[w], 0), end = lane_i32(g.irp[w + 1], 0);
                    const G<int32_t>* ccol = g.icol + lane_i32(g.irp[g.n], 0);
                    for (int32_t base = beg; base < end && sel < 0; base += 64 * WALK_UNROLL) {
                        int32_t u[WALK_UNROLL];
                        uint64_t wt[WALK_UNROLL];
#pragma unroll
                        for (int k = 0; k < WALK_UNROLL; k++) {
                            const int32_t i = base + k * 64 + lane;
                            u[k] = i < end ? ccol[i] : -1;
                        }
#pragma unroll
                        for (int k = 0; k < WALK_UNROLL; k++) {
                            wt[k] = 0;
                            int pu = 0;
                            bool in_ball = false;
                            if (u[k] >= 0) {
                                if constexpr (CMP) {
                                    pu = table_find<HBITS_C>(tab<HBITS_C>(on_s ? 0 : 1), u[k]);
                                    in_ball = pu >= 0;
                                } else {
                                    in_ball = member<LDS, TB>(V, sh, on_s ? 0 : 1, u[k]);
                                }
                            }
                            if (in_ball) {
                                uint32_t lvu;
                                uint64_t su;
                                rc.lv_ws(on_s ? 0 : 1, u[k], pu, lvu, su);
                                if ((lvu & LVMASK) == want) wt[k] = su;
                            }
                            if (u[k] >= 0) cn.E++;
                        }
#pragma unroll
                        for (int k = 0; k < WALK_UNROLL; k++) {
                            if (sel >= 0) continue;
                            const uint64_t incl = wave_incl_scan_u64(wt[k]);
                            const uint64_t tot = lane_u64(incl, 63);
                            if (r < tot) {
                                const unsigned long long m = __ballot(incl > r);
                                const int l = __ffsll((long long)m) - 1;
                                r -= lane_u64(incl - wt[k], l);
                                sel = lane_i32(u[k], l);
                            } else {
                                r -= tot;
                            }
                        }
                    }
                }
                if (sel < 0) { err = 1; break; }
                w = sel;
                if (lane == 0) {
                    // the path is kept (the meeting layer's queue is free by
                    // now) and credited only once the walk reaches s
                    if (dbg) {
                        if (p < dbg_cap) dbg->path[p] = w;
                    } else {
                        __hip_atomic_store(q_d + p, w, __ATOMIC_RELAXED, WGS);
                    }
                    cn.V++;
                }
            }
            if (lane == 0) sh.walk_err = err;
        }
    }
    // ---- the next sample's pair, by wave 1 while wave 0 walks (a one-wave
    // workgroup claims it after its walk)
    if (next && wid == (BSZ >= 128 ? 1 : 0)) claim_next(*next, npairs, sh);
    __syncthreads();
    // ---- one hit to each internal node of a path the walk completed
    if (!dbg && sh.status == 1 && !sh.ovf && !sh.walk_err) {
        for (int p = 1 + tid; p < L; p += BSZ)
            __hip_atomic_fetch_add(gptr(T.hits) + g.orig[ldq(q_d + p)], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    phase_mark(3);

    // ---- per-sample statistics
    if (tid == 0) {
        if (!dbg) {
            if (sh.status == 3) {
                // outgrew the compact slot: listed for the per-node slots,
                // which count the sample
                const unsigned long long at = atomicAdd(next->nbig, 1ull);
                next->big[at] = PairRec{q_rel, s, t, task};
                sh.deferred++;
            } else {
                sh.acc_samples++;
            }
            if (sh.spilled[0] | sh.spilled[1]) sh.spills++;
            if (sh.status == 1) {
                if (sh.ovf && !sh.walk_err) {
                    // sigma_st >= 2^64: listed for the 128-bit path, which
                    // adds the sample's statistics and hits
                    const unsigned long long at = atomicAdd(next->nwide, 1ull);
                    next->wide[at] = PairRec{q_rel, s, t, task};
                } else if (sh.walk_err) {
                    // no predecessor at some step: a broken invariant of the
                    // search; the sample adds no hits and fails the call
                    sh.walk_errs++;
                } else {
                    const unsigned long long I = (unsigned long long)(L - 1);
                    sh.acc_reach++;
                    sh.acc_sum_I += I;
                    sh.acc_sum_I2 += I * I;
                }
            }
        } else {
            dbg->L = sh.status == 1 ? L : -1;
            dbg->overflow = (sh.status == 1 && (sh.ovf || sh.walk_err)) ? (sh.walk_err ? 2 : 1) : 0;
            dbg->sigma = sh.status == 1 ? (sh.ovf ? ~0ull : sh.sigma) : 0;
            if (sh.status == 1 && L < dbg_cap) {
                dbg->path[0] = sh.s;
                dbg->path[L] = sh.t;
            }
        }
    }

    // ---- clear what this sample touched (every node reached is in q_s or q_t)
    const int ts = sh.tail_s, tt = sh.tail_t;
    const bool bm_s = !LDS || sh.spilled[0], bm_t = !LDS || sh.spilled[1];
    // (queue entries are node ids, or table positions in compact slots)
    for (int i = tid; i < ts; i += BSZ) {
        const int32_t e = ldq(q_s + i);
        rc.clear(0, e, e);
        if (!CMP && bm_s) B::clear_word(V.bm[0], e);
    }
    for (int i = tid; i < tt; i += BSZ) {
        const int32_t e = ldq(q_t + i);
        rc.clear(1, e, e);
        if (!CMP && bm_t) B::clear_word(V.bm[1], e);
    }
    if (LDS) {
        for (int i = tid; i < 2 * Tab<TB>::CAP; i += BSZ) __hip_atomic_store(dyn_lds + i, 0u, __ATOMIC_RELAXED, WGS);
    }
    level_barrier();
    phase_mark(4);
}

__device__ void flush_counters(const Counters& cn, DevStats* st) {
    unsigned long long E = cn.E, A = cn.A, V = cn.V, Vd = cn.Vd;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        E += __shfl_xor(E, o, 64);
        A += __shfl_xor(A, o, 64);
        V += __shfl_xor(V, o, 64);
        Vd += __shfl_xor(Vd, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&st->edges, E);
        atomicAdd(&st->sigma_adds, A);
        atomicAdd(&st->vexp, V);
        atomicAdd(&st->vdisc, Vd);
    }
}

template <int BSZ, bool LDS>
__device__ __forceinline__ Vis<LDS> slot_vis(const GSlots& sl, int slot) {
    Vis<LDS> v;
    G<uint32_t>* base = sl.bm + (int64_t)slot * 2 * sl.words;
    v.bm[0] = base;
    v.bm[1] = base + sl.words;
    return v;
}

// Occupancy target of the sampler (waves per SIMD), a build knob (0 = the
// compiler's choice): the sampler is latency-bound, so samples in flight
// count, but spilled registers cost memory round trips. Measured on R-MAT 18
// (unroll 8): 4 waves 34.5M, 5 waves (96 registers) 36.7M, 6 waves (80) 35.7M,
// 7 waves 28.8M samples/s.
#ifndef PERCIS_SAMPLER_WAVES_PER_EU
#define PERCIS_SAMPLER_WAVES_PER_EU 5
#endif
// A workgroup of 512 threads or more has 8+ waves, so at most 2 fit on a CU
// (4 waves per SIMD) whatever the register budget: those kernels get the
// 4-wave budget (128 VGPRs) instead of spilling at 96.
#if PERCIS_SAMPLER_WAVES_PER_EU > 0
#define SAMPLER_OCCUPANCY \
    __attribute__((amdgpu_waves_per_eu(BSZ >= 512 && PERCIS_SAMPLER_WAVES_PER_EU > 4 ? 4 : PERCIS_SAMPLER_WAVES_PER_EU)))
#else
#define SAMPLER_OCCUPANCY
#endif

// CMP: compact slots (records by table position; a sample that outgrows them
// is listed in L.big for per-node slots).
template <int BSZ, bool LDS, bool CMP>
__global__ __launch_bounds__(BSZ) SAMPLER_OCCUPANCY void sampler_kernel(DevSlots slots, SampleLaunch L) {
    __shared__ SampleShared sh;
    const int tid = threadIdx.x;
    const GSlots sl = sview(slots);
    const int64_t so = (int64_t)blockIdx.x * sl.stride;
    const Vis<LDS> V = slot_vis<BSZ, LDS>(sl, blockIdx.x);
    Counters cn = {0, 0, 0, 0};
    if (LDS) {
        for (int i = tid; i < 2 * Tab<tbits<BSZ, CMP>()>::CAP; i += BSZ) dyn_lds[i] = 0;
    }
    if (tid == 0) {
        for (int i = 0; i < 5; i++) sh.phase_ticks[i] = 0;
        sh.spills = 0;
        sh.deferred = 0;
        sh.walk_errs = 0;
        sh.balance = L.balance;
        sh.acc_task = -1;
        flush_task_stats(sh, L);
    }
    __syncthreads();
    const unsigned long long npairs = lane_u64(*L.npairs, 0);
    if (tid < 64) claim_next(L, npairs, sh);
    __syncthreads();
    // Every thread reads the claimed sample here; wave 1 claims the next one
    // only after run_sample's first barrier, and run_sample ends on a barrier.
    for (;;) {
        if (!sh.nx_ok) break;
        const unsigned long long q = sh.nx_idx;
        const int k = __builtin_amdgcn_readfirstlane(sh.nx_task);
        const int32_t s = __builtin_amdgcn_readfirstlane(sh.nx_s), t = __builtin_amdgcn_readfirstlane(sh.nx_t);
        const DevTask& T = L.tasks[k];
        if (tid == 0 && k != sh.acc_task) {
            flush_task_stats(sh, L);
            sh.acc_task = k;
        }
        run_sample<BSZ, LDS, CMP>(gview(T.g), sl, so, V, T.first + (q - T.offset), T, s, t, &L, npairs,
                                  (uint32_t)(q - L.base), k, sh, cn, nullptr, 0, 0);
    }
    flush_counters(cn, L.stats);
    if (tid == 0) {
        flush_task_stats(sh, L);
        for (int i = 0; i < 5; i++) atomicAdd(&L.stats->phase_ticks[i], sh.phase_ticks[i]);
        atomicAdd(&L.stats->spills, sh.spills);
        if (CMP) atomicAdd(&L.stats->deferred, sh.deferred);
        if (sh.walk_errs) atomicAdd(&L.stats->walk_errors, sh.walk_errs);
    }
}

template <int BSZ, bool LDS>
__global__ __launch_bounds__(BSZ) void debug_path_kernel(DevGraph g, DevSlots slots, int32_t s, int32_t t, uint64_t r,
                                                         DebugOut* out, int32_t cap) {
    __shared__ SampleShared sh;
    const GSlots sl = sview(slots);
    const Vis<LDS> V = slot_vis<BSZ, LDS>(sl, 0);
    Counters cn = {0, 0, 0, 0};
    if (LDS) {
        for (int i = threadIdx.x; i < 2 * Tab<tbits<BSZ, false>()>::CAP; i += BSZ) dyn_lds[i] = 0;
    }
    if (threadIdx.x == 0) {
        for (int i = 0; i < 5; i++) sh.phase_ticks[i] = 0;
        sh.balance = 100;
    }
    __syncthreads();
    DevTask T = {};
    run_sample<BSZ, LDS, false>(gview(g), sl, 0, V, 0, T, s, t, nullptr, 0, 0, -1, sh, cn, out, r, cap);
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void fill_u8_kernel(uint8_t* p, int64_t bytes) {
    const int64_t words = bytes / 16;
    uint4* p4 = (uint4*)p;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (int64_t)gridDim.x * blockDim.x)
        p4[i] = make_uint4(0, 0, 0, 0);
    for (int64_t i = words * 16 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < bytes;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// The pairs of one chunk of a launch, one lane per sample (Algorithm 2: U_s
// picks rank s by the prefix sums P, U_t picks rank t > s by F_s, both
// searches binary). Pairs whose s has no out-arcs or whose t has no in-arcs
// are counted as samples of their task (unreachable); the others are listed
// for the sampler.
__global__ __launch_bounds__(256) void pair_kernel(SampleLaunch L) {
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t count = (int64_t)L.count;
    for (int64_t b = wave * 64; b < count; b += nwaves * 64) {
        const int64_t qi = b + lane;
        int32_t k = 0, s = 0, t = 0;
        bool listed = false, trivial = false;
        if (qi < count) {
            const unsigned long long q = L.base + (unsigned long long)qi;
            // the task holding launch index q: last task with offset <= q
            int lo = 0, hi = L.ntasks - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (L.tasks[mid].offset <= q) lo = mid; else hi = mid - 1;
            }
            k = lo;
            const DevTask& T = L.tasks[k];
            const DevCdf& cdf = T.cdf;
            const uint64_t idx = T.first + (q - T.offset);
            const uint64_t Us = draw_bounded(T.seed, T.phase, idx, 0, cdf.C);
            const int32_t sr = lane_search(1, cdf.n, [&](int32_t d) { return Us < cdf.P[d]; });
            const uint64_t cs = cdf.P[sr] - cdf.P[sr - 1];
            const uint64_t Ut = draw_bounded(T.seed, T.phase, idx, 1, cs);
            const uint64_t ks = cdf.kr[sr], Ws = cdf.W[sr];
            const int32_t tr = lane_search(sr + 1, cdf.n, [&](int32_t d) {
                return Ut < (uint64_t)(d - sr + 1) * ks - (Ws - cdf.W[d + 1]);
            });
            s = cdf.perm[sr];
            t = cdf.perm[tr];
            // no path if s has no out-arcs or t no in-arcs (for an undirected
            // graph: an end without arcs)
            trivial = s >= T.g.n_act || t >= T.g.n_act || T.g.rp[s + 1] == T.g.rp[s] ||
                      T.g.irp[t + 1] == T.g.irp[t];
            listed = !trivial;
        }
        const unsigned long long lst = __ballot(listed);
        if (lst) {
            const unsigned long long at = wave_fetch_add(L.npairs, (unsigned long long)__popcll(lst));
            if (listed) L.pairs[at + __popcll(lst & below)] = PairRec{(uint32_t)qi, s, t, k};
        }
        // lane 0 is always in range here; its task takes one add per wave
        const int k0 = __builtin_amdgcn_readfirstlane(k);
        const unsigned long long same = __ballot(trivial && k == k0);
        if (same) (void)wave_fetch_add(&L.tasks[k0].stats->samples, (unsigned long long)__popcll(same));
        if (trivial && k != k0) atomicAdd(&L.tasks[k].stats->samples, 1ull);
    }
}

__global__ void init_chunk_kernel(unsigned long long* work, unsigned long long* npairs, unsigned long long* nwide,
                                  unsigned long long* nbig, unsigned long long* big_work) {
    if (threadIdx.x == 0) {
        *work = 0;
        *npairs = 0;
        *nwide = 0;
        *nbig = 0;
        *big_work = 0;
    }
}

// ------------------------------------------------------- 128-bit path
// Samples whose sigma_st reaches 2^64 are redone here with exact 128-bit
// counts (saturating at 2^128 - 1, which is an overflow): a plain
// level-synchronous BFS from s in which each new node pulls its count from
// its in-neighbours one level up (no atomics on counts), stopped at t's
// level, then r in [0, sigma_st) by Lemire's method at 128 bits and the
// canonical backward walk with 128-bit weights. Rare, so kept simple.
typedef unsigned __int128 u128;
constexpr int WB = 256;

__device__ __forceinline__ u128 sat_add128(u128 a, u128 b) {
    const u128 c = a + b;
    return c < a ? ~(u128)0 : c;
}

// Words 0 and 1 of the Philox4x64-10 block (the 64-bit path uses word 0).
__device__ void philox_words01(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0, uint64_t k1,
                               uint64_t& w0, uint64_t& w1) {
    for (int i = 0; i < 10; i++) {
        const uint64_t m0 = 0xD2E7470EE14C6C93ull, m1 = 0xCA5A826395121157ull;
        const uint64_t hi0 = __umul64hi(m0, c0), lo0 = m0 * c0;
        const uint64_t hi1 = __umul64hi(m1, c2), lo1 = m1 * c2;
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
    w0 = c0;
    w1 = c1;
}

// a * b as 256 bits (hi, lo) from 64-bit partial products.
__device__ __forceinline__ void mul_128x128(u128 a, u128 b, u128& hi, u128& lo) {
    const uint64_t a0 = (uint64_t)a, a1 = (uint64_t)(a >> 64), b0 = (uint64_t)b, b1 = (uint64_t)(b >> 64);
    const u128 p00 = (u128)a0 * b0, p01 = (u128)a0 * b1, p10 = (u128)a1 * b0, p11 = (u128)a1 * b1;
    const u128 mid = (p00 >> 64) + (uint64_t)p01 + (uint64_t)p10;
    lo = (u128)(uint64_t)p00 | (mid << 64);
    hi = p11 + (p01 >> 64) + (p10 >> 64) + (mid >> 64);
}

// r uniform in [0, N): the 64-bit draw of the sampler for N < 2^64, else
// Lemire at 128 bits on x = word 0 + 2^64 word 1.
__device__ u128 draw_r_wide(uint64_t seed, uint64_t phase, uint64_t idx, u128 N) {
    if ((N >> 64) == 0) return draw_bounded(seed, phase, idx, 2, (uint64_t)N);
    for (uint64_t attempt = 0;; attempt++) {
        uint64_t w0, w1;
        philox_words01(idx, 2, attempt, 0, seed, phase, w0, w1);
        const u128 x = (u128)w0 | ((u128)w1 << 64);
        u128 hi, lo;
        mul_128x128(x, N, hi, lo);
        if (lo < N) {
            const u128 thr = (u128)(0 - N) % N;
            if (lo < thr) continue;
        }
        return hi;
    }
}

struct WideShared {
    int32_t lo, hi, tail, level;
    unsigned long long q;
};

// BFS of one (s, t) on this workgroup's wide slot; returns d(s,t) or -1 (all
// threads), with sigma[t] complete. Leaves every reached node in q[0, tail).
__device__ int32_t wide_bfs(const DevGraph& g, int32_t* dist, u128* sig, int32_t* q, int32_t s, int32_t t,
                            WideShared& sh) {
    const int tid = threadIdx.x;
    if (tid == 0) {
        dist[s] = 0;
        sig[s] = 1;
        q[0] = s;
        sh.lo = 0; sh.hi = 1; sh.tail = 1; sh.level = 0;
    }
    __syncthreads();
    for (;;) {
        const int lo = sh.lo, hi = sh.hi, level = sh.level;
        if (__hip_atomic_load(dist + t, __ATOMIC_RELAXED, WGS) >= 0) return level;
        for (int i = lo + tid; i < hi; i += WB) {
            const int32_t u = q[i];
            for (int32_t e = g.rp[u]; e < g.rp[u + 1]; e++) {
                const int32_t v = g.col[e];
                int32_t expect = -1;
                if (__hip_atomic_load(dist + v, __ATOMIC_RELAXED, WGS) == -1 &&
                    __hip_atomic_compare_exchange_strong(dist + v, &expect, level + 1, __ATOMIC_RELAXED,
                                                         __ATOMIC_RELAXED, WGS))
                    q[atomicAdd(&sh.tail, 1)] = v;
            }
        }
        __syncthreads();
        const int nhi = sh.tail;
        if (nhi == hi) return -1;
        const bool t_new = __hip_atomic_load(dist + t, __ATOMIC_RELAXED, WGS) == level + 1;
        // counts of the new level (only t's once t is reached)
        for (int i = hi + tid; i < nhi; i += WB) {
            const int32_t v = q[i];
            if (t_new && v != t) continue;
            u128 acc = 0;
            for (int32_t e = g.irp[v]; e < g.irp[v + 1]; e++) {
                const int32_t u = g.icol[e];
                if (__hip_atomic_load(dist + u, __ATOMIC_RELAXED, WGS) == level) acc = sat_add128(acc, sig[u]);
            }
            sig[v] = acc;
        }
        __syncthreads();
        if (tid == 0) {
            sh.lo = hi;
            sh.hi = nhi;
            sh.level = level + 1;
        }
        __syncthreads();
    }
}

// Canonical walk with 128-bit weights (one thread), from t down to s: adds a
// hit to every internal node when hits is given, writes path[L] = t ..
// path[0] = s when path is given (cap entries); false if a step finds no
// predecessor (callers check a walk without hits first).
__device__ bool wide_walk(const DevGraph& g, const int32_t* dist, const u128* sig, int32_t t, int32_t L, u128 r,
                          uint32_t* hits, int32_t* path, int32_t cap) {
    int32_t w = t;
    if (path && L < cap) path[L] = t;
    for (int32_t pos = L; pos >= 1; pos--) {
        int32_t next = -1;
        for (int32_t e = g.irp[w]; e < g.irp[w + 1]; e++) {
            const int32_t u = g.ccol[e];  // ascending caller id
            if (dist[u] != pos - 1) continue;
            if (r < sig[u]) { next = u; break; }
            r -= sig[u];
        }
        if (next < 0) return false;
        if (path && pos - 1 < cap) path[pos - 1] = next;
        if (hits && pos - 1 >= 1) atomicAdd(hits + g.orig[next], 1u);
        w = next;
    }
    return true;
}

__device__ void wide_clear(int32_t* dist, u128* sig, const int32_t* q, int tail) {
    for (int i = threadIdx.x; i < tail; i += WB) {
        const int32_t v = q[i];
        dist[v] = -1;
        sig[v] = 0;
    }
}

__global__ __launch_bounds__(WB) void wide_kernel(SampleLaunch L, WideSlots W) {
    __shared__ WideShared sh;
    const int tid = threadIdx.x;
    const unsigned long long nwide = *L.nwide;
    int32_t* dist = W.dist + (int64_t)blockIdx.x * W.stride;
    u128* sig = W.sigma + (int64_t)blockIdx.x * W.stride;
    int32_t* q = W.queue + (int64_t)blockIdx.x * W.stride;
    for (;;) {
        if (tid == 0) sh.q = atomicAdd(W.work, 1ull);
        __syncthreads();
        const unsigned long long i = sh.q;
        if (i >= nwide) break;
        const PairRec rec = L.wide[i];
        const DevTask& T = L.tasks[rec.task];
        const unsigned long long lq = L.base + rec.q;
        const uint64_t idx = T.first + (lq - T.offset);
        const int32_t Ld = wide_bfs(T.g, dist, sig, q, rec.s, rec.t, sh);
        if (tid == 0 && Ld >= 0) {
            DevStats* st = T.stats;
            const u128 sg = sig[rec.t];
            if (sg == ~(u128)0) {
                atomicAdd(&st->overflow, 1ull);
                atomicMin(&st->first_overflow, (unsigned long long)idx);
            } else {
                const u128 r = draw_r_wide(T.seed, T.phase, idx, sg);
                // the walk is checked to reach s before it is walked again
                // with hits (the same path: it depends on r and the counts)
                if (wide_walk(T.g, dist, sig, rec.t, Ld, r, nullptr, nullptr, 0)) {
                    (void)wide_walk(T.g, dist, sig, rec.t, Ld, r, T.hits, nullptr, 0);
                    const unsigned long long I = (unsigned long long)(Ld - 1);
                    atomicAdd(&st->reachable, 1ull);
                    atomicAdd(&st->sum_I, I);
                    atomicAdd(&st->sum_I2, I * I);
                } else {
                    atomicAdd(&L.stats->walk_errors, 1ull);
                }
            }
        }
        __syncthreads();
        wide_clear(dist, sig, q, sh.tail);
        __syncthreads();
    }
}

__global__ __launch_bounds__(WB) void wide_debug_kernel(DevGraph g, WideSlots W, WideDebug* dbg) {
    __shared__ WideShared sh;
    const int32_t s = dbg->s, t = dbg->t;
    const int32_t Ld = wide_bfs(g, W.dist, W.sigma, W.queue, s, t, sh);
    if (threadIdx.x == 0) {
        dbg->L = Ld;
        dbg->sigma = Ld >= 0 ? W.sigma[t] : 0;
        dbg->overflow = (Ld >= 0 && dbg->sigma == ~(u128)0) ? 1 : 0;
        if (Ld >= 0 && !dbg->overflow && dbg->r < dbg->sigma && Ld + 1 <= dbg->cap) {
            if (!wide_walk(g, W.dist, W.sigma, t, Ld, dbg->r, nullptr, dbg->path, dbg->cap)) dbg->overflow = 2;
        }
    }
    __syncthreads();
    wide_clear(W.dist, W.sigma, W.queue, sh.tail);
}

__global__ void init_stats_kernel(DevStats* st, unsigned long long* work) {
    if (threadIdx.x == 0) {
        st->samples = st->reachable = st->sum_I = st->sum_I2 = st->overflow = 0;
        st->first_overflow = ~0ull;
        st->edges = st->sigma_adds = st->vexp = st->vdisc = st->spills = st->deferred = st->walk_errors = 0;
        for (int i = 0; i < 5; i++) st->phase_ticks[i] = 0;
        *work = 0;
    }
}

__global__ void clear_tasks_kernel(const DevTask* tasks, int ntasks) {
    const int k = blockIdx.y;
    if (k >= ntasks) return;
    const DevTask& T = tasks[k];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        DevStats* st = T.stats;
        st->samples = st->reachable = st->sum_I = st->sum_I2 = st->overflow = 0;
        st->first_overflow = ~0ull;
        st->edges = st->sigma_adds = st->vexp = st->vdisc = st->spills = st->deferred = st->walk_errors = 0;
        for (int i = 0; i < 5; i++) st->phase_ticks[i] = 0;
    }
    if (T.clear_hits) {
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < T.g.n; i += (int64_t)gridDim.x * blockDim.x)
            T.hits[i] = 0;
    }
}

static int fill_grid(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b < 1) b = 1;
    if (b > 4096) b = 4096;
    return (int)b;
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t count, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(fill_grid(count)), dim3(256), 0, stream, p, v, count);
    return hipGetLastError();
}

hipError_t launch_fill_u8(void* p, int64_t bytes, hipStream_t stream) {
    if (bytes <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u8_kernel, dim3(fill_grid(bytes / 16 + 1)), dim3(256), 0, stream, (uint8_t*)p, bytes);
    return hipGetLastError();
}

hipError_t launch_wide(const SampleLaunch& a, const WideSlots& w, int slots, hipStream_t stream) {
    if (slots <= 0) return hipSuccess;
    hipLaunchKernelGGL(init_chunk_kernel, dim3(1), dim3(64), 0, stream, w.work, w.work, w.work, w.work, w.work);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(wide_kernel, dim3(slots), dim3(WB), 0, stream, a, w);
    return hipGetLastError();
}

hipError_t launch_wide_debug(const DevGraph& g, const WideSlots& w, WideDebug* dbg, hipStream_t stream) {
    hipLaunchKernelGGL(wide_debug_kernel, dim3(1), dim3(WB), 0, stream, g, w, dbg);
    return hipGetLastError();
}

hipError_t launch_pairs(const SampleLaunch& a, hipStream_t stream) {
    hipLaunchKernelGGL(init_chunk_kernel, dim3(1), dim3(64), 0, stream, a.work, a.npairs, a.nwide, a.nbig, a.big_work);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || a.count == 0) return e;
    int64_t blocks = ((int64_t)a.count + 255) / 256;
    blocks = blocks < 1 ? 1 : (blocks > 8192 ? 8192 : blocks);
    hipLaunchKernelGGL(pair_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_init_stats(DevStats* st, unsigned long long* work, hipStream_t stream) {
    hipLaunchKernelGGL(init_stats_kernel, dim3(1), dim3(64), 0, stream, st, work);
    return hipGetLastError();
}

hipError_t launch_clear_tasks(const DevTask* tasks, int ntasks, int64_t max_n, hipStream_t stream) {
    if (ntasks <= 0) return hipSuccess;
    int64_t bx = (max_n + 255) / 256;
    bx = bx < 1 ? 1 : (bx > 512 ? 512 : bx);
    hipLaunchKernelGGL(clear_tasks_kernel, dim3((unsigned)bx, (unsigned)ntasks), dim3(256), 0, stream, tasks, ntasks);
    return hipGetLastError();
}

int64_t sampler_static_lds() { return (int64_t)sizeof(SampleShared); }
int64_t sampler_table_lds(bool compact, int block) {
    return (int64_t)2 * ((int64_t)1 << table_bits(block, compact)) * (int64_t)sizeof(uint32_t);
}
int sampler_table_cap(bool compact) { return compact ? CCAP : HCAP; }

template <int BSZ, bool LDS>
static const void* sampler_fn() {
    return reinterpret_cast<const void*>(&sampler_kernel<BSZ, LDS, false>);
}

static const void* pick_sampler(const SamplerShape& s) {
    if (s.compact) {
        if (!s.lds_sets) return nullptr;
        switch (s.block) {
            case 64: return reinterpret_cast<const void*>(&sampler_kernel<64, true, true>);
            case 128: return reinterpret_cast<const void*>(&sampler_kernel<128, true, true>);
            case 256: return reinterpret_cast<const void*>(&sampler_kernel<256, true, true>);
            default: return nullptr;
        }
    }
    switch (s.block) {
        case 64: return s.lds_sets ? sampler_fn<64, true>() : sampler_fn<64, false>();
        case 128: return s.lds_sets ? sampler_fn<128, true>() : sampler_fn<128, false>();
        case 256: return s.lds_sets ? sampler_fn<256, true>() : sampler_fn<256, false>();
        case 512: return s.lds_sets ? sampler_fn<512, true>() : sampler_fn<512, false>();
        case 1024: return s.lds_sets ? sampler_fn<1024, true>() : sampler_fn<1024, false>();
        default: return nullptr;
    }
}

int sampler_occupancy(const SamplerShape& s) {
    const void* fn = pick_sampler(s);
    if (!fn) return 0;
    int blocks = 0;
    const size_t dyn = s.lds_sets ? (size_t)sampler_table_lds(s.compact, s.block) : 0;
    if (dyn > 0) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
    (void)hipGetLastError();
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, s.block, dyn) != hipSuccess) return 0;
    return blocks;
}

hipError_t launch_sampler(const DevSlots& slots, const SampleLaunch& a, const SamplerShape& shape,
                          hipStream_t stream) {
    if (a.count == 0 || a.slots <= 0) return hipSuccess;
    const void* fn = pick_sampler(shape);
    if (!fn) return hipErrorInvalidValue;
    const size_t dyn = shape.lds_sets ? (size_t)sampler_table_lds(shape.compact, shape.block) : 0;
    if (dyn > 0) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
    (void)hipGetLastError();
    void* args[] = {(void*)&slots, (void*)&a};
    return hipLaunchKernel(fn, dim3(a.slots), dim3(shape.block), args, dyn, stream);
}

hipError_t launch_debug_path(const DevGraph& g, const DevSlots& slots, int32_t s, int32_t t, uint64_t r,
                             DebugOut* out, int32_t cap, const SamplerShape& shape, hipStream_t stream) {
    const void* fn = nullptr;
    switch (shape.block) {
        case 64: fn = shape.lds_sets ? (const void*)&debug_path_kernel<64, true> : (const void*)&debug_path_kernel<64, false>; break;
        case 128: fn = shape.lds_sets ? (const void*)&debug_path_kernel<128, true> : (const void*)&debug_path_kernel<128, false>; break;
        case 256: fn = shape.lds_sets ? (const void*)&debug_path_kernel<256, true> : (const void*)&debug_path_kernel<256, false>; break;
        case 512: fn = shape.lds_sets ? (const void*)&debug_path_kernel<512, true> : (const void*)&debug_path_kernel<512, false>; break;
        case 1024: fn = shape.lds_sets ? (const void*)&debug_path_kernel<1024, true> : (const void*)&debug_path_kernel<1024, false>; break;
        default: return hipErrorInvalidValue;
    }
    const size_t dyn = shape.lds_sets ? (size_t)sampler_table_lds(shape.compact, shape.block) : 0;
    if (dyn > 0) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
    (void)hipGetLastError();
    void* args[] = {(void*)&g, (void*)&slots, (void*)&s, (void*)&t, (void*)&r, (void*)&out, (void*)&cap};
    return hipLaunchKernel(fn, dim3(1), dim3(shape.block), args, dyn, stream);
}

}  // namespace percis
