// Device-side setup and reductions of the PercIS library on gfx950.
//
// * The exact integer pair distribution of Algorithm 2's preprocessing
//   (appendix), built from the states on the device: the ranks sorted by
//   (k non-increasing, caller id increasing) come from a stable two-pass LSD
//   radix sort on the 16-bit key 65535 - k (8-bit digits, one wave per tile of
//   1024 nodes, in-wave ranks by ballots so that each pass keeps id order);
//   W (suffix sums of the ranked states) and P (prefix sums of the pair
//   weights c_i = (n-i+1) kr_i - W_i, total C) are two device scans; per node,
//   S_v = C - sum_u |k_v - k_u| (the pairs that avoid v, Definition 1) comes
//   from a histogram of the 65536 state values, and d_v = C / S_v.
// * VertexDiamUB of Algorithm 1 (Section III-B): connected components of the
//   active nodes by min-label hooking with pointer jumping (weakly connected
//   components for directed graphs); for undirected graphs one multi-source
//   BFS from every component's node of smallest caller id gives that node's
//   eccentricity,
//   and a component bounds the vertex diameter by min(|C| - 2, 2 ecc - 1);
//   for directed graphs by |C| - 2.
// * The largest phase-1 weight max_v d_v h_v (the bound of Proposition 3 is
//   increasing in it, so its maximum over v is reached there) and the final
//   estimates d_v h_v / l of Algorithm 1.
// Every integer result equals a serial computation exactly; d_v, S_v and the
// estimates are single IEEE operations on exact integers, so they do too.
#include "percis_setup.h"

namespace percis {

namespace {

constexpr int EB = 256;           // threads per workgroup of the elementwise kernels
constexpr int RADIX_TILE = 1024;  // nodes per wave in a radix pass
constexpr int SCAN_B = 1024;      // elements per workgroup of a scan (one per thread)
constexpr int ARCS_PER_THREAD = 16;

#define AGENT __HIP_MEMORY_SCOPE_AGENT

__device__ __forceinline__ int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ int64_t gstride() { return (int64_t)gridDim.x * blockDim.x; }
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }
__device__ __forceinline__ int32_t uniform(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t lanes_below() { return (1ull << lane_id()) - 1ull; }

int grid_for(int64_t count, int block) {
    int64_t g = (count + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return (int)g;
}

__device__ __forceinline__ uint32_t shfl_up_t(uint32_t x, int o) { return (uint32_t)__shfl_up((int)x, o, 64); }
__device__ __forceinline__ uint64_t shfl_up_t(uint64_t x, int o) {
    const uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)x, o, 64);
    const uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)(x >> 32), o, 64);
    return ((uint64_t)hi << 32) | lo;
}

// Inclusive scan over a workgroup of SCAN_B threads (one element each);
// `total` receives the workgroup's sum. wsum holds SCAN_B / 64 entries.
template <class T>
__device__ T block_incl_scan(T x, T* wsum, T& total) {
    const int lane = lane_id(), wid = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const T y = shfl_up_t(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    T pre = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < SCAN_B / 64; i++) {
        const T s = wsum[i];
        if (i < wid) pre += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return x + pre;
}

// ---------------------------------------------------------------------------
// Scans. A scan is described by a functor with load(j) and store(j, incl, x)
// over j = 0 .. count-1: pass 1 sums each workgroup's elements, pass 2 turns
// the sums into exclusive offsets (one workgroup), pass 3 writes the scan.
// ---------------------------------------------------------------------------

// The radix histogram [digit][tile], exclusive, in place.
struct HistScan {
    uint32_t* h;
    __device__ uint32_t load(int64_t j) const { return h[j]; }
    __device__ void store(int64_t j, uint32_t incl, uint32_t x) const { h[j] = incl - x; }
};

// W[i] = sum_{j >= i} kr[j] for i = n .. 1 (element j of the scan is rank n - j).
struct SuffixW {
    const uint32_t* kr;
    uint64_t* W;
    int32_t n;
    __device__ uint64_t load(int64_t j) const { return kr[n - j]; }
    __device__ void store(int64_t j, uint64_t incl, uint64_t) const { W[n - j] = incl; }
};

// P[i] = sum_{j <= i} c_j with c_j = (n - j + 1) kr[j] - W[j] (element j of the
// scan is rank j + 1).
struct PrefixP {
    const uint32_t* kr;
    const uint64_t* W;
    uint64_t* P;
    int32_t n;
    __device__ uint64_t load(int64_t j) const {
        const int64_t i = j + 1;
        return (uint64_t)(n - i + 1) * kr[i] - W[i];
    }
    __device__ void store(int64_t j, uint64_t incl, uint64_t) const { P[j + 1] = incl; }
};

template <class T, class F>
__global__ void __launch_bounds__(SCAN_B) scan_sums_kernel(F f, int64_t count, T* sums) {
    __shared__ T wsum[SCAN_B / 64];
    const int64_t j = (int64_t)blockIdx.x * SCAN_B + threadIdx.x;
    const T x = j < count ? f.load(j) : (T)0;
    T tot;
    (void)block_incl_scan(x, wsum, tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

template <class T>
__global__ void __launch_bounds__(SCAN_B) scan_offsets_kernel(T* sums, int64_t nb) {
    __shared__ T wsum[SCAN_B / 64];
    T carry = 0;
    for (int64_t base = 0; base < nb; base += SCAN_B) {
        const int64_t j = base + threadIdx.x;
        const T x = j < nb ? sums[j] : (T)0;
        T tot;
        const T inc = block_incl_scan(x, wsum, tot);
        if (j < nb) sums[j] = carry + inc - x;
        carry += tot;
    }
}

template <class T, class F>
__global__ void __launch_bounds__(SCAN_B) scan_apply_kernel(F f, int64_t count, const T* sums) {
    __shared__ T wsum[SCAN_B / 64];
    const int64_t j = (int64_t)blockIdx.x * SCAN_B + threadIdx.x;
    const T x = j < count ? f.load(j) : (T)0;
    T tot;
    const T inc = block_incl_scan(x, wsum, tot) + sums[blockIdx.x];
    if (j < count) f.store(j, inc, x);
}

template <class T, class F>
hipError_t run_scan(const F& f, int64_t count, T* sums, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    const int64_t nb = (count + SCAN_B - 1) / SCAN_B;
    hipLaunchKernelGGL((scan_sums_kernel<T, F>), dim3((unsigned)nb), dim3(SCAN_B), 0, stream, f, count, sums);
    hipLaunchKernelGGL((scan_offsets_kernel<T>), dim3(1), dim3(SCAN_B), 0, stream, sums, nb);
    hipLaunchKernelGGL((scan_apply_kernel<T, F>), dim3((unsigned)nb), dim3(SCAN_B), 0, stream, f, count,
                       (const T*)sums);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// State build.
// ---------------------------------------------------------------------------

__global__ void fill_i32_kernel(int32_t* p, int64_t count, int32_t value) {
    for (int64_t i = gtid(); i < count; i += gstride()) p[i] = value;
}

__global__ void zero_u32_kernel(uint32_t* p, int64_t count) {
    for (int64_t i = gtid(); i < count; i += gstride()) p[i] = 0u;
}

// State histogram. Skewed states (most nodes at one value) would put most
// atomics on one bin, so up to four rounds per wave first gather the lanes
// that share the lowest pending lane's value into a single add.
__global__ void count_states_kernel(const uint16_t* k, int32_t n, uint32_t* cnt) {
    const int64_t n_pad = ((int64_t)n + 63) / 64 * 64;
    for (int64_t v = gtid(); v < n_pad; v += gstride()) {
        const bool ok = v < n;
        const int32_t kv = ok ? (int32_t)k[v] : -1;
        bool pending = ok;
#pragma unroll
        for (int round = 0; round < 4; round++) {
            const uint64_t act = __ballot(pending);
            if (!act) break;
            const int leader = __ffsll((unsigned long long)act) - 1;
            const int32_t kl = __shfl(kv, leader, 64);
            const uint64_t same = __ballot(pending && kv == kl);
            if (lane_id() == leader) atomicAdd(&cnt[kl], (uint32_t)__popcll(same));
            pending = pending && kv != kl;
        }
        if (pending) atomicAdd(&cnt[kv], 1u);
    }
}

// lt_cnt[x] = #{v : k_v < x}, lt_sum[x] = sum of k_v < x, for x = 0 .. 65536
// (one workgroup; thread t owns values 64t .. 64t+63).
__global__ void __launch_bounds__(1024) state_bins_kernel(const uint32_t* cnt, uint64_t* lt_cnt, uint64_t* lt_sum) {
    __shared__ uint64_t wc[16], ws[16];
    const int t = threadIdx.x;
    uint64_t c = 0, s = 0;
    for (int j = 0; j < 64; j++) {
        const uint64_t q = cnt[t * 64 + j];
        c += q;
        s += q * (uint64_t)(t * 64 + j);
    }
    uint64_t tc, ts;
    const uint64_t ic = block_incl_scan(c, wc, tc);
    const uint64_t is = block_incl_scan(s, ws, ts);
    uint64_t pc = ic - c, ps = is - s;
    for (int j = 0; j < 64; j++) {
        const int x = t * 64 + j;
        lt_cnt[x] = pc;
        lt_sum[x] = ps;
        const uint64_t q = cnt[x];
        pc += q;
        ps += q * (uint64_t)x;
    }
    if (t == 1023) {
        lt_cnt[65536] = pc;
        lt_sum[65536] = ps;
    }
}

// Radix pass PASS (0: low byte, 1: high byte of key = 65535 - k): per-tile
// digit counts into hist[digit * ntiles + tile]. Four waves per workgroup,
// one tile each.
template <int PASS>
__global__ void __launch_bounds__(256) radix_hist_kernel(const uint16_t* k, const uint16_t* keys, int32_t n,
                                                         int32_t ntiles, uint32_t* hist) {
    __shared__ uint32_t h[4][256];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    for (int d = lane; d < 256; d += 64) h[w][d] = 0;
    __syncthreads();
    const int64_t tile = (int64_t)blockIdx.x * 4 + w;
    if (tile < ntiles) {
        const int64_t beg = tile * RADIX_TILE, end = min((int64_t)n, beg + RADIX_TILE);
        for (int64_t i = beg + lane; i < end; i += 64) {
            const uint32_t key = PASS == 0 ? 65535u - k[i] : (uint32_t)keys[i];
            atomicAdd(&h[w][PASS == 0 ? (key & 255u) : (key >> 8)], 1u);
        }
    }
    __syncthreads();
    if (tile < ntiles)
        for (int d = lane; d < 256; d += 64) hist[(int64_t)d * ntiles + tile] = h[w][d];
}

// Radix pass PASS: each wave walks its tile in order, 64 nodes at a time; a
// node's place is its digit's offset for the tile plus the number of earlier
// nodes with the same digit (earlier rounds, then lower lanes), so the pass is
// stable. Pass 0 writes (key, caller id) pairs; pass 1 writes the ranks.
template <int PASS>
__global__ void __launch_bounds__(256) radix_scatter_kernel(const uint16_t* k, const uint16_t* keys_in,
                                                            const uint32_t* vals_in, int32_t n, int32_t ntiles,
                                                            const uint32_t* offs, uint16_t* keys_out,
                                                            uint32_t* vals_out, const int32_t* newid, int32_t* perm,
                                                            uint32_t* kr) {
    __shared__ uint32_t base[4][256];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int64_t tile = (int64_t)blockIdx.x * 4 + w;
    if (tile < ntiles)
        for (int d = lane; d < 256; d += 64) base[w][d] = offs[(int64_t)d * ntiles + tile];
    __syncthreads();
    if (tile >= ntiles) return;
    const int64_t beg = tile * RADIX_TILE, end = min((int64_t)n, beg + RADIX_TILE);
    for (int64_t i0 = beg; i0 < end; i0 += 64) {
        const int64_t i = i0 + lane;
        const bool ok = i < end;
        uint32_t key = 0, val = 0;
        if (ok) {
            if (PASS == 0) {
                key = 65535u - k[i];
                val = (uint32_t)i;
            } else {
                key = keys_in[i];
                val = vals_in[i];
            }
        }
        const uint32_t d = PASS == 0 ? (key & 255u) : (key >> 8);
        uint64_t eq = __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            eq &= bit ? bb : ~bb;
        }
        const uint32_t pos = ok ? base[w][d] + (uint32_t)__popcll(eq & lanes_below()) : 0u;
        __builtin_amdgcn_wave_barrier();
        if (ok && (eq >> lane) == 1ull) base[w][d] += (uint32_t)__popcll(eq);  // last lane of its digit
        __builtin_amdgcn_wave_barrier();
        if (ok) {
            if (PASS == 0) {
                keys_out[pos] = (uint16_t)key;
                vals_out[pos] = val;
            } else {
                perm[1 + pos] = newid[val];
                kr[1 + pos] = 65535u - key;
            }
        }
    }
}

__global__ void state_ends_kernel(int32_t n, int32_t* perm, uint32_t* kr, uint64_t* W, uint64_t* P) {
    if (gtid() == 0) {
        perm[0] = -1;
        kr[0] = 0;
        kr[n + 1] = 0;
        W[0] = 0;
        W[n + 1] = 0;
        P[0] = 0;
    }
}

__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
    return x;
}

__device__ __forceinline__ int64_t wave_max(int64_t x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const int64_t y = __shfl_xor((long long)x, o, 64);
        x = y > x ? y : x;
    }
    return x;
}

// S_v = C - (sum over u of |k_v - k_u|) and d_v = C / S_v, by caller id;
// result[0] = C, result[1] = max of the d_v bit patterns (pre-zeroed).
__global__ void node_weights_kernel(const uint16_t* k, int32_t n, const uint64_t* lt_cnt, const uint64_t* lt_sum,
                                    const uint64_t* P, double* d_v, double* S_v, uint64_t* result) {
    const uint64_t C = P[n];
    if (gtid() == 0) result[0] = C;
    double m = 0.0;
    const int64_t n_pad = ((int64_t)n + 63) / 64 * 64;  // whole waves in the loop
    for (int64_t v = gtid(); v < n_pad; v += gstride()) {
        if (v < n) {
            const uint64_t kv = k[v];
            const uint64_t below = lt_cnt[kv] * kv - lt_sum[kv];
            const uint64_t above = (lt_sum[65536] - lt_sum[kv + 1]) - (lt_cnt[65536] - lt_cnt[kv + 1]) * kv;
            const uint64_t S = C - (below + above);
            const double d = S ? (double)C / (double)S : 0.0;
            d_v[v] = d;
            S_v[v] = (double)S;
            m = fmax(m, d);
        }
    }
    m = wave_max(m);
    if (lane_id() == 0) atomicMax((unsigned long long*)&result[1], (unsigned long long)__double_as_longlong(m));
}

struct BuildLayout {
    int64_t cnt, lt_cnt, lt_sum, keys, vals, hist, sums, result, total;
    int32_t ntiles;
};

BuildLayout build_layout(int32_t n) {
    auto up = [](int64_t x) { return (x + 255) / 256 * 256; };
    BuildLayout L;
    L.ntiles = (int32_t)(((int64_t)n + RADIX_TILE - 1) / RADIX_TILE);
    const int64_t hist_n = 256LL * L.ntiles;
    const int64_t scan_n = hist_n > n ? hist_n : (int64_t)n;
    int64_t o = 0;
    L.cnt = o;    o += up(4LL * 65536);
    L.lt_cnt = o; o += up(8LL * 65537);
    L.lt_sum = o; o += up(8LL * 65537);
    L.keys = o;   o += up(2LL * n);
    L.vals = o;   o += up(4LL * n);
    L.hist = o;   o += up(4LL * hist_n);
    L.sums = o;   o += up(8LL * ((scan_n + SCAN_B - 1) / SCAN_B));
    L.result = o; o += up(16);
    L.total = o;
    return L;
}

// ---------------------------------------------------------------------------
// VertexDiamUB.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int32_t ld_relaxed(int32_t* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, AGENT); }

// Parents only ever decrease and never exceed the node, so the chase ends.
// The same chase with loads that may be served by the CU's cache, so a value
// can be stale within a kernel. Parents only decrease and stay inside their
// component, so a stale parent is still an ancestor in the same component:
// a stale root only makes a hook link two nodes of one component, or count a
// join that a later round finds settled. A round with no join writes nothing,
// so its reads are exact and the final check is exact too.
__device__ __forceinline__ int32_t find_root_cached(int32_t* parent, int32_t x) {
    int32_t p = __hip_atomic_load(parent + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    while (p != x) {
        x = p;
        p = __hip_atomic_load(parent + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    return x;
}

__device__ __forceinline__ int32_t find_root(int32_t* parent, int32_t x) {
    int32_t p = ld_relaxed(parent + x);
    while (p != x) {
        x = p;
        p = ld_relaxed(parent + x);
    }
    return x;
}

__global__ void wcc_init_kernel(int32_t* parent, int32_t na, uint32_t* ctr) {
    for (int64_t v = gtid(); v < na; v += gstride()) parent[v] = (int32_t)v;
    if (gtid() == 0)
        for (int i = 0; i < 4; i++) ctr[i] = 0u;
}

// One hooking round over the arcs (each thread a run of ARCS_PER_THREAD
// consecutive arcs): the larger of two different roots is linked under the
// smaller. ctr[0] := 1 if any arc joined two trees.
__global__ void wcc_hook_kernel(const int32_t* rp, const int32_t* col, int32_t na, int64_t m, int undirected,
                                int32_t* parent, uint32_t* ctr) {
    int64_t j = gtid() * ARCS_PER_THREAD;
    if (j >= m) return;
    const int64_t jend = min(m, j + ARCS_PER_THREAD);
    int32_t lo = 0, hi = na - 1;  // the row of arc j: the largest u with rp[u] <= j
    while (lo < hi) {
        const int32_t mid = (int32_t)(((int64_t)lo + hi + 1) >> 1);
        if (rp[mid] <= j) lo = mid; else hi = mid - 1;
    }
    int32_t u = lo;
    int32_t ru = -1;  // u's root, found again after a hook and for each new row
    bool joined = false;
    for (; j < jend; j++) {
        while (rp[u + 1] <= j) {
            u++;
            ru = -1;
        }
        const int32_t w = col[j];
        if (undirected && w < u) continue;  // each edge once
        if (ru < 0) ru = find_root_cached(parent, u);
        const int32_t rw = find_root_cached(parent, w);
        if (ru == rw) continue;
        atomicMin(&parent[ru > rw ? ru : rw], ru > rw ? rw : ru);
        joined = true;
        ru = -1;
    }
    if (joined) atomicOr(&ctr[0], 1u);
}

__global__ void wcc_compress_kernel(int32_t* parent, int32_t na) {
    for (int64_t v = gtid(); v < na; v += gstride()) {
        const int32_t r = find_root(parent, (int32_t)v);
        if (r != v) parent[v] = r;
    }
}

// first[c] := the smallest caller id in component c (c = its hooking root);
// first must hold INT32_MAX at the component roots.
__global__ void comp_first_kernel(const int32_t* parent, const int32_t* orig, int32_t na, int32_t* first) {
    for (int64_t v = gtid(); v < na; v += gstride()) atomicMin(&first[parent[v]], orig[v]);
}

// dist := 0 at each component's BFS root (its node of smallest caller id),
// -1 elsewhere; the roots form the first BFS frontier; ctr[1] counts them.
__global__ void bfs_init_kernel(const int32_t* parent, const int32_t* orig, const int32_t* first, int32_t na,
                                int32_t* dist, int32_t* q, uint32_t* ctr) {
    const int64_t na_pad = ((int64_t)na + 63) / 64 * 64;
    for (int64_t v = gtid(); v < na_pad; v += gstride()) {
        const bool root = v < na && orig[v] == first[parent[v]];
        if (v < na) dist[v] = root ? 0 : -1;
        const uint64_t bal = __ballot(root);
        uint32_t at = 0;
        if (bal && lane_id() == 0) at = atomicAdd(&ctr[1], (uint32_t)__popcll(bal));
        at = (uint32_t)__shfl((int)at, 0, 64);
        if (root) q[at + __popcll(bal & lanes_below())] = (int32_t)v;
    }
}

// Rows longer than SEG entries are split into segments of SEG entries that
// any wave can take, so that a hub's row does not hold one wave for a level.
constexpr int32_t SEG = 1024;
constexpr int BFS_BATCH = 8;  // BFS levels queued per host check (the count words fit the 256-byte counter block)

// The arcs col[b, e) of a frontier node, one wave, its lanes over the arcs:
// first visits are claimed by compare-and-swap and appended to the next
// frontier (count in *nout).
__device__ __forceinline__ void bfs_visit_row(const int32_t* col, int32_t b, int32_t e, int32_t* qout, uint32_t* nout,
                                              int32_t* dist, int32_t level) {
    const int lane = lane_id();
    for (int32_t j0 = b; j0 < e; j0 += 64) {
        const int32_t j = j0 + lane;
        bool found = false;
        int32_t y = 0;
        if (j < e) {
            y = col[j];
            if (ld_relaxed(dist + y) < 0) found = atomicCAS(&dist[y], -1, level + 1) == -1;
        }
        const uint64_t bal = __ballot(found);
        uint32_t at = 0;
        if (bal && lane == 0) at = atomicAdd(nout, (uint32_t)__popcll(bal));
        at = (uint32_t)__shfl((int)at, 0, 64);
        if (found) qout[at + __popcll(bal & lanes_below())] = y;
    }
}

// One BFS level: a wave per frontier node. A row longer than SEG is not
// scanned here: its segments (node, first entry) go to segs (count in *nseg)
// for bfs_segment_kernel.
__global__ void bfs_level_kernel(const int32_t* rp, const int32_t* col, const int32_t* qin, const uint32_t* nin_p,
                                 int32_t* qout, uint32_t* nout, int32_t* dist, int32_t level, int2* segs,
                                 uint32_t* nseg) {
    const int lane = lane_id();
    const int64_t nw = gstride() >> 6;
    const int64_t nin = (int64_t)uniform((int32_t)*nin_p);
    for (int64_t f = uniform((int32_t)(gtid() >> 6)); f < nin; f += nw) {
        const int32_t x = uniform(qin[f]);
        const int32_t b = uniform(rp[x]), e = uniform(rp[x + 1]);
        if (e - b > SEG) {
            const int32_t k = (e - b + SEG - 1) / SEG;
            uint32_t at = 0;
            if (lane == 0) at = atomicAdd(nseg, (uint32_t)k);
            at = (uint32_t)__shfl((int)at, 0, 64);
            for (int32_t i = lane; i < k; i += 64) segs[at + i] = make_int2(x, b + i * SEG);
        } else {
            bfs_visit_row(col, b, e, qout, nout, dist, level);
        }
    }
}

// Counts of a batch of BFS levels: lc[0] := *head (the current frontier's
// count, possibly lc[K] itself), lc[1..K] := 0, sc[0..K-1] := 0. One thread.
__global__ void bfs_batch_counts_kernel(const uint32_t* head, uint32_t* lc, uint32_t* sc, int K) {
    if (gtid() != 0) return;
    const uint32_t h = *head;
    for (int i = 1; i <= K; i++) lc[i] = 0u;
    for (int i = 0; i < K; i++) sc[i] = 0u;
    lc[0] = h;
}

// The long-row segments of the level: a wave per segment.
__global__ void bfs_segment_kernel(const int32_t* rp, const int32_t* col, const int2* segs, const uint32_t* nseg,
                                   int32_t* qout, uint32_t* nout, int32_t* dist, int32_t level) {
    const int64_t nw = gstride() >> 6;
    const int64_t ns = (int64_t)uniform((int32_t)*nseg);
    for (int64_t f = uniform((int32_t)(gtid() >> 6)); f < ns; f += nw) {
        const int2 sg = segs[f];
        const int32_t x = uniform(sg.x), b = uniform(sg.y);
        const int32_t e = (int32_t)min((int64_t)b + SEG, (int64_t)uniform(rp[x + 1]));
        bfs_visit_row(col, b, e, qout, nout, dist, level);
    }
}

// Component sizes and (if dist) the largest distance from each root. Lanes
// in the first lane's component are summed in the wave first.
__global__ void comp_stats_kernel(const int32_t* parent, const int32_t* dist, int32_t na, uint32_t* size,
                                  int32_t* ecc) {
    const int64_t na_pad = ((int64_t)na + 63) / 64 * 64;
    for (int64_t v = gtid(); v < na_pad; v += gstride()) {
        const bool ok = v < na;
        const int32_t r = ok ? parent[v] : -1;
        const int32_t d = ok && dist ? dist[v] : 0;
        const int32_t r0 = uniform(r);
        const bool same = ok && r == r0;
        const uint64_t bal = __ballot(same);
        const int64_t dm = wave_max((int64_t)(same ? d : 0));
        if (bal && lane_id() == 0) {
            atomicAdd(&size[r0], (uint32_t)__popcll(bal));
            if (dist) atomicMax(&ecc[r0], (int32_t)dm);
        }
        if (ok && !same) {
            atomicAdd(&size[r], 1u);
            if (dist) atomicMax(&ecc[r], d);
        }
    }
}

// D = max over components of min(|C| - 2, 2 ecc - 1) (undirected) or |C| - 2.
__global__ void diam_final_kernel(const int32_t* parent, const uint32_t* size, const int32_t* ecc, int32_t na,
                                  unsigned long long* D) {
    const int64_t na_pad = ((int64_t)na + 63) / 64 * 64;
    int64_t best = 0;
    for (int64_t v = gtid(); v < na_pad; v += gstride()) {
        if (v < na && parent[v] == v) {
            int64_t Dc = (int64_t)size[v] - 2;
            if (ecc) Dc = min(Dc, 2 * (int64_t)ecc[v] - 1);
            best = Dc > best ? Dc : best;
        }
    }
    best = wave_max(best);
    if (lane_id() == 0 && best > 0) atomicMax(D, (unsigned long long)best);
}

// ---------------------------------------------------------------------------
// Reductions and outputs of Algorithm 1.
// ---------------------------------------------------------------------------

__global__ void hit_weight_max_kernel(const double* d_v, const uint32_t* hits, int32_t n, unsigned long long* out) {
    double m = 0.0;
    for (int64_t v = gtid(); v < n; v += gstride()) m = fmax(m, d_v[v] * (double)hits[v]);
    m = wave_max(m);
    if (lane_id() == 0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

__global__ void estimates_kernel(const double* d_v, const uint32_t* hits, int32_t n, double l, double* p) {
    for (int64_t v = gtid(); v < n; v += gstride()) p[v] = d_v[v] * (double)hits[v] / l;
}

__global__ void exact_finish_kernel(const double* num, const double* S_v, const int32_t* newid, int32_t n,
                                    int32_t n_act, double* p) {
    for (int64_t v = gtid(); v < n; v += gstride()) {
        const int32_t i = newid[v];
        p[v] = (i < n_act && S_v[v] > 0) ? num[i] / S_v[v] : 0.0;
    }
}

__global__ void states_internal_kernel(const uint16_t* k, const int32_t* newid, int32_t n, uint16_t* kint) {
    for (int64_t v = gtid(); v < n; v += gstride()) kint[newid[v]] = k[v];
}

}  // namespace

int64_t state_build_bytes(int32_t n) { return build_layout(n).total; }

hipError_t launch_state_build(const StateArrays& a, void* scratch, const uint64_t** result_dev, hipStream_t stream) {
    const int32_t n = a.n;
    const BuildLayout L = build_layout(n);
    char* s = (char*)scratch;
    uint32_t* cnt = (uint32_t*)(s + L.cnt);
    uint64_t* lt_cnt = (uint64_t*)(s + L.lt_cnt);
    uint64_t* lt_sum = (uint64_t*)(s + L.lt_sum);
    uint16_t* keys = (uint16_t*)(s + L.keys);
    uint32_t* vals = (uint32_t*)(s + L.vals);
    uint32_t* hist = (uint32_t*)(s + L.hist);
    uint64_t* sums = (uint64_t*)(s + L.sums);
    uint64_t* result = (uint64_t*)(s + L.result);
    *result_dev = result;
    const int64_t hist_n = 256LL * L.ntiles;
    const int rgrid = (L.ntiles + 3) / 4;

    hipLaunchKernelGGL(zero_u32_kernel, dim3(grid_for(65536, EB)), dim3(EB), 0, stream, cnt, (int64_t)65536);
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(64), 0, stream, (uint32_t*)result, (int64_t)4);
    hipLaunchKernelGGL(count_states_kernel, dim3(grid_for(n, EB)), dim3(EB), 0, stream, a.k, n, cnt);
    hipLaunchKernelGGL(state_bins_kernel, dim3(1), dim3(1024), 0, stream, (const uint32_t*)cnt, lt_cnt, lt_sum);
    // pass 0: low byte of 65535 - k, from the states in caller-id order
    hipLaunchKernelGGL(radix_hist_kernel<0>, dim3(rgrid), dim3(256), 0, stream, a.k, (const uint16_t*)nullptr, n,
                       L.ntiles, hist);
    hipError_t e = run_scan<uint32_t>(HistScan{hist}, hist_n, (uint32_t*)sums, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(radix_scatter_kernel<0>, dim3(rgrid), dim3(256), 0, stream, a.k, (const uint16_t*)nullptr,
                       (const uint32_t*)nullptr, n, L.ntiles, (const uint32_t*)hist, keys, vals,
                       (const int32_t*)nullptr, (int32_t*)nullptr, (uint32_t*)nullptr);
    // pass 1: high byte; writes the ranks
    hipLaunchKernelGGL(radix_hist_kernel<1>, dim3(rgrid), dim3(256), 0, stream, (const uint16_t*)nullptr,
                       (const uint16_t*)keys, n, L.ntiles, hist);
    if ((e = run_scan<uint32_t>(HistScan{hist}, hist_n, (uint32_t*)sums, stream)) != hipSuccess) return e;
    hipLaunchKernelGGL(radix_scatter_kernel<1>, dim3(rgrid), dim3(256), 0, stream, (const uint16_t*)nullptr,
                       (const uint16_t*)keys, (const uint32_t*)vals, n, L.ntiles, (const uint32_t*)hist,
                       (uint16_t*)nullptr, (uint32_t*)nullptr, a.newid, a.perm, a.kr);
    hipLaunchKernelGGL(state_ends_kernel, dim3(1), dim3(64), 0, stream, n, a.perm, a.kr, a.W, a.P);
    if ((e = run_scan<uint64_t>(SuffixW{a.kr, a.W, n}, n, sums, stream)) != hipSuccess) return e;
    if ((e = run_scan<uint64_t>(PrefixP{a.kr, a.W, a.P, n}, n, sums, stream)) != hipSuccess) return e;
    hipLaunchKernelGGL(node_weights_kernel, dim3(grid_for(n, EB)), dim3(EB), 0, stream, a.k, n,
                       (const uint64_t*)lt_cnt, (const uint64_t*)lt_sum, (const uint64_t*)a.P, a.d_v, a.S_v, result);
    return hipGetLastError();
}

// Long-row segments of one BFS level: at most one per SEG arcs plus one per
// frontier node.
static int64_t max_segments(int32_t na, int64_t m) { return m / SEG + (int64_t)na + 64; }

int64_t diam_scratch_bytes(int32_t n_act, int64_t m) {
    const int64_t na = n_act > 0 ? n_act : 1;
    return 6 * ((4 * na + 255) / 256 * 256) + 256 + max_segments((int32_t)na, m) * (int64_t)sizeof(int2);
}

hipError_t run_vertex_diam_ub(const int32_t* rp, const int32_t* col, const int32_t* orig, int32_t na, int64_t m,
                              bool directed, void* scratch, int64_t* D_out, int32_t* levels_out, int32_t* rounds_out,
                              hipStream_t stream) {
    *D_out = 0;
    *levels_out = 0;
    *rounds_out = 0;
    if (na <= 0) return hipSuccess;
    const int64_t seg = (4LL * na + 255) / 256 * 256;
    char* s = (char*)scratch;
    int32_t* parent = (int32_t*)s;
    int32_t* dist = (int32_t*)(s + seg);
    int32_t* qa = (int32_t*)(s + 2 * seg);
    int32_t* qb = (int32_t*)(s + 3 * seg);
    uint32_t* size = (uint32_t*)(s + 4 * seg);
    int32_t* ecc = (int32_t*)(s + 5 * seg);
    uint32_t* ctr = (uint32_t*)(s + 6 * seg);            // [0] joined, [1] frontier count, [2..3] D, [4] segments
    unsigned long long* Dd = (unsigned long long*)(ctr + 2);
    int2* segs = (int2*)(s + 6 * seg + 256);
    hipError_t e = hipSuccess;
    const int g = grid_for(na, EB);
    hipLaunchKernelGGL(wcc_init_kernel, dim3(g), dim3(EB), 0, stream, parent, na, ctr);
    hipLaunchKernelGGL(zero_u32_kernel, dim3(grid_for(na, EB)), dim3(EB), 0, stream, size, (int64_t)na);
    hipLaunchKernelGGL(zero_u32_kernel, dim3(grid_for(na, EB)), dim3(EB), 0, stream, (uint32_t*)ecc, (int64_t)na);
    const int64_t hook_threads = (m + ARCS_PER_THREAD - 1) / ARCS_PER_THREAD;
    const int hook_grid = (int)((hook_threads + EB - 1) / EB);
    for (int round = 1;; round++) {
        uint32_t joined = 0;
        hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(64), 0, stream, ctr, (int64_t)1);
        if (m > 0)
            hipLaunchKernelGGL(wcc_hook_kernel, dim3(hook_grid > 0 ? hook_grid : 1), dim3(EB), 0, stream, rp, col, na,
                               m, directed ? 0 : 1, parent, ctr);
        hipLaunchKernelGGL(wcc_compress_kernel, dim3(g), dim3(EB), 0, stream, parent, na);
        if ((e = hipMemcpyAsync(&joined, ctr, sizeof joined, hipMemcpyDeviceToHost, stream)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(stream)) != hipSuccess) return e;
        *rounds_out = round;
        if (!joined) break;
    }
    const int32_t* dist_arg = nullptr;
    const int32_t* ecc_arg = nullptr;
    if (!directed) {
        // qb (free until the first level) holds each component's smallest caller id
        hipLaunchKernelGGL(fill_i32_kernel, dim3(g), dim3(EB), 0, stream, qb, (int64_t)na, INT32_MAX);
        hipLaunchKernelGGL(comp_first_kernel, dim3(g), dim3(EB), 0, stream, (const int32_t*)parent, orig, na, qb);
        hipLaunchKernelGGL(bfs_init_kernel, dim3(g), dim3(EB), 0, stream, (const int32_t*)parent, orig,
                           (const int32_t*)qb, na, dist, qa, ctr);
        uint32_t nin = 0;
        if ((e = hipMemcpyAsync(&nin, ctr + 1, sizeof nin, hipMemcpyDeviceToHost, stream)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(stream)) != hipSuccess) return e;
        int32_t level = 0;
        // Levels are queued BFS_BATCH at a time: each kernel reads its
        // frontier's count from device memory (an empty frontier makes the
        // rest of the batch no-ops), and the host looks once per batch.
        const int sgrid = grid_for(std::min<int64_t>(max_segments(na, m), 8192) * 64, EB);
        const int lgrid = grid_for(std::min<int64_t>(na, 8192) * 64, EB);
        uint32_t* lc = ctr + 8;    // [0..BFS_BATCH] frontier counts of the batch
        uint32_t* sc = ctr + 24;   // [0..BFS_BATCH) long-row segment counts
        const uint32_t* head = ctr + 1;
        while (nin > 0) {
            hipLaunchKernelGGL(bfs_batch_counts_kernel, dim3(1), dim3(64), 0, stream, head, lc, sc, BFS_BATCH);
            for (int i = 0; i < BFS_BATCH; i++) {
                hipLaunchKernelGGL(bfs_level_kernel, dim3(lgrid), dim3(EB), 0, stream, rp, col, (const int32_t*)qa,
                                   (const uint32_t*)(lc + i), qb, lc + i + 1, dist, level + i, segs, sc + i);
                hipLaunchKernelGGL(bfs_segment_kernel, dim3(sgrid), dim3(EB), 0, stream, rp, col, (const int2*)segs,
                                   (const uint32_t*)(sc + i), qb, lc + i + 1, dist, level + i);
                int32_t* t = qa;
                qa = qb;
                qb = t;
            }
            uint32_t counts[BFS_BATCH + 1];
            if ((e = hipMemcpyAsync(counts, lc, sizeof counts, hipMemcpyDeviceToHost, stream)) != hipSuccess) return e;
            if ((e = hipStreamSynchronize(stream)) != hipSuccess) return e;
            int done = BFS_BATCH;  // non-empty frontiers of this batch
            for (int i = 1; i <= BFS_BATCH; i++)
                if (counts[i] == 0) {
                    done = i;
                    break;
                }
            level += done;
            nin = counts[BFS_BATCH];
            head = lc + BFS_BATCH;
        }
        *levels_out = level;
        dist_arg = dist;
        ecc_arg = ecc;
    }
    hipLaunchKernelGGL(comp_stats_kernel, dim3(g), dim3(EB), 0, stream, (const int32_t*)parent, dist_arg, na, size,
                       (int32_t*)ecc_arg);
    hipLaunchKernelGGL(diam_final_kernel, dim3(g), dim3(EB), 0, stream, (const int32_t*)parent,
                       (const uint32_t*)size, ecc_arg, na, Dd);
    unsigned long long D = 0;
    if ((e = hipMemcpyAsync(&D, Dd, sizeof D, hipMemcpyDeviceToHost, stream)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(stream)) != hipSuccess) return e;
    *D_out = (int64_t)D;
    return hipGetLastError();
}

hipError_t launch_hit_weight_max(const double* d_v, const uint32_t* hits, int32_t n, unsigned long long* out,
                                 hipStream_t stream) {
    hipLaunchKernelGGL(hit_weight_max_kernel, dim3(grid_for(n, EB)), dim3(EB), 0, stream, d_v, hits, n, out);
    return hipGetLastError();
}

hipError_t launch_estimates(const double* d_v, const uint32_t* hits, int32_t n, uint64_t l, double* p,
                            hipStream_t stream) {
    hipLaunchKernelGGL(estimates_kernel, dim3(grid_for(n, EB)), dim3(EB), 0, stream, d_v, hits, n, (double)l, p);
    return hipGetLastError();
}

hipError_t launch_exact_finish(const double* num, const double* S_v, const int32_t* newid, int32_t n, int32_t n_act,
                               double* p, hipStream_t stream) {
    hipLaunchKernelGGL(exact_finish_kernel, dim3(grid_for(n, EB)), dim3(EB), 0, stream, num, S_v, newid, n, n_act, p);
    return hipGetLastError();
}

hipError_t launch_states_internal(const uint16_t* k, const int32_t* newid, int32_t n, uint16_t* kint,
                                  hipStream_t stream) {
    hipLaunchKernelGGL(states_internal_kernel, dim3(grid_for(n, EB)), dim3(EB), 0, stream, k, newid, n, kint);
    return hipGetLastError();
}

}  // namespace percis
