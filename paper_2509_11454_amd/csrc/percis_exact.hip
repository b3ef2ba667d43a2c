// Exact percolation centrality (Definition 1, Eq. 1) on gfx950 by the
// Brandes-style dependency accumulation that the paper uses for its exact
// values (Section IV-A).
//
// For a source s, with R_s(w) = max(0, k_s - k_w), the dependency
//   delta_s(v) = sum_{t != s, v} sigma_st(v) / sigma_st * R_s(t)
// obeys delta_s(v) = sum over successors w of v on shortest paths from s of
// sigma_sv / sigma_sw * (R_s(w) + delta_s(w)), and
//   p(v) = sum_{s != v} delta_s(v) / S_v.
// One persistent workgroup per slot takes sources from a counter; per
// source it runs a full level-synchronous BFS (shortest-path counts in
// double), then walks the levels back accumulating dependencies, and adds
// delta_s(v) into the slot's own partial sum (no cross-slot atomics). A final
// kernel sums the slots' partials. Floating-point sums run in a different
// order than a serial loop, so results match the CPU oracle to rounding.
#include "percis_internal.h"

namespace percis {

namespace {

constexpr int XB = 512;   // threads per workgroup
constexpr int XCH = 512;  // frontier nodes staged per chunk

#define XWG __HIP_MEMORY_SCOPE_WORKGROUP

__device__ __forceinline__ uint32_t xld32(uint32_t* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, XWG); }
__device__ __forceinline__ double xldd(double* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, XWG); }
__device__ __forceinline__ int32_t xldq(int32_t* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, XWG); }
__device__ __forceinline__ void xaddd(double* p, double v) {
    (void)__hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, XWG);
}

struct ExactShared {
    int32_t beg[XCH];
    int32_t off[XCH];
    double val[XCH];
    int32_t wsum[XB / 64];
    int32_t tail;
    int32_t nlev;
    unsigned long long idx;
};

__device__ __forceinline__ int xscan(int v, int32_t* wsum, int& total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    int pre = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < XB / 64; i++) {
        const int s = wsum[i];
        if (i < wid) pre += s;
        tot += s;
    }
    total = tot;
    return pre + x - v;
}

__device__ __forceinline__ int xowner(const ExactShared& sh, int cnt, int e) {
    int l2 = 0, h2 = cnt - 1;
    while (l2 < h2) {
        const int mid = (l2 + h2 + 1) >> 1;
        if (sh.off[mid] <= e) l2 = mid; else h2 = mid - 1;
    }
    return l2;
}

}  // namespace

struct ExactArgs {
    DevGraph g;
    const uint16_t* k;       // [n] states by internal id
    uint32_t* lv;            // [slots][stride] level + 1
    double* sigma;           // [slots][stride]
    double* delta;           // [slots][stride]
    int32_t* queue;          // [slots][stride]
    double* acc;             // [slots][stride] partial sums of delta
    int32_t* lstart;         // [slots][stride + 2] queue offset of each BFS level
    int64_t stride;
    unsigned long long* work;
};

__global__ __launch_bounds__(XB) void exact_kernel(ExactArgs A) {
    __shared__ ExactShared sh;
    const int tid = threadIdx.x;
    const int64_t so = (int64_t)blockIdx.x * A.stride;
    uint32_t* lv = A.lv + so;
    double* sg = A.sigma + so;
    double* dl = A.delta + so;
    int32_t* q = A.queue + so;
    double* acc = A.acc + so;
    int32_t* ls = A.lstart + (int64_t)blockIdx.x * (A.stride + 2);
    const DevGraph& g = A.g;
    for (;;) {
        if (tid == 0) sh.idx = atomicAdd(A.work, 1ull);
        __syncthreads();
        const unsigned long long src = sh.idx;
        if (src >= (unsigned long long)g.n_act) break;
        const int32_t s = (int32_t)src;
        if (tid == 0) {
            lv[s] = 1;
            sg[s] = 1.0;
            q[0] = s;
            sh.tail = 1;
            sh.nlev = 1;
            ls[0] = 0;
            ls[1] = 1;
        }
        __syncthreads();
        // ---- forward: full BFS with shortest-path counts
        int lo = 0, hi = 1;
        uint32_t d = 0;  // level of the frontier
        while (lo < hi) {
            const uint32_t nl = d + 2;  // stored value of the next level
            for (int base = lo; base < hi; base += XCH) {
                const int cnt = min(XCH, hi - base);
                int deg = 0, beg = 0;
                double su = 0.0;
                if (tid < cnt) {
                    const int32_t u = xldq(q + base + tid);
                    beg = g.rp[u];
                    deg = g.rp[u + 1] - beg;
                    su = xldd(sg + u);
                }
                int total;
                const int ex = xscan(deg, sh.wsum, total);
                if (tid < XCH) {
                    sh.beg[tid] = beg;
                    sh.off[tid] = ex;
                    sh.val[tid] = su;
                }
                __syncthreads();
                for (int e = tid; e < total; e += XB) {
                    const int j = xowner(sh, cnt, e);
                    const int32_t w = g.col[sh.beg[j] + (e - sh.off[j])];
                    uint32_t lw = xld32(lv + w);
                    if (lw == 0) {
                        uint32_t expct = 0;
                        if (__hip_atomic_compare_exchange_strong(lv + w, &expct, nl, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                                 XWG)) {
                            lw = nl;
                            const int pos = atomicAdd(&sh.tail, 1);
                            q[pos] = w;
                        } else {
                            lw = expct;
                        }
                    }
                    if (lw == nl) xaddd(sg + w, sh.val[j]);
                }
                __syncthreads();
            }
            lo = hi;
            hi = sh.tail;
            d++;
            if (tid == 0) {
                ls[sh.nlev + 1] = hi;
                sh.nlev++;
            }
            __syncthreads();
        }
        // levels: [ls[i], ls[i+1]) is level i, i < nlev (the last is empty)
        const int nlev = sh.nlev;
        const int ks = A.k[s];
        // ---- backward: dependencies, deepest level first
        for (int lvl = nlev - 1; lvl >= 1; lvl--) {
            const int lo2 = xldq(ls + lvl), hi2 = xldq(ls + lvl + 1);
            for (int base = lo2; base < hi2; base += XCH) {
                const int cnt = min(XCH, hi2 - base);
                int deg = 0, beg = 0;
                double cw = 0.0;
                if (tid < cnt) {
                    const int32_t w = xldq(q + base + tid);
                    beg = g.irp[w];
                    deg = g.irp[w + 1] - beg;
                    const int kw = A.k[w];
                    const double R = ks > kw ? (double)(ks - kw) : 0.0;
                    cw = (R + xldd(dl + w)) / xldd(sg + w);
                }
                int total;
                const int ex = xscan(deg, sh.wsum, total);
                if (tid < XCH) {
                    sh.beg[tid] = beg;
                    sh.off[tid] = ex;
                    sh.val[tid] = cw;
                }
                __syncthreads();
                const uint32_t want = (uint32_t)lvl;  // stored value of level lvl - 1
                for (int e = tid; e < total; e += XB) {
                    const int j = xowner(sh, cnt, e);
                    const int32_t v = g.icol[sh.beg[j] + (e - sh.off[j])];
                    if (xld32(lv + v) == want) xaddd(dl + v, xldd(sg + v) * sh.val[j]);
                }
                __syncthreads();
            }
        }
        // ---- accumulate and clear
        const int tot = sh.tail;
        for (int i = tid; i < tot; i += XB) {
            const int32_t v = xldq(q + i);
            if (v != s) acc[v] += xldd(dl + v);
            lv[v] = 0;
            sg[v] = 0.0;
            dl[v] = 0.0;
        }
        __syncthreads();
    }
}

__global__ void exact_reduce_kernel(const double* acc, int64_t stride, int slots, int32_t n_act, double* out) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n_act; v += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int i = 0; i < slots; i++) s += acc[(int64_t)i * stride + v];
        out[v] = s;
    }
}

hipError_t launch_exact(const DevGraph& g, const uint16_t* k, void* scratch, int64_t stride, int slots,
                        unsigned long long* work, double* out, hipStream_t stream) {
    ExactArgs A;
    A.g = g;
    A.k = k;
    char* p = (char*)scratch;
    const int64_t cnt = (int64_t)slots * stride;
    A.lv = (uint32_t*)p; p += cnt * 4;
    A.queue = (int32_t*)p; p += cnt * 4;
    A.sigma = (double*)p; p += cnt * 8;
    A.delta = (double*)p; p += cnt * 8;
    A.acc = (double*)p; p += cnt * 8;
    A.lstart = (int32_t*)p; p += (int64_t)slots * (stride + 2) * 4;
    A.stride = stride;
    A.work = work;
    hipLaunchKernelGGL(exact_kernel, dim3(slots), dim3(XB), 0, stream, A);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int64_t blocks = (g.n_act + 255) / 256;
    blocks = blocks < 1 ? 1 : (blocks > 4096 ? 4096 : blocks);
    hipLaunchKernelGGL(exact_reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, A.acc, stride, slots, g.n_act,
                       out);
    return hipGetLastError();
}

int64_t exact_scratch_bytes(int64_t stride, int slots) {
    return (int64_t)slots * stride * (4 + 4 + 8 + 8 + 8) + (int64_t)slots * (stride + 2) * 4;
}

}  // namespace percis
