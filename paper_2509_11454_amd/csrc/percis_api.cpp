// Host side of the PercIS library: the C ABI of include/percis.h.
//
// Responsibilities: validation of inputs, the device copies of the graph
// (out- and in-adjacency), the exact integer pair distribution built from the
// states (the preprocessing of Algorithm 2), per-slot scratch, kernel
// launches, and the scalar bounds of Algorithm 1 (VertexDiamUB, Propositions 2
// and 3, Theorem 1). Every per-sample step runs on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "percis.h"
#include "percis_internal.h"

using namespace percis;

struct percis_ctx {
    int device = 0;
    bool host_only = false;                // created with PERCIS_HOST_ONLY: validation and host math only
    hipStream_t stream = nullptr;
    std::string err;
    int cu_count = 0;
    double wall_hz = 0.0;                  // device wall-clock rate

    // graph
    bool has_graph = false, directed = false;
    int32_t n = 0;
    int64_t m = 0;
    int32_t n_act = 0;                     // nodes with at least one arc (internal ids 0..n_act-1)
    std::vector<int32_t> h_rp, h_col;      // out-adjacency in internal ids, rows sorted
    std::vector<int32_t> h_irp, h_icol;    // in-adjacency (directed graphs only)
    std::vector<int32_t> h_orig, h_newid;  // internal id -> caller id, and back
    int32_t* d_orig = nullptr;
    bool graph_on_device = false;
    int32_t *d_rp = nullptr, *d_col = nullptr, *d_irp = nullptr, *d_icol = nullptr;

    // states
    bool has_states = false;
    uint64_t C = 0;
    std::vector<double> d_v;               // C / S_v, 0 where S_v = 0
    double d_hat = 1.0;
    std::vector<int32_t> h_perm;
    std::vector<uint32_t> h_kr;
    std::vector<uint64_t> h_W, h_P;
    bool states_on_device = false;
    int32_t* d_perm = nullptr;
    uint32_t* d_kr = nullptr;
    uint64_t *d_W = nullptr, *d_P = nullptr;

    // slots
    void* slot_mem = nullptr;
    int nslots = 0;
    int64_t slot_stride = 0;
    DevSlots slots{};

    // per-call buffers
    DevStats* d_stats = nullptr;
    unsigned long long* d_work = nullptr;
    uint32_t* d_hits = nullptr;            // internal hits [n]
    DebugOut* d_dbg = nullptr;
    int32_t dbg_cap = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;

    int64_t D_override = -1;
    int64_t opt_slots = 0, opt_scratch_mb = 0, opt_block = 0, opt_bitmaps = 0;
    SamplerShape shape{};
};

namespace {

int fail(percis_ctx* c, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

#define HIPCHK(c, expr)                                                                            \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail((c), e_ == hipErrorOutOfMemory ? PERCIS_E_NOMEM : PERCIS_E_DEVICE,          \
                        "%s: %s", #expr, hipGetErrorString(e_));                                   \
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
    if (e != hipSuccess) return fail(c, PERCIS_E_NOMEM, "hipMalloc(%zu bytes): %s", sizeof(T) * count, hipGetErrorString(e));
    p = (T*)q;
    return PERCIS_OK;
}

int set_device(percis_ctx* c) {
    HIPCHK(c, hipSetDevice(c->device));
    return PERCIS_OK;
}

void free_slots(percis_ctx* c) {
    if (c->slot_mem) (void)hipFree(c->slot_mem);
    c->slot_mem = nullptr;
    c->nslots = 0;
    c->slot_stride = 0;
    c->slots = DevSlots{};
}

void free_states(percis_ctx* c) {
    dfree(c->d_perm);
    dfree(c->d_kr);
    dfree(c->d_W);
    dfree(c->d_P);
    c->has_states = false;
    c->states_on_device = false;
    c->d_v.clear();
    c->h_perm.clear();
    c->h_kr.clear();
    c->h_W.clear();
    c->h_P.clear();
}

void free_graph(percis_ctx* c) {
    if (c->d_irp != c->d_rp) dfree(c->d_irp); else c->d_irp = nullptr;
    if (c->d_icol != c->d_col) dfree(c->d_icol); else c->d_icol = nullptr;
    dfree(c->d_rp);
    dfree(c->d_col);
    dfree(c->d_hits);
    dfree(c->d_orig);
    c->h_orig.clear();
    c->h_newid.clear();
    c->h_rp.clear();
    c->h_col.clear();
    c->h_irp.clear();
    c->h_icol.clear();
    c->has_graph = false;
    c->graph_on_device = false;
    free_slots(c);
    free_states(c);
}

// Uploads whatever of the graph and the pair distribution is not on the
// device yet. Host-only contexts stop here.
int ensure_graph_device(percis_ctx* c) {
    if (c->host_only) return fail(c, PERCIS_E_STATE, "host-only context: no device work possible");
    if (!c->has_graph) return fail(c, PERCIS_E_STATE, "load a graph first");
    int rc = set_device(c);
    if (rc) return rc;
    const int32_t n = c->n;
    const int64_t m = c->m;
    if (!c->graph_on_device) {
        if ((rc = dalloc(c, c->d_rp, (size_t)n + 1))) return rc;
        if ((rc = dalloc(c, c->d_col, (size_t)m))) return rc;
        HIPCHK(c, hipMemcpy(c->d_rp, c->h_rp.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice));
        if (m) HIPCHK(c, hipMemcpy(c->d_col, c->h_col.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice));
        if (c->directed) {
            if ((rc = dalloc(c, c->d_irp, (size_t)n + 1))) return rc;
            if ((rc = dalloc(c, c->d_icol, (size_t)m))) return rc;
            HIPCHK(c, hipMemcpy(c->d_irp, c->h_irp.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice));
            if (m) HIPCHK(c, hipMemcpy(c->d_icol, c->h_icol.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice));
        } else {
            c->d_irp = c->d_rp;
            c->d_icol = c->d_col;
        }
        if ((rc = dalloc(c, c->d_hits, (size_t)n))) return rc;
        if ((rc = dalloc(c, c->d_orig, (size_t)n))) return rc;
        HIPCHK(c, hipMemcpy(c->d_orig, c->h_orig.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
        c->graph_on_device = true;
    }
    return PERCIS_OK;
}

int ensure_device(percis_ctx* c) {
    int rc = ensure_graph_device(c);
    if (rc) return rc;
    if (!c->has_states) return fail(c, PERCIS_E_STATE, "set states first");
    const int32_t n = c->n;
    if (!c->states_on_device) {
        if ((rc = dalloc(c, c->d_perm, (size_t)n + 1))) return rc;
        if ((rc = dalloc(c, c->d_kr, (size_t)n + 2))) return rc;
        if ((rc = dalloc(c, c->d_W, (size_t)n + 2))) return rc;
        if ((rc = dalloc(c, c->d_P, (size_t)n + 1))) return rc;
        HIPCHK(c, hipMemcpy(c->d_perm, c->h_perm.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(c->d_kr, c->h_kr.data(), sizeof(uint32_t) * (n + 2), hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(c->d_W, c->h_W.data(), sizeof(uint64_t) * (n + 2), hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(c->d_P, c->h_P.data(), sizeof(uint64_t) * (n + 1), hipMemcpyHostToDevice));
        c->states_on_device = true;
    }
    return PERCIS_OK;
}

constexpr int64_t kSlotBytesPerNode = 4 + 4 + 8 + 8 + 4 + 4 + 4;
constexpr int64_t kLdsPerCu = 160 * 1024;

// Picks the launch shape and allocates (once per graph) the per-slot
// scratch: one slot per resident workgroup, capped by a memory budget.
int ensure_slots(percis_ctx* c) {
    if (c->slot_mem) return PERCIS_OK;
    const int64_t act = std::max<int32_t>(c->n_act, 1);
    const int64_t stride = (act + 63) / 64 * 64;
    const int64_t words = ((act + 31) / 32 + 63) / 64 * 64;
    SamplerShape sh{};
    sh.block = c->opt_block ? (int)c->opt_block : 1024;
    const int64_t lds_need = 3 * words * 4;
    const bool fits = lds_need + sampler_static_lds() <= kLdsPerCu;
    if (c->opt_bitmaps == 2 && !fits) return fail(c, PERCIS_E_INVAL, "bitmaps of %lld nodes do not fit in LDS", (long long)act);
    sh.lds_bitmaps = c->opt_bitmaps == 2 || (c->opt_bitmaps == 0 && fits);
    sh.lds_bytes = sh.lds_bitmaps ? lds_need : 0;
    const int occ = sampler_occupancy(sh);
    if (occ <= 0) return fail(c, PERCIS_E_DEVICE, "sampler shape (block %d, %s bitmaps) cannot launch", sh.block,
                              sh.lds_bitmaps ? "LDS" : "global");
    const int64_t per_slot = stride * kSlotBytesPerNode + (sh.lds_bitmaps ? 0 : 3 * words * 4);
    size_t free_b = 0, total_b = 0;
    HIPCHK(c, hipMemGetInfo(&free_b, &total_b));
    const int64_t budget = c->opt_scratch_mb > 0 ? c->opt_scratch_mb * (1ll << 20)
                                                 : std::min<int64_t>((int64_t)free_b / 2, 48ll << 30);
    const int64_t want = c->opt_slots > 0 ? c->opt_slots : (int64_t)std::max(c->cu_count, 1) * occ;
    int64_t ns = std::max<int64_t>(1, std::min(want, budget / per_slot));
    void* mem = nullptr;
    hipError_t e = hipErrorOutOfMemory;
    while (ns >= 1) {
        e = hipMalloc(&mem, (size_t)(ns * per_slot));
        if (e == hipSuccess) break;
        (void)hipGetLastError();
        ns /= 2;
    }
    if (e != hipSuccess || !mem) return fail(c, PERCIS_E_NOMEM, "cannot allocate sampler scratch");
    if (launch_fill_u8(mem, ns * per_slot, c->stream) != hipSuccess) {
        (void)hipFree(mem);
        return fail(c, PERCIS_E_DEVICE, "scratch clear failed");
    }
    char* p = (char*)mem;
    DevSlots s{};
    s.stride = stride;
    s.words = words;
    const int64_t cnt = ns * stride;
    s.lv_s = (uint32_t*)p; p += cnt * 4;
    s.lv_t = (uint32_t*)p; p += cnt * 4;
    s.sg_s = (uint64_t*)p; p += cnt * 8;
    s.sg_t = (uint64_t*)p; p += cnt * 8;
    s.q_s = (int32_t*)p; p += cnt * 4;
    s.q_t = (int32_t*)p; p += cnt * 4;
    s.q_d = (int32_t*)p; p += cnt * 4;
    s.bm = sh.lds_bitmaps ? nullptr : (uint32_t*)p;
    c->slot_mem = mem;
    c->slots = s;
    c->nslots = (int)ns;
    c->slot_stride = stride;
    c->shape = sh;
    return PERCIS_OK;
}

DevGraph dev_graph(const percis_ctx* c) {
    DevGraph g;
    g.n = c->n;
    g.n_act = c->n_act;
    g.orig = c->d_orig;
    g.rp = c->d_rp;
    g.col = c->d_col;
    g.irp = c->d_irp;
    g.icol = c->d_icol;
    return g;
}

DevCdf dev_cdf(const percis_ctx* c) {
    DevCdf d;
    d.n = c->n;
    d.C = c->C;
    d.perm = c->d_perm;
    d.kr = c->d_kr;
    d.W = c->d_W;
    d.P = c->d_P;
    return d;
}

// Undirected: BFS per connected component from its smallest node u; the
// component's shortest paths have at most min(|comp| - 2, 2 ecc(u) - 1)
// internal nodes. Directed: largest weakly connected component size - 2.
int64_t vertex_diam_ub(const percis_ctx* c) {
    const int32_t n = c->n;
    if (!c->directed) {
        std::vector<int32_t> dist(n, -1), queue(n);
        int64_t D = 0;
        for (int32_t u = 0; u < n; u++) {
            if (dist[u] >= 0) continue;
            size_t head = 0, tail = 0;
            dist[u] = 0;
            queue[tail++] = u;
            int32_t ecc = 0;
            while (head < tail) {
                int32_t x = queue[head++];
                ecc = std::max(ecc, dist[x]);
                for (int32_t e = c->h_rp[x]; e < c->h_rp[x + 1]; e++) {
                    int32_t y = c->h_col[e];
                    if (dist[y] < 0) {
                        dist[y] = dist[x] + 1;
                        queue[tail++] = y;
                    }
                }
            }
            int64_t Dc = std::min<int64_t>((int64_t)tail - 2, 2 * (int64_t)ecc - 1);
            D = std::max(D, Dc);
        }
        return D;
    }
    // union-find over arcs
    std::vector<int32_t> parent(n);
    for (int32_t v = 0; v < n; v++) parent[v] = v;
    auto find = [&](int32_t x) {
        while (parent[x] != x) {
            parent[x] = parent[parent[x]];
            x = parent[x];
        }
        return x;
    };
    for (int32_t u = 0; u < n; u++)
        for (int32_t e = c->h_rp[u]; e < c->h_rp[u + 1]; e++) {
            int32_t a = find(u), b = find(c->h_col[e]);
            if (a != b) parent[std::max(a, b)] = std::min(a, b);
        }
    std::vector<int64_t> size(n, 0);
    int64_t best = 0;
    for (int32_t v = 0; v < n; v++) best = std::max(best, ++size[find(v)]);
    return std::max<int64_t>(0, best - 2);
}

// Theorem 1 with the constants of Algorithm 1, as a function of x.
double sample_bound(double x, double d, double rho, double eps, double delta) {
    const double gx = x * (d - x);
    const double y = eps * d / gx;
    const double hy = (1.0 + y) * std::log1p(y) - y;
    return d * d * std::log(4.0 * d * rho / (x * delta)) / (gx * hy);
}

// sup over (0, x_hat]: a log-spaced scan over 16 decades, then golden-section
// refinement in log x around the best scan point, then the end point x_hat.
double sample_size_sup(double d, double rho, double v, double eps, double delta, double* x_hat_out) {
    const double q = d * d / 4.0;
    const double x_hat = d / 2.0 - std::sqrt(q - std::min(q, v));
    *x_hat_out = x_hat;
    const int N = 4096;
    const double lx_hi = std::log(x_hat), lx_lo = lx_hi - 16.0 * std::log(10.0);
    double best = sample_bound(x_hat, d, rho, eps, delta);
    int arg = N;
    for (int i = 0; i < N; i++) {
        const double lx = lx_lo + (lx_hi - lx_lo) * i / N;
        const double f = sample_bound(std::exp(lx), d, rho, eps, delta);
        if (f > best) { best = f; arg = i; }
    }
    if (arg < N) {
        const double step = (lx_hi - lx_lo) / N;
        double a = lx_lo + step * (arg - 1), b = std::min(lx_hi, lx_lo + step * (arg + 1));
        const double gr = (std::sqrt(5.0) - 1.0) / 2.0;
        double x1 = b - gr * (b - a), x2 = a + gr * (b - a);
        double f1 = sample_bound(std::exp(x1), d, rho, eps, delta), f2 = sample_bound(std::exp(x2), d, rho, eps, delta);
        for (int it = 0; it < 200 && b - a > 1e-13; it++) {
            if (f1 < f2) { a = x1; x1 = x2; f1 = f2; x2 = a + gr * (b - a); f2 = sample_bound(std::exp(x2), d, rho, eps, delta); }
            else { b = x2; x2 = x1; f2 = f1; x1 = b - gr * (b - a); f1 = sample_bound(std::exp(x1), d, rho, eps, delta); }
        }
        best = std::max(best, std::max(f1, f2));
    }
    return best;
}

int run_sampler(percis_ctx* c, uint64_t first, uint64_t count, uint64_t seed, uint32_t phase, uint32_t* d_hits,
                bool accumulate, percis_stats* st_out) {
    int rc = ensure_slots(c);
    if (rc) return rc;
    if (!accumulate) HIPCHK(c, launch_fill_u32(d_hits, 0u, c->n, c->stream));
    HIPCHK(c, launch_init_stats(c->d_stats, c->d_work, c->stream));
    SampleLaunch a{};
    a.first = first;
    a.count = count;
    a.seed = seed;
    a.phase = phase;
    a.hits = d_hits;
    a.stats = c->d_stats;
    a.work = c->d_work;
    a.slots = (int)std::min<uint64_t>((uint64_t)c->nslots, std::max<uint64_t>(count, 1));
    HIPCHK(c, hipEventRecord(c->ev0, c->stream));
    HIPCHK(c, launch_sampler(dev_graph(c), dev_cdf(c), c->slots, a, c->shape, c->stream));
    HIPCHK(c, hipEventRecord(c->ev1, c->stream));
    DevStats hs{};
    HIPCHK(c, hipMemcpyAsync(&hs, c->d_stats, sizeof hs, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
    percis_stats st{};
    st.samples = hs.samples;
    st.reachable = hs.reachable;
    st.sum_I = hs.sum_I;
    st.sum_I2 = hs.sum_I2;
    st.overflow = hs.overflow;
    st.first_overflow = hs.first_overflow;
    st.edges = hs.edges;
    st.sigma_adds = hs.sigma_adds;
    st.vertices_expanded = hs.vexp;
    st.vertices_discovered = hs.vdisc;
    st.kernel_ms = ms;
    for (int i = 0; i < 5; i++) st.phase_ms[i] = c->wall_hz > 0 ? (double)hs.phase_ticks[i] / c->wall_hz * 1e3 : 0.0;
    if (st_out) *st_out = st;
    if (st.samples != count)
        return fail(c, PERCIS_E_DEVICE, "sampler processed %llu of %llu samples", (unsigned long long)st.samples,
                    (unsigned long long)count);
    if (st.overflow)
        return fail(c, PERCIS_E_SIGMA_OVERFLOW, "%llu sample(s) with sigma_st >= 2^64, first index %llu",
                    (unsigned long long)st.overflow, (unsigned long long)st.first_overflow);
    return PERCIS_OK;
}

}  // namespace

extern "C" {

const char* percis_status_str(int s) {
    switch (s) {
        case PERCIS_OK: return "ok";
        case PERCIS_E_INVAL: return "invalid argument";
        case PERCIS_E_STATE: return "call out of order";
        case PERCIS_E_NOMEM: return "out of memory";
        case PERCIS_E_DEVICE: return "device error";
        case PERCIS_E_DEGENERATE: return "all percolation states are equal";
        case PERCIS_E_TOO_LARGE: return "input too large";
        case PERCIS_E_SIGMA_OVERFLOW: return "shortest-path count overflow";
        default: return "unknown status";
    }
}

const char* percis_last_error(const percis_ctx* c) { return c ? c->err.c_str() : "null context"; }

int percis_create(int device, void* hip_stream, percis_ctx** out) {
    if (!out) return PERCIS_E_INVAL;
    *out = nullptr;
    if (device == PERCIS_HOST_ONLY) {
        percis_ctx* c = new (std::nothrow) percis_ctx();
        if (!c) return PERCIS_E_NOMEM;
        c->host_only = true;
        c->device = -1;
        *out = c;
        return PERCIS_OK;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return PERCIS_E_DEVICE;
    if (device < 0 || device >= ndev) return PERCIS_E_INVAL;
    percis_ctx* c = new (std::nothrow) percis_ctx();
    if (!c) return PERCIS_E_NOMEM;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    if (hipSetDevice(device) != hipSuccess) { delete c; return PERCIS_E_DEVICE; }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) { delete c; return PERCIS_E_DEVICE; }
    c->cu_count = prop.multiProcessorCount;
    int wall_khz = 0;
    if (hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, device) == hipSuccess) c->wall_hz = wall_khz * 1e3;
    if (hipMalloc((void**)&c->d_stats, sizeof(DevStats)) != hipSuccess ||
        hipMalloc((void**)&c->d_work, sizeof(unsigned long long)) != hipSuccess ||
        hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
        percis_destroy(c);
        return PERCIS_E_DEVICE;
    }
    *out = c;
    return PERCIS_OK;
}

void percis_destroy(percis_ctx* c) {
    if (!c) return;
    if (!c->host_only) {
        (void)hipSetDevice(c->device);
        if (c->stream) (void)hipStreamSynchronize(c->stream); else (void)hipDeviceSynchronize();
    }
    free_graph(c);
    dfree(c->d_stats);
    dfree(c->d_work);
    dfree(c->d_dbg);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    delete c;
}

int percis_set_stream(percis_ctx* c, void* hip_stream) {
    if (!c) return PERCIS_E_INVAL;
    if (c->host_only) return fail(c, PERCIS_E_STATE, "host-only context has no stream");
    c->stream = (hipStream_t)hip_stream;
    return PERCIS_OK;
}

int percis_load_csr(percis_ctx* c, int32_t n, int64_t m, const int32_t* row_ptr, const int32_t* col, uint32_t flags) {
    if (!c) return PERCIS_E_INVAL;
    if (n < 1 || m < 0 || !row_ptr || (m > 0 && !col)) return fail(c, PERCIS_E_INVAL, "bad graph arguments");
    if (n > (1 << 25)) return fail(c, PERCIS_E_TOO_LARGE, "n = %d exceeds 2^25", n);
    if (m > 2147483647LL) return fail(c, PERCIS_E_TOO_LARGE, "m exceeds 2^31 - 1");
    if ((flags & PERCIS_DEVICE_PTRS) && c->host_only) return fail(c, PERCIS_E_INVAL, "device pointers on a host-only context");
    if (!c->host_only) {
        int rc = set_device(c);
        if (rc) return rc;
        if (c->stream) HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    free_graph(c);
    std::vector<int32_t> rp(n + 1), cl((size_t)m);
    if (flags & PERCIS_DEVICE_PTRS) {
        HIPCHK(c, hipMemcpy(rp.data(), row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost));
        if (m) HIPCHK(c, hipMemcpy(cl.data(), col, sizeof(int32_t) * m, hipMemcpyDeviceToHost));
    } else {
        std::memcpy(rp.data(), row_ptr, sizeof(int32_t) * (n + 1));
        if (m) std::memcpy(cl.data(), col, sizeof(int32_t) * m);
    }
    if (rp[0] != 0 || (int64_t)rp[n] != m) return fail(c, PERCIS_E_INVAL, "row_ptr[0] must be 0 and row_ptr[n] = m");
    for (int32_t v = 0; v < n; v++)
        if (rp[v + 1] < rp[v]) return fail(c, PERCIS_E_INVAL, "row_ptr decreases at row %d", v);
    for (int64_t e = 0; e < m; e++)
        if (cl[e] < 0 || cl[e] >= n) return fail(c, PERCIS_E_INVAL, "col[%lld] = %d out of range", (long long)e, cl[e]);
    for (int32_t v = 0; v < n; v++) {
        int32_t* b = cl.data() + rp[v];
        int32_t* e = cl.data() + rp[v + 1];
        if (!std::is_sorted(b, e)) std::sort(b, e);
        for (int32_t* p = b; p < e; p++) {
            if (*p == v) return fail(c, PERCIS_E_INVAL, "self-loop at node %d", v);
            if (p > b && p[-1] == *p) return fail(c, PERCIS_E_INVAL, "duplicate arc %d -> %d", v, *p);
        }
    }
    const bool directed = (flags & PERCIS_DIRECTED) != 0;
    if (!directed) {
        for (int32_t u = 0; u < n; u++)
            for (int32_t e = rp[u]; e < rp[u + 1]; e++) {
                const int32_t v = cl[e];
                if (!std::binary_search(cl.data() + rp[v], cl.data() + rp[v + 1], u))
                    return fail(c, PERCIS_E_INVAL, "undirected graph lacks arc %d -> %d (reverse of %d -> %d)", v, u, u, v);
            }
    }
    // internal ids: nodes with an arc first (in caller order), then the rest
    std::vector<uint8_t> has_arc(n, 0);
    for (int32_t u = 0; u < n; u++)
        if (rp[u + 1] > rp[u]) has_arc[u] = 1;
    for (int64_t e = 0; e < m; e++) has_arc[cl[e]] = 1;
    std::vector<int32_t> newid(n), orig(n);
    int32_t next = 0;
    for (int32_t v = 0; v < n; v++)
        if (has_arc[v]) { newid[v] = next; orig[next] = v; next++; }
    const int32_t n_act = next;
    for (int32_t v = 0; v < n; v++)
        if (!has_arc[v]) { newid[v] = next; orig[next] = v; next++; }
    std::vector<int32_t> irp2(n + 1, 0), icl2((size_t)m);
    irp2[0] = 0;
    for (int32_t i = 0; i < n; i++) {
        const int32_t v = orig[i];
        irp2[i + 1] = irp2[i] + (rp[v + 1] - rp[v]);
        int32_t o = irp2[i];
        for (int32_t e = rp[v]; e < rp[v + 1]; e++) icl2[o++] = newid[cl[e]];
        // the relabelling keeps the order of nodes with arcs, so rows stay sorted
    }
    rp.swap(irp2);
    cl.swap(icl2);
    if (directed) {
        // in-adjacency by a counting sort on the head; scanning tails in
        // increasing order keeps every in-row sorted
        std::vector<int32_t> irp(n + 1, 0), icl((size_t)m);
        for (int64_t e = 0; e < m; e++) irp[cl[e] + 1]++;
        for (int32_t v = 0; v < n; v++) irp[v + 1] += irp[v];
        std::vector<int32_t> pos(irp.begin(), irp.end() - 1);
        for (int32_t u = 0; u < n; u++)
            for (int32_t e = rp[u]; e < rp[u + 1]; e++) icl[pos[cl[e]]++] = u;
        c->h_irp.swap(irp);
        c->h_icol.swap(icl);
    }
    c->h_rp.swap(rp);
    c->h_col.swap(cl);
    c->h_orig.swap(orig);
    c->h_newid.swap(newid);
    c->n = n;
    c->n_act = n_act;
    c->m = m;
    c->directed = directed;
    c->has_graph = true;
    c->graph_on_device = false;
    return PERCIS_OK;
}

int percis_set_states(percis_ctx* c, const uint16_t* k_in, uint32_t flags) {
    if (!c) return PERCIS_E_INVAL;
    if (!c->has_graph) return fail(c, PERCIS_E_STATE, "load a graph first");
    if (!k_in) return fail(c, PERCIS_E_INVAL, "null states");
    if ((flags & PERCIS_DEVICE_PTRS) && c->host_only) return fail(c, PERCIS_E_INVAL, "device pointers on a host-only context");
    const int32_t n = c->n;
    std::vector<uint16_t> k(n);
    if (flags & PERCIS_DEVICE_PTRS) {
        int rc = set_device(c);
        if (rc) return rc;
        HIPCHK(c, hipMemcpy(k.data(), k_in, sizeof(uint16_t) * n, hipMemcpyDeviceToHost));
    } else {
        std::memcpy(k.data(), k_in, sizeof(uint16_t) * n);
    }
    if (!c->host_only) {
        int rc = set_device(c);
        if (rc) return rc;
        if (c->stream) HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    free_states(c);

    // ranks: counting sort on (65535 - k), stable in node id
    std::vector<int64_t> start(65537, 0);
    for (int32_t v = 0; v < n; v++) start[65535 - k[v] + 1]++;
    for (int i = 0; i < 65536; i++) start[i + 1] += start[i];
    std::vector<int32_t> perm(n + 1, -1);
    for (int32_t v = 0; v < n; v++) perm[1 + start[65535 - k[v]]++] = v;
    std::vector<uint32_t> kr(n + 2, 0);
    for (int32_t i = 1; i <= n; i++) kr[i] = k[perm[i]];
    for (int32_t i = 1; i <= n; i++) perm[i] = c->h_newid[perm[i]];  // the device works in internal ids
    std::vector<uint64_t> W(n + 2, 0), P(n + 1, 0);
    for (int32_t i = n; i >= 1; i--) W[i] = W[i + 1] + kr[i];
    for (int32_t i = 1; i <= n; i++) {
        const uint64_t ci = (uint64_t)(n - i + 1) * kr[i] - W[i];
        P[i] = P[i - 1] + ci;
    }
    const uint64_t C = P[n];
    if (C == 0) return fail(c, PERCIS_E_DEGENERATE, "all percolation states are equal");

    // d_v = C / S_v with S_v = C - sum_u |k_v - k_u| (the pairs that avoid v)
    std::vector<uint64_t> cnt(65537, 0), sum(65537, 0);
    for (int32_t v = 0; v < n; v++) { cnt[k[v] + 1]++; sum[k[v] + 1] += k[v]; }
    for (int i = 0; i < 65536; i++) { cnt[i + 1] += cnt[i]; sum[i + 1] += sum[i]; }
    c->d_v.assign(n, 0.0);
    double dh = 1.0;
    for (int32_t v = 0; v < n; v++) {
        const uint64_t kv = k[v];
        const uint64_t lo = cnt[kv] * kv - sum[kv];
        const uint64_t hi = (sum[65536] - sum[kv + 1]) - (cnt[65536] - cnt[kv + 1]) * kv;
        const uint64_t Sv = C - (lo + hi);
        c->d_v[v] = Sv ? (double)C / (double)Sv : 0.0;
        dh = std::max(dh, c->d_v[v]);
    }
    c->d_hat = dh;
    c->C = C;
    c->h_perm.swap(perm);
    c->h_kr.swap(kr);
    c->h_W.swap(W);
    c->h_P.swap(P);
    c->has_states = true;
    c->states_on_device = false;
    return PERCIS_OK;
}

int percis_sample_range(percis_ctx* c, uint64_t first, uint64_t count, uint64_t seed, uint32_t phase, uint32_t* hits,
                        uint32_t flags, percis_stats* st) {
    if (!c) return PERCIS_E_INVAL;
    if (!c->has_graph || !c->has_states) return fail(c, PERCIS_E_STATE, "load a graph and set states first");
    if (!hits) return fail(c, PERCIS_E_INVAL, "null hits");
    if (count >= (1ull << 32)) return fail(c, PERCIS_E_TOO_LARGE, "at most 2^32 - 1 samples per call");
    int rc = ensure_device(c);
    if (rc) return rc;
    const bool dev = (flags & PERCIS_DEVICE_PTRS) != 0;
    const bool acc = (flags & PERCIS_ACCUMULATE) != 0;
    uint32_t* dh = dev ? hits : c->d_hits;
    if (!dev && acc) HIPCHK(c, hipMemcpyAsync(dh, hits, sizeof(uint32_t) * c->n, hipMemcpyHostToDevice, c->stream));
    rc = run_sampler(c, first, count, seed, phase, dh, acc, st);
    if (rc != PERCIS_OK && rc != PERCIS_E_SIGMA_OVERFLOW) return rc;
    if (!dev) {
        HIPCHK(c, hipMemcpyAsync(hits, dh, sizeof(uint32_t) * c->n, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return rc;
}

int percis_sample(percis_ctx* c, uint64_t n_samples, uint64_t seed, uint32_t* hits, uint32_t flags, percis_stats* st) {
    return percis_sample_range(c, 0, n_samples, seed, 0, hits, flags, st);
}

int percis_set_vertex_diameter(percis_ctx* c, int64_t D) {
    if (!c) return PERCIS_E_INVAL;
    c->D_override = D;
    return PERCIS_OK;
}

int percis_estimate(percis_ctx* c, double eps, double delta, uint64_t seed, double* p_out, percis_estimate_info* info) {
    if (!c) return PERCIS_E_INVAL;
    if (!c->has_graph || !c->has_states) return fail(c, PERCIS_E_STATE, "load a graph and set states first");
    if (!(eps > 0 && eps < 1) || !(delta > 0 && delta < 1) || !p_out)
        return fail(c, PERCIS_E_INVAL, "need 0 < eps < 1, 0 < delta < 1 and an output array");
    int rc0 = ensure_device(c);
    if (rc0) return rc0;
    auto t0 = std::chrono::steady_clock::now();
    percis_estimate_info I{};
    const int32_t n = c->n;
    I.D = c->D_override >= 0 ? c->D_override : vertex_diam_ub(c);
    I.d_hat = c->d_hat;
    const double l1d = std::max(1000.0, std::log(1.0 / delta) / eps);
    I.l1 = (uint64_t)std::ceil(l1d);
    std::vector<uint32_t> h(n);

    // phase 1
    percis_stats s1{};
    int rc = percis_sample_range(c, 0, I.l1, seed, 1, h.data(), 0, &s1);
    if (rc != PERCIS_OK) {
        I.overflow = s1.overflow;
        if (info) *info = I;
        return rc;
    }
    I.phase1_ms = s1.kernel_ms;
    auto tb = std::chrono::steady_clock::now();
    const double l1 = (double)I.l1;
    I.rho_tilde = (double)s1.sum_I / l1;
    const unsigned __int128 num = (unsigned __int128)I.l1 * s1.sum_I2 - (unsigned __int128)s1.sum_I * s1.sum_I;
    I.Lambda = (double)num / (l1 * (l1 - 1.0));
    const double L8 = std::log(8.0 / delta), L4 = std::log(4.0 / delta);
    I.rho_hat = I.rho_tilde + std::sqrt(2.0 * I.Lambda * L8 / l1) + 7.0 * (double)I.D * L8 / (3.0 * (l1 - 1.0));
    double vmax = 0.0;
    for (int32_t v = 0; v < n; v++) {
        const double p1 = c->d_v[v] * h[v] / l1;
        vmax = std::max(vmax, p1 + std::sqrt(2.0 * p1 * L4 / l1) + L4 / (3.0 * l1));
    }
    I.v_hat = c->d_hat * c->d_hat * vmax;
    const double lb = sample_size_sup(c->d_hat, I.rho_hat, I.v_hat, eps, delta, &I.x_hat);
    if (!(lb < 4294967295.0)) {
        if (info) *info = I;
        return fail(c, PERCIS_E_TOO_LARGE, "phase-2 sample size %.3g exceeds 2^32 - 1", lb);
    }
    I.l = (uint64_t)std::ceil(lb);
    auto te = std::chrono::steady_clock::now();
    I.bounds_ms = std::chrono::duration<double, std::milli>(te - tb).count();

    // phase 2
    percis_stats s2{};
    rc = percis_sample_range(c, 0, I.l, seed, 2, h.data(), 0, &s2);
    I.overflow = s1.overflow + s2.overflow;
    I.phase2_ms = s2.kernel_ms;
    if (rc != PERCIS_OK) {
        if (info) *info = I;
        return rc;
    }
    for (int32_t v = 0; v < n; v++) p_out[v] = c->d_v[v] * (double)h[v] / (double)I.l;
    I.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = I;
    return PERCIS_OK;
}

int percis_debug_path(percis_ctx* c, int32_t s, int32_t t, uint64_t r, int32_t* path, int32_t cap, int32_t* L,
                      uint64_t* sigma, int32_t* overflow) {
    if (!c) return PERCIS_E_INVAL;
    if (!c->has_graph) return fail(c, PERCIS_E_STATE, "load a graph first");
    if (s < 0 || s >= c->n || t < 0 || t >= c->n || s == t || cap < 0 || (cap > 0 && !path))
        return fail(c, PERCIS_E_INVAL, "bad debug_path arguments");
    int rc = ensure_graph_device(c);  // the path needs the graph only
    if (rc) return rc;
    if ((rc = ensure_slots(c))) return rc;
    const int32_t need = std::max<int32_t>(cap, 1);
    if (need > c->dbg_cap) {
        dfree(c->d_dbg);
        void* p = nullptr;
        HIPCHK(c, hipMalloc(&p, sizeof(DebugOut) + sizeof(int32_t) * need));
        c->d_dbg = (DebugOut*)p;
        c->dbg_cap = need;
    }
    HIPCHK(c, launch_fill_u8(c->d_dbg, sizeof(DebugOut) + sizeof(int32_t) * need, c->stream));
    HIPCHK(c, launch_debug_path(dev_graph(c), c->slots, c->h_newid[s], c->h_newid[t], r, c->d_dbg, cap, c->shape,
                                c->stream));
    std::vector<char> buf(sizeof(DebugOut) + sizeof(int32_t) * need);
    HIPCHK(c, hipMemcpyAsync(buf.data(), c->d_dbg, buf.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const DebugOut* o = (const DebugOut*)buf.data();
    if (L) *L = o->L;
    if (sigma) *sigma = o->sigma;
    if (overflow) *overflow = o->overflow;
    if (o->overflow == 2) return fail(c, PERCIS_E_DEVICE, "canonical walk found no predecessor");
    if (path && o->L >= 0 && !o->overflow && r < o->sigma && o->L + 1 <= cap)
        for (int32_t i = 0; i <= o->L; i++) path[i] = c->h_orig[o->path[i]];
    return PERCIS_OK;
}

int percis_set_option(percis_ctx* c, int option, int64_t value) {
    if (!c) return PERCIS_E_INVAL;
    if (value < 0) return fail(c, PERCIS_E_INVAL, "negative option value");
    switch (option) {
        case PERCIS_OPT_SLOTS: c->opt_slots = value; break;
        case PERCIS_OPT_SCRATCH_MB: c->opt_scratch_mb = value; break;
        case PERCIS_OPT_BLOCK:
            if (value != 0 && value != 256 && value != 512 && value != 1024)
                return fail(c, PERCIS_E_INVAL, "block must be 256, 512 or 1024");
            c->opt_block = value;
            break;
        case PERCIS_OPT_BITMAPS:
            if (value > 2) return fail(c, PERCIS_E_INVAL, "bitmaps option is 0 (auto), 1 (global) or 2 (LDS)");
            c->opt_bitmaps = value;
            break;
        default: return fail(c, PERCIS_E_INVAL, "unknown option %d", option);
    }
    if (!c->host_only && set_device(c) == PERCIS_OK) {
        if (c->stream) (void)hipStreamSynchronize(c->stream); else (void)hipDeviceSynchronize();
        free_slots(c);
    }
    return PERCIS_OK;
}

int percis_get_option(percis_ctx* c, int option, int64_t* value) {
    if (!c || !value) return PERCIS_E_INVAL;
    switch (option) {
        case PERCIS_OPT_SLOTS: {
            if (c->host_only || !c->has_graph) { *value = c->opt_slots; return PERCIS_OK; }
            int rc = set_device(c);
            if (rc) return rc;
            if ((rc = ensure_slots(c))) return rc;
            *value = c->nslots;
            return PERCIS_OK;
        }
        case PERCIS_OPT_SCRATCH_MB: *value = c->opt_scratch_mb; return PERCIS_OK;
        case PERCIS_OPT_BLOCK:
        case PERCIS_OPT_BITMAPS: {
            if (c->host_only || !c->has_graph) {
                *value = option == PERCIS_OPT_BLOCK ? c->opt_block : c->opt_bitmaps;
                return PERCIS_OK;
            }
            int rc = set_device(c);
            if (rc) return rc;
            if ((rc = ensure_slots(c))) return rc;
            *value = option == PERCIS_OPT_BLOCK ? c->shape.block : (c->shape.lds_bitmaps ? 2 : 1);
            return PERCIS_OK;
        }
        default: return fail(c, PERCIS_E_INVAL, "unknown option %d", option);
    }
}

}  // extern "C"
