// Host side of the PercIS library: the C ABI of include/percis.h.
//
// Responsibilities: validation of inputs, the internal numbering of a graph
// (nodes with arcs by degree, rows sorted, in-rows also kept in caller order)
// and its device copies, driving the device builds of the exact integer pair
// distribution (the preprocessing of Algorithm 2) and of VertexDiamUB,
// per-slot scratch, task launches and captures, the autotuner, and the scalar
// bounds of Algorithm 1 (Propositions 2 and 3, Theorem 1). Every per-sample
// step runs on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "percis.h"
#include "percis_host.h"
#include "percis_internal.h"
#include "percis_setup.h"

using namespace percis;

namespace percis {

int fail(percis_ctx* c, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

static void graph_free_states(GraphData& G) {
    dfree(G.d_k);
    dfree(G.d_perm);
    dfree(G.d_kr);
    dfree(G.d_W);
    dfree(G.d_P);
    dfree(G.d_dv);
    dfree(G.d_Sv);
    dfree(G.d_p);
    dfree(G.d_red);
    if (G.build_mem) (void)hipFree(G.build_mem);
    G.build_mem = nullptr;
    G.has_states = false;
    G.states_on_device = false;
}

static void graph_free_device(GraphData& G) {
    if (G.d_irp != G.d_rp) dfree(G.d_irp); else G.d_irp = nullptr;
    if (G.d_icol != G.d_col) dfree(G.d_icol); else G.d_icol = nullptr;
    dfree(G.d_rp);
    dfree(G.d_col);
    G.d_ccol = nullptr;  // inside the in-row buffer
    dfree(G.d_orig);
    dfree(G.d_newid);
    dfree(G.d_hits);
    graph_free_states(G);
    G.graph_on_device = false;
}

static void graph_clear(GraphData& G) {
    graph_free_device(G);
    G.h_rp.clear();
    G.h_col.clear();
    G.h_irp.clear();
    G.h_icol.clear();
    G.h_ccol.clear();
    G.h_orig.clear();
    G.h_newid.clear();
    G.has_graph = false;
    G.n = G.n_act = 0;
    G.m = 0;
    G.D_cached = -1;
}

// Host threads for a graph's load: one per 4 M arcs, at most the hardware's
// threads and 16.
static int host_threads(int64_t m) {
    const int hw = std::max(1u, std::thread::hardware_concurrency());
    return (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)hw, 16, m / (4 << 20) + 1}));
}

// nth contiguous row ranges with about equal arc counts: rows [r[t], r[t+1]).
static std::vector<int32_t> row_split(const std::vector<int32_t>& rp, int nth) {
    const int32_t n = (int32_t)rp.size() - 1;
    const int64_t m = rp[n];
    std::vector<int32_t> r(nth + 1, n);
    r[0] = 0;
    for (int t = 1; t < nth; t++) {
        const int32_t target = (int32_t)(m * t / nth);
        r[t] = std::max(r[t - 1], (int32_t)(std::lower_bound(rp.begin(), rp.end(), target) - rp.begin()));
        r[t] = std::min(r[t], n);
    }
    return r;
}

// fn(t) for t in [0, nth) on nth threads (the caller's thread takes t = 0).
template <class F>
static void parallel_ranges(int nth, F fn) {
    std::vector<std::thread> th;
    for (int t = 1; t < nth; t++) {
        try {
            th.emplace_back(fn, t);
        } catch (...) {
            fn(t);  // no thread to be had: this range runs here
        }
    }
    fn(0);
    for (auto& x : th) x.join();
}

static int graph_load(percis_ctx* c, GraphData& G, int32_t n, int64_t m, const int32_t* row_ptr, const int32_t* col,
                      uint32_t flags) {
    if (n < 1 || m < 0 || !row_ptr || (m > 0 && !col)) return fail(c, PERCIS_E_INVAL, "bad graph arguments");
    if (n > (1 << 25)) return fail(c, PERCIS_E_TOO_LARGE, "n = %d exceeds 2^25", n);
    if (m > 2147483647LL) return fail(c, PERCIS_E_TOO_LARGE, "m exceeds 2^31 - 1");
    if ((flags & PERCIS_DEVICE_PTRS) && c->host_only) return fail(c, PERCIS_E_INVAL, "device pointers on a host-only context");
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
    // The checks and the renumbering below run over row ranges on host
    // threads; each thread keeps the first failure of its range, and the
    // first one over all ranges is reported, as a serial pass would.
    const int nth = host_threads(m);
    const std::vector<int32_t> rows = row_split(rp, nth);
    {
        std::vector<int64_t> bad(nth, -1);
        parallel_ranges(nth, [&](int t) {
            for (int64_t e = rp[rows[t]]; e < rp[rows[t + 1]]; e++)
                if (cl[e] < 0 || cl[e] >= n) { bad[t] = e; return; }
        });
        for (int t = 0; t < nth; t++)
            if (bad[t] >= 0)
                return fail(c, PERCIS_E_INVAL, "col[%lld] = %d out of range", (long long)bad[t], cl[bad[t]]);
    }
    {
        struct Bad { int32_t v = -1; int kind = 0; int32_t w = 0; };  // kind 1: self-loop, 2: duplicate
        std::vector<Bad> bad(nth);
        parallel_ranges(nth, [&](int t) {
            for (int32_t v = rows[t]; v < rows[t + 1]; v++) {
                int32_t* b = cl.data() + rp[v];
                int32_t* e = cl.data() + rp[v + 1];
                if (!std::is_sorted(b, e)) std::sort(b, e);
                for (int32_t* q = b; q < e; q++) {
                    if (*q == v) { bad[t] = Bad{v, 1, v}; return; }
                    if (q > b && q[-1] == *q) { bad[t] = Bad{v, 2, *q}; return; }
                }
            }
        });
        for (int t = 0; t < nth; t++) {
            if (bad[t].kind == 1) return fail(c, PERCIS_E_INVAL, "self-loop at node %d", bad[t].v);
            if (bad[t].kind == 2) return fail(c, PERCIS_E_INVAL, "duplicate arc %d -> %d", bad[t].v, bad[t].w);
        }
    }
    const bool directed = (flags & PERCIS_DIRECTED) != 0;
    if (!directed) {
        std::vector<int64_t> bad(nth, -1);
        parallel_ranges(nth, [&](int t) {
            for (int32_t u = rows[t]; u < rows[t + 1]; u++)
                for (int32_t e = rp[u]; e < rp[u + 1]; e++) {
                    const int32_t v = cl[e];
                    if (!std::binary_search(cl.data() + rp[v], cl.data() + rp[v + 1], u)) {
                        bad[t] = e;
                        return;
                    }
                }
        });
        for (int t = 0; t < nth; t++)
            if (bad[t] >= 0) {
                const int32_t v = cl[bad[t]];
                const int32_t u = (int32_t)(std::upper_bound(rp.begin(), rp.end(), (int32_t)bad[t]) - rp.begin()) - 1;
                return fail(c, PERCIS_E_INVAL, "undirected graph lacks arc %d -> %d (reverse of %d -> %d)", v, u, u, v);
            }
    }
    // Internal ids: nodes with an arc first, by degree (out + in) from the
    // largest down, ties in caller order; then the nodes without arcs. The
    // arcs a search touches mostly end at high-degree nodes, so their node
    // records, bitmap words and row bounds share cache lines.
    std::vector<int64_t> deg(n, 0);
    parallel_ranges(nth, [&](int t) {
        for (int32_t u = rows[t]; u < rows[t + 1]; u++) deg[u] = rp[u + 1] - rp[u];
    });
    if (directed)
        parallel_ranges(nth, [&](int t) {
            for (int64_t e = rp[rows[t]]; e < rp[rows[t + 1]]; e++) __atomic_fetch_add(&deg[cl[e]], 1, __ATOMIC_RELAXED);
        });
    int64_t dmax = 0;
    for (int32_t u = 0; u < n; u++) dmax = std::max(dmax, deg[u]);
    std::vector<int32_t> newid(n), orig(n);
    {
        // counting sort on degree, largest first, stable in caller order
        std::vector<int64_t> start((size_t)dmax + 2, 0);
        for (int32_t u = 0; u < n; u++) start[(size_t)(dmax - deg[u]) + 1]++;
        for (size_t d = 1; d < start.size(); d++) start[d] += start[d - 1];
        for (int32_t u = 0; u < n; u++) {
            const int32_t id = (int32_t)start[(size_t)(dmax - deg[u])]++;
            newid[u] = id;
            orig[id] = u;
        }
    }
    int32_t n_act = 0;
    while (n_act < n && deg[orig[n_act]] > 0) n_act++;
    std::vector<int64_t>().swap(deg);
    std::vector<int32_t> rp2(n + 1, 0), cl2((size_t)m);
    for (int32_t i = 0; i < n; i++) rp2[i + 1] = rp2[i] + (rp[orig[i] + 1] - rp[orig[i]]);
    const std::vector<int32_t> rows2 = row_split(rp2, nth);
    parallel_ranges(nth, [&](int t) {
        for (int32_t i = rows2[t]; i < rows2[t + 1]; i++) {
            const int32_t v = orig[i];
            int32_t o = rp2[i];
            for (int32_t e = rp[v]; e < rp[v + 1]; e++) cl2[o++] = newid[cl[e]];
        }
    });
    std::vector<int32_t>().swap(cl);
    graph_clear(G);
    if (directed) {
        // in-adjacency by a counting sort on the head, each thread over a
        // range of tails in caller order (rows of the caller's numbering);
        // the threads' counts give each one its place in every in-row, so
        // every in-row lists its tails in caller order
        std::vector<int32_t> irp(n + 1, 0), icl((size_t)m);
        const int nt2 = std::max(1, std::min<int>(nth, (int)((int64_t)(512 << 20) / (4 * (int64_t)n + 4))));
        const std::vector<int32_t> trows = row_split(rp, nt2);
        std::vector<std::vector<int32_t>> cnt(nt2);
        parallel_ranges(nt2, [&](int t) {
            cnt[t].assign(n, 0);
            for (int32_t v = trows[t]; v < trows[t + 1]; v++) {
                const int32_t u = newid[v];
                for (int32_t e = rp2[u]; e < rp2[u + 1]; e++) cnt[t][cl2[e]]++;
            }
        });
        for (int32_t h = 0; h < n; h++) {
            int32_t tot = 0;
            for (int t = 0; t < nt2; t++) tot += cnt[t][h];
            irp[h + 1] = irp[h] + tot;
        }
        parallel_ranges(nth, [&](int t) {
            // per head, each tail range's first slot
            const int32_t h0 = (int32_t)((int64_t)n * t / nth), h1 = (int32_t)((int64_t)n * (t + 1) / nth);
            for (int32_t h = h0; h < h1; h++) {
                int32_t at = irp[h];
                for (int r = 0; r < nt2; r++) {
                    const int32_t k = cnt[r][h];
                    cnt[r][h] = at;
                    at += k;
                }
            }
        });
        parallel_ranges(nt2, [&](int t) {
            for (int32_t v = trows[t]; v < trows[t + 1]; v++) {
                const int32_t u = newid[v];
                for (int32_t e = rp2[u]; e < rp2[u + 1]; e++) icl[cnt[t][cl2[e]]++] = u;
            }
        });
        std::vector<std::vector<int32_t>>().swap(cnt);
        // the canonical walk reads in-rows in caller order; the searches read
        // them sorted by internal id
        G.h_ccol = icl;
        const std::vector<int32_t> irows = row_split(irp, nth);
        parallel_ranges(nth, [&](int t) {
            for (int32_t v = irows[t]; v < irows[t + 1]; v++) std::sort(icl.begin() + irp[v], icl.begin() + irp[v + 1]);
        });
        G.h_irp.swap(irp);
        G.h_icol.swap(icl);
    } else {
        G.h_ccol = cl2;
    }
    parallel_ranges(nth, [&](int t) {
        for (int32_t v = rows2[t]; v < rows2[t + 1]; v++) std::sort(cl2.begin() + rp2[v], cl2.begin() + rp2[v + 1]);
    });
    G.h_rp.swap(rp2);
    G.h_col.swap(cl2);
    G.h_orig.swap(orig);
    G.h_newid.swap(newid);
    G.n = n;
    G.n_act = n_act;
    G.m = m;
    G.directed = directed;
    G.has_graph = true;
    return PERCIS_OK;
}

// Sets the states of G. On a device context the pair distribution of
// Algorithm 2 (preprocessing) and the weights d_v, S_v are built on the
// device from k (a state-only update re-uses the graph's device copy and its
// arrays); the host receives C and d_hat. A host-only context only checks the
// states: C = 0 exactly when all states are equal.
static int graph_set_states(percis_ctx* c, GraphData& G, const uint16_t* k_in, uint32_t flags) {
    if (!G.has_graph) return fail(c, PERCIS_E_STATE, "load a graph first");
    if (!k_in) return fail(c, PERCIS_E_INVAL, "null states");
    if ((flags & PERCIS_DEVICE_PTRS) && c->host_only) return fail(c, PERCIS_E_INVAL, "device pointers on a host-only context");
    const int32_t n = G.n;
    if (c->host_only) {
        bool equal = true;
        for (int32_t v = 1; v < n && equal; v++) equal = k_in[v] == k_in[0];
        G.has_states = false;
        if (equal) return fail(c, PERCIS_E_DEGENERATE, "all percolation states are equal");
        G.has_states = true;
        return PERCIS_OK;
    }
    int rc = graph_upload(c, G, false);
    if (rc) return rc;
    G.has_states = false;
    G.states_on_device = false;
    if (!G.d_k) {
        if ((rc = dalloc(c, G.d_k, (size_t)n)) || (rc = dalloc(c, G.d_perm, (size_t)n + 1)) ||
            (rc = dalloc(c, G.d_kr, (size_t)n + 2)) || (rc = dalloc(c, G.d_W, (size_t)n + 2)) ||
            (rc = dalloc(c, G.d_P, (size_t)n + 1)) || (rc = dalloc(c, G.d_dv, (size_t)n)) ||
            (rc = dalloc(c, G.d_Sv, (size_t)n)) || (rc = dalloc(c, G.d_p, (size_t)n)) ||
            (rc = dalloc(c, G.d_red, 2))) {
            graph_free_states(G);
            return rc;
        }
        if (hipMalloc(&G.build_mem, (size_t)state_build_bytes(n)) != hipSuccess) {
            (void)hipGetLastError();
            G.build_mem = nullptr;
            graph_free_states(G);
            return fail(c, PERCIS_E_NOMEM, "cannot allocate the state-build scratch");
        }
    }
    HIPCHK(c, hipMemcpyAsync(G.d_k, k_in, sizeof(uint16_t) * n,
                             (flags & PERCIS_DEVICE_PTRS) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
    StateArrays a;
    a.n = n;
    a.k = G.d_k;
    a.newid = G.d_newid;
    a.perm = G.d_perm;
    a.kr = G.d_kr;
    a.W = G.d_W;
    a.P = G.d_P;
    a.d_v = G.d_dv;
    a.S_v = G.d_Sv;
    const uint64_t* res = nullptr;
    // The build rewrites the arrays a captured launch reads, whatever its
    // outcome (all-equal states leave them zero): no capture survives it.
    c->generation++;
    HIPCHK(c, launch_state_build(a, G.build_mem, &res, c->stream));
    uint64_t h[2] = {0, 0};
    HIPCHK(c, hipMemcpyAsync(h, res, sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (h[0] == 0) return fail(c, PERCIS_E_DEGENERATE, "all percolation states are equal");
    double dmax;
    std::memcpy(&dmax, &h[1], sizeof dmax);
    G.C = h[0];
    G.d_hat = std::max(1.0, dmax);
    G.has_states = true;
    G.states_on_device = true;
    c->generation++;  // a captured launch holds the old total weight
    return PERCIS_OK;
}

int set_device(percis_ctx* c) {
    if (c->host_only) return fail(c, PERCIS_E_STATE, "host-only context: no device work possible");
    HIPCHK(c, hipSetDevice(c->device));
    return PERCIS_OK;
}

// Uploads the graph if it is not on the device yet; with `states`, also
// checks that the states (built on the device by set_states) are there.
int graph_upload(percis_ctx* c, GraphData& G, bool states) {
    if (!G.has_graph) return fail(c, PERCIS_E_STATE, "load a graph first");
    if (states && !G.has_states) return fail(c, PERCIS_E_STATE, "set states first");
    int rc = set_device(c);
    if (rc) return rc;
    const int32_t n = G.n;
    const int64_t m = G.m;
    if (!G.graph_on_device) {
        // the in-row buffer (col itself if undirected) holds 2m entries: the
        // in-rows sorted by internal id, then the same rows in caller order
        if ((rc = dalloc(c, G.d_rp, (size_t)n + 1))) return rc;
        if ((rc = dalloc(c, G.d_col, (size_t)(G.directed ? m : 2 * m)))) return rc;
        HIPCHK(c, hipMemcpy(G.d_rp, G.h_rp.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice));
        if (m) HIPCHK(c, hipMemcpy(G.d_col, G.h_col.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice));
        if (G.directed) {
            if ((rc = dalloc(c, G.d_irp, (size_t)n + 1))) return rc;
            if ((rc = dalloc(c, G.d_icol, (size_t)(2 * m)))) return rc;
            HIPCHK(c, hipMemcpy(G.d_irp, G.h_irp.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice));
            if (m) HIPCHK(c, hipMemcpy(G.d_icol, G.h_icol.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice));
        } else {
            G.d_irp = G.d_rp;
            G.d_icol = G.d_col;
        }
        G.d_ccol = G.d_icol + m;
        if (m) HIPCHK(c, hipMemcpy(G.d_ccol, G.h_ccol.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice));
        if ((rc = dalloc(c, G.d_hits, (size_t)n))) return rc;
        if ((rc = dalloc(c, G.d_orig, (size_t)n))) return rc;
        if ((rc = dalloc(c, G.d_newid, (size_t)n))) return rc;
        HIPCHK(c, hipMemcpy(G.d_orig, G.h_orig.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(G.d_newid, G.h_newid.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
        G.graph_on_device = true;
    }
    if (states && !G.states_on_device) return fail(c, PERCIS_E_STATE, "set states first");
    return PERCIS_OK;
}

static DevGraph dev_graph(const GraphData& G) {
    DevGraph g;
    g.n = G.n;
    g.n_act = G.n_act;
    g.rp = G.d_rp;
    g.col = G.d_col;
    g.irp = G.d_irp;
    g.icol = G.d_icol;
    g.ccol = G.d_ccol;
    g.orig = G.d_orig;
    return g;
}

static DevCdf dev_cdf(const GraphData& G) {
    DevCdf d;
    d.n = G.n;
    d.C = G.C;
    d.perm = G.d_perm;
    d.kr = G.d_kr;
    d.W = G.d_W;
    d.P = G.d_P;
    return d;
}

static void free_slots(percis_ctx* c) {
    c->generation++;
    if (c->slot_mem) (void)hipFree(c->slot_mem);
    if (c->cslot_mem) (void)hipFree(c->cslot_mem);
    c->cslot_mem = nullptr;
    c->ncslots = 0;
    c->cslots = DevSlots{};
    if (c->wide_mem) (void)hipFree(c->wide_mem);
    c->wide_mem = nullptr;
    c->wide_slots = 0;
    c->wslots = WideSlots{};
    c->slot_mem = nullptr;
    c->nslots = 0;
    c->slot_act = 0;
    c->slots = DevSlots{};
}

constexpr int64_t kSlotBytesPerNode = (int64_t)sizeof(NodeRec) + 4 + 4 + 4 + 4;
constexpr int64_t kLdsPerCu = 160 * 1024;
constexpr int64_t kBitmapPlanes = 2;  // s-side and t-side visited
// DAG arcs a sample may record for its walk: per-node slots, which run the
// samples with large balls when compact slots are on, keep more (a walk step
// past a dropped arc scans its node's in-row instead)
constexpr int64_t kArcsPerSlot = 16384;
constexpr int64_t kArcsPerCompactSlot = 4096;
// Arcs into the other ball a level lists past its LDS list (8 bytes each,
// per slot); a meeting level with more rescans its rows for them.
constexpr int64_t kMeetListPerSlot = 8192;
// Samples per pair-kernel chunk by default (the pair, wide and handed-on lists
// take 16 bytes each per sample). Fewer chunks end fewer sampler tails: R-MAT
// 24 directed, 10^7 samples: 2^22 8.66M, 2^23 8.86M, 2^24 9.11M samples/s.
constexpr uint64_t kPairChunk = 1ull << 24;
constexpr uint64_t kMaxPairChunk = 1ull << 30;  // list entries index their chunk in 32 bits
// side rule of the bidirectional search: the s ball grows while its frontier
// degree sum is at most kBalance % of the t ball's (100: the smaller frontier)
constexpr uint32_t kBalance = 100;
constexpr int kMinBalance = 25, kMaxBalance = 400;
constexpr uint64_t kNoAllocChunk = 1ull << 16;  // samples per chunk of a no-allocation call
constexpr int64_t kWideSlots = 16;           // workgroups of the 128-bit path
constexpr int64_t kWideBytesPerNode = 4 + 16 + 4;
constexpr int kDeferBlock = 512;             // per-node slots' block while compact slots are on
// Compact slots' block unless the caller set one: R-MAT 24 directed, 10^7
// samples, 9.98M samples/s at 128 threads (1792 slots), 11.48M at 256 (1280).
constexpr int kCompactBlock = 256;
// A launch of at most kFewPerSlot samples per slot ends with its slowest
// sample chains, so it runs with kFewBlock threads per sample (fewer slots).
// An estimate at eps = 0.01 on R-MAT 18 (about 7K samples per phase): 3.5 ms
// at 128 threads, 1.6 ms at 512; at eps = 0.005 (24K): 4.2 and 2.8 ms; at
// eps = 0.001 (481K), 512 threads are slower (23 against 15.6 ms).
constexpr uint64_t kFewPerSlot = 16;
constexpr int kFewBlock = 512;
// Share of free device memory the per-node slots may take by default. Only
// graphs too large for slots to fill the device reach it; there the per-node
// slots run the samples compact slots hand on (R-MAT 24 directed: 7.75M
// samples/s at 60 %, 8.38M at 78 %).
constexpr double kScratchFraction = 0.8;

static int64_t bitmap_words(int64_t act) { return ((std::max<int64_t>(act, 1) + 31) / 32 + 63) / 64 * 64; }

// Bytes of one per-node slot for graphs of up to `stride` nodes with arcs
// (stride a multiple of 64): records and queues, the bitmap planes and the
// DAG-arc list.
static int64_t node_slot_bytes(int64_t stride, int64_t words) {
    return stride * kSlotBytesPerNode + 8 + kBitmapPlanes * words * 4 + kArcsPerSlot * (int64_t)sizeof(DagArc) +
           kMeetListPerSlot * 8;
}

// ns per-node slots laid out from p (node_slot_bytes each, all zero before use).
static DevSlots node_slots_at(char* p, int64_t ns, int64_t stride, int64_t words) {
    DevSlots s{};
    s.stride = stride;
    s.words = words;
    const int64_t cnt = ns * stride;
    s.rec = (NodeRec*)p; p += cnt * (int64_t)sizeof(NodeRec);
    s.q_s = (int32_t*)p; p += cnt * 4;
    s.q_t = (int32_t*)p; p += cnt * 4;
    s.q_d = (int32_t*)p; p += cnt * 4;
    s.tls = (int32_t*)p; p += ns * (stride + 2) * 4;
    s.bm = (uint32_t*)p; p += ns * kBitmapPlanes * words * 4;
    s.mlx = (uint32_t*)p; p += ns * kMeetListPerSlot * 8;
    s.mlxcap = (int32_t)kMeetListPerSlot;
    s.arcs = (DagArc*)p;
    s.acap = (int32_t)kArcsPerSlot;
    return s;
}

// Bytes of one compact slot (records by table position, whatever the graph).
static int64_t compact_slot_bytes() {
    const int64_t cap = sampler_table_cap(true);
    return 2 * cap * (int64_t)sizeof(CRec) + 4 * cap * 4 + (cap + 2) * 4 + kArcsPerCompactSlot * (int64_t)sizeof(DagArc) +
           kMeetListPerSlot * 8;
}

// nc compact slots laid out from p (compact_slot_bytes each, all zero before use).
static DevSlots compact_slots_at(char* p, int64_t nc) {
    const int64_t cap = sampler_table_cap(true);
    DevSlots d{};
    d.stride = cap;
    d.crec = (CRec*)p; p += nc * 2 * cap * (int64_t)sizeof(CRec);
    d.q_s = (int32_t*)p; p += nc * cap * 4;
    d.q_t = (int32_t*)p; p += nc * cap * 4;
    d.q_d = (int32_t*)p; p += nc * 2 * cap * 4;
    d.tls = (int32_t*)p; p += nc * (cap + 2) * 4;
    d.mlx = (uint32_t*)p; p += nc * kMeetListPerSlot * 8;
    d.mlxcap = (int32_t)kMeetListPerSlot;
    d.arcs = (DagArc*)p;
    d.acap = (int32_t)kArcsPerCompactSlot;
    return d;
}

// nw slots of the 128-bit path laid out from p (kWideBytesPerNode per node
// each; before use the counts must be zero and the distances -1).
static WideSlots wide_slots_at(char* p, int64_t nw, int64_t stride, unsigned long long* work) {
    WideSlots w{};
    w.stride = stride;
    w.sigma = (unsigned __int128*)p; p += nw * stride * 16;
    w.dist = (int32_t*)p; p += nw * stride * 4;
    w.queue = (int32_t*)p;
    w.work = work;
    return w;
}

// The launch shape for graphs of up to `act` nodes with arcs, given the
// context's options.
static int pick_shape(percis_ctx* c, int64_t act, SamplerShape* out, int* occ_out) {
    const int64_t words = bitmap_words(act);
    SamplerShape sh{};
    sh.block = c->opt_block ? (int)c->opt_block : 128;
    (void)words;
    const int64_t lds_need = sampler_table_lds(false, sh.block);
    const bool fits = lds_need + sampler_static_lds() <= kLdsPerCu;
    if (c->opt_bitmaps == 2 && !fits)
        return fail(c, PERCIS_E_INVAL, "visited-set tables do not fit in LDS");
    if (c->opt_compact == 2 && c->opt_bitmaps == 1)
        return fail(c, PERCIS_E_INVAL, "compact slots need the LDS tables (bitmaps option 0 or 2)");
    if (c->opt_bitmaps == 0 && c->opt_compact == 2) {
        sh.lds_sets = fits;  // compact slots index their records by table position
    } else if (c->opt_bitmaps == 0) {
        // LDS tables unless they cost resident samples: the sampler is
        // latency-bound, so samples in flight per CU matter more than where
        // the visited sets live
        SamplerShape dev = sh, lds = sh;
        lds.lds_sets = true;
        lds.lds_bytes = lds_need;
        sh.lds_sets = fits && sampler_occupancy(lds) >= sampler_occupancy(dev);
    } else {
        sh.lds_sets = c->opt_bitmaps == 2;
    }
    sh.lds_bytes = sh.lds_sets ? lds_need : 0;
    const int occ = sampler_occupancy(sh);
    if (occ <= 0)
        return fail(c, PERCIS_E_DEVICE, "sampler shape (block %d, visited sets in %s) cannot launch", sh.block,
                    sh.lds_sets ? "LDS tables" : "device bitmaps");
    *out = sh;
    *occ_out = occ;
    return PERCIS_OK;
}

// Allocates the per-slot scratch for graphs of up to `act` nodes with arcs:
// one slot per resident workgroup, capped by a memory budget. Keeps the
// current scratch if it is large enough.
static int ensure_slots(percis_ctx* c, int64_t act) {
    act = std::max<int64_t>(act, 1);
    if (c->slot_mem && act <= c->slot_act) return PERCIS_OK;
    if (c->slot_mem) {
        if (c->stream) HIPCHK(c, hipStreamSynchronize(c->stream)); else HIPCHK(c, hipDeviceSynchronize());
        free_slots(c);
    }
    SamplerShape sh;
    int occ = 0;
    int rc = pick_shape(c, act, &sh, &occ);
    if (rc) return rc;
    const int64_t stride = (act + 63) / 64 * 64;
    const int64_t words = bitmap_words(act);
    const int64_t per_slot = node_slot_bytes(stride, words);
    size_t free_b = 0, total_b = 0;
    HIPCHK(c, hipMemGetInfo(&free_b, &total_b));
    const int64_t budget =
        c->opt_scratch_mb > 0 ? c->opt_scratch_mb * (1ll << 20) : (int64_t)((double)free_b * kScratchFraction);
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
    const DevSlots s = node_slots_at((char*)mem, ns, stride, words);
    // scratch of the 128-bit path: distances -1, counts 0
    const int64_t wbudget = std::max<int64_t>(budget / 8, stride * kWideBytesPerNode);
    int64_t nw = std::max<int64_t>(1, std::min<int64_t>(kWideSlots, wbudget / (stride * kWideBytesPerNode)));
    void* wmem = nullptr;
    while (nw >= 1) {
        e = hipMalloc(&wmem, (size_t)(nw * stride * kWideBytesPerNode));
        if (e == hipSuccess) break;
        (void)hipGetLastError();
        nw /= 2;
    }
    if (e != hipSuccess || !wmem) {
        (void)hipFree(mem);
        return fail(c, PERCIS_E_NOMEM, "cannot allocate the 128-bit path's scratch");
    }
    const WideSlots w = wide_slots_at((char*)wmem, nw, stride, c->d_work + 3);
    if (launch_fill_u8(w.sigma, nw * stride * 16, c->stream) != hipSuccess ||
        launch_fill_u32((uint32_t*)w.dist, 0xFFFFFFFFu, nw * stride, c->stream) != hipSuccess) {
        (void)hipFree(mem);
        (void)hipFree(wmem);
        return fail(c, PERCIS_E_DEVICE, "scratch clear failed");
    }
    c->slot_mem = mem;
    c->slots = s;
    c->nslots = (int)ns;
    c->slot_act = act;
    c->shape = sh;
    c->wide_mem = wmem;
    c->wide_slots = (int)nw;
    c->wslots = w;

    // Compact slots: records by table position, so a slot costs a fixed
    // ~150 KB whatever the graph; the per-node slots above then only redo the
    // samples a table cannot hold. Auto: when the per-node slots are too few
    // (memory) to fill the device.
    const bool compact = sh.lds_sets && (c->opt_compact == 2 || (c->opt_compact == 0 && ns < want));
    if (compact) {
        SamplerShape cs = sh;
        cs.compact = true;
        if (c->opt_block == 0) cs.block = kCompactBlock;
        cs.lds_bytes = sampler_table_lds(true, cs.block);
        const int cocc = sampler_occupancy(cs);
        const int64_t cper = compact_slot_bytes();
        int64_t nc = c->opt_slots > 0 ? c->opt_slots : (int64_t)std::max(c->cu_count, 1) * cocc;
        void* cmem = nullptr;
        e = hipErrorOutOfMemory;
        while (cocc > 0 && nc >= 1) {
            e = hipMalloc(&cmem, (size_t)(nc * cper));
            if (e == hipSuccess) break;
            (void)hipGetLastError();
            nc /= 2;
        }
        if (e != hipSuccess || !cmem || launch_fill_u8(cmem, nc * cper, c->stream) != hipSuccess) {
            if (cmem) (void)hipFree(cmem);
            (void)hipGetLastError();
            free_slots(c);
            return fail(c, PERCIS_E_NOMEM, "cannot allocate compact slots");
        }
        const DevSlots d = compact_slots_at((char*)cmem, nc);
        c->cslot_mem = cmem;
        c->cslots = d;
        c->ncslots = (int)nc;
        c->cshape = cs;
        // the per-node slots now see only samples with large balls: more
        // threads per sample pay off there
        SamplerShape big = sh;
        big.block = c->opt_defer_block > 0 ? (int)c->opt_defer_block : kDeferBlock;
        big.lds_bytes = sampler_table_lds(false, big.block);
        if (sampler_occupancy(big) > 0) c->shape = big;
    }
    return PERCIS_OK;
}

// VertexDiamUB (Algorithm 1) on the device, once per graph: D_override if
// set, else the cached device result (the graph never changes after loading).
// Undirected: per connected component, a BFS from its smallest node u; the
// component's shortest paths have at most min(|comp| - 2, 2 ecc(u) - 1)
// internal nodes. Directed: largest weakly connected component size - 2.
int vertex_diam_ub(percis_ctx* c, GraphData& G, int64_t* D) {
    if (G.D_override >= 0) {
        *D = G.D_override;
        return PERCIS_OK;
    }
    if (G.D_cached >= 0) {
        *D = G.D_cached;
        return PERCIS_OK;
    }
    int rc = graph_upload(c, G, false);
    if (rc) return rc;
    void* scratch = nullptr;
    if (hipMalloc(&scratch, (size_t)diam_scratch_bytes(G.n_act, G.m)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, PERCIS_E_NOMEM, "cannot allocate the VertexDiamUB scratch");
    }
    int64_t d = 0;
    int32_t levels = 0, rounds = 0;
    const hipError_t e =
        run_vertex_diam_ub(G.d_rp, G.d_col, G.d_orig, G.n_act, G.m, G.directed, scratch, &d, &levels, &rounds,
                           c->stream);
    (void)hipFree(scratch);
    if (e != hipSuccess) return fail(c, PERCIS_E_DEVICE, "VertexDiamUB: %s", hipGetErrorString(e));
    G.D_cached = d;
    *D = d;
    return PERCIS_OK;
}

// Theorem 1 with the constants of Algorithm 1, as a function of x.
static double sample_bound(double x, double d, double rho, double eps, double delta) {
    const double gx = x * (d - x);
    const double y = eps * d / gx;
    const double hy = (1.0 + y) * std::log1p(y) - y;
    return d * d * std::log(4.0 * d * rho / (x * delta)) / (gx * hy);
}

// sup over (0, x_hat]: a log-spaced scan over 16 decades, then golden-section
// refinement in log x around the best scan point, then the end point x_hat.
static double sample_size_sup(double d, double rho, double v, double eps, double delta, double* x_hat_out) {
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

// Propositions 2 and 3 and Theorem 1 (with the constants of Algorithm 1)
// from the phase-1 |I| sums and hits (device); I->D must be set. The bound of
// Proposition 3 is non-decreasing in p1 = d_v h_v / l1 (in floating point
// too: every operation in it is monotone), so its maximum over v is its value
// at max_v d_v h_v, which a device reduction provides.
int phase1_bounds(percis_ctx* c, const GraphData& G, uint64_t l1u, uint64_t sum_I, uint64_t sum_I2,
                  const uint32_t* d_hits1, double eps, double delta, percis_estimate_info* I, hipStream_t stream) {
    HIPCHK(c, launch_fill_u32((uint32_t*)G.d_red, 0u, 2, stream));
    HIPCHK(c, launch_hit_weight_max(G.d_dv, d_hits1, G.n, G.d_red, stream));
    uint64_t bits = 0;
    HIPCHK(c, hipMemcpyAsync(&bits, G.d_red, sizeof bits, hipMemcpyDeviceToHost, stream));
    HIPCHK(c, hipStreamSynchronize(stream));
    double hw;
    std::memcpy(&hw, &bits, sizeof hw);
    const double l1 = (double)l1u;
    I->l1 = l1u;
    I->d_hat = G.d_hat;
    I->rho_tilde = (double)sum_I / l1;
    const unsigned __int128 num = (unsigned __int128)l1u * sum_I2 - (unsigned __int128)sum_I * sum_I;
    I->Lambda = (double)num / (l1 * (l1 - 1.0));
    const double L8 = std::log(8.0 / delta), L4 = std::log(4.0 / delta);
    I->rho_hat = I->rho_tilde + std::sqrt(2.0 * I->Lambda * L8 / l1) + 7.0 * (double)I->D * L8 / (3.0 * (l1 - 1.0));
    const double p1 = hw / l1;
    const double vmax = p1 + std::sqrt(2.0 * p1 * L4 / l1) + L4 / (3.0 * l1);
    I->v_hat = G.d_hat * G.d_hat * vmax;
    const double lb = sample_size_sup(G.d_hat, I->rho_hat, I->v_hat, eps, delta, &I->x_hat);
    I->l = lb < 4294967295.0 ? (uint64_t)std::ceil(lb) : ~0ull;
    return PERCIS_OK;
}

// p_out[v] = d_v h_v / l (Algorithm 1's estimate), computed on the device and
// copied to the host array p_out.
int estimates_to_host(percis_ctx* c, const GraphData& G, const uint32_t* d_hits, uint64_t l, double* p_out,
                      hipStream_t stream) {
    HIPCHK(c, launch_estimates(G.d_dv, d_hits, G.n, l, G.d_p, stream));
    HIPCHK(c, hipMemcpyAsync(p_out, G.d_p, sizeof(double) * G.n, hipMemcpyDeviceToHost, stream));
    HIPCHK(c, hipStreamSynchronize(stream));
    return PERCIS_OK;
}

static void stats_from_dev(const DevStats& hs, percis_stats* st) {
    std::memset(st, 0, sizeof *st);
    st->samples = hs.samples;
    st->reachable = hs.reachable;
    st->sum_I = hs.sum_I;
    st->sum_I2 = hs.sum_I2;
    st->overflow = hs.overflow;
    st->first_overflow = hs.first_overflow;
}

// What a launch over a task list needs before its kernels are enqueued:
// graphs and slots on the device, the task table uploaded to `table` (stats
// to `tstats`) from `ht`, which must outlive the copy (the caller's stream
// synchronisation), list buffers of one chunk.
struct LaunchPlan {
    int nt = 0;
    int64_t max_n = 1;
    uint64_t total = 0, chunk = 1;
    size_t nchunks = 0;
};

static int plan_tasks(percis_ctx* c, const std::vector<TaskSpec>& tasks, DevTask* table, DevStats* tstats,
                      std::vector<DevTask>& ht, LaunchPlan* lp) {
    int rc = set_device(c);
    if (rc) return rc;
    const int nt = (int)tasks.size();
    int64_t max_act = 1, max_n = 1;
    uint64_t total = 0;
    for (const TaskSpec& t : tasks) {
        GraphData& G = *c->graphs[t.graph];
        if ((rc = graph_upload(c, G, true))) return rc;
        max_act = std::max<int64_t>(max_act, G.n_act);
        max_n = std::max<int64_t>(max_n, G.n);
        total += t.count;
    }
    if ((rc = ensure_slots(c, max_act))) return rc;
    ht.assign(nt, DevTask{});
    uint64_t off = 0;
    for (int i = 0; i < nt; i++) {
        const TaskSpec& t = tasks[i];
        GraphData& G = *c->graphs[t.graph];
        DevTask& d = ht[i];
        std::memset(&d, 0, sizeof d);
        d.g = dev_graph(G);
        d.cdf = dev_cdf(G);
        d.first = t.first;
        d.count = t.count;
        d.seed = t.seed;
        d.phase = t.phase;
        d.hits = t.d_hits;
        d.stats = tstats + i;
        d.offset = off;
        d.clear_hits = t.accumulate ? 0u : 1u;
        off += t.count;
    }
    HIPCHK(c, hipMemcpyAsync(table, ht.data(), sizeof(DevTask) * nt, hipMemcpyHostToDevice, c->stream));
    // The launch runs in chunks of at most kPairChunk samples: the pair kernel
    // draws a chunk's pairs and lists those that need a search, then the
    // sampler works through the list.
    const uint64_t chunk =
        std::max<uint64_t>(1, std::min<uint64_t>(total, c->opt_pair_chunk > 0 ? (uint64_t)c->opt_pair_chunk : kPairChunk));
    if (chunk > c->pair_cap) {
        if (c->stream) HIPCHK(c, hipStreamSynchronize(c->stream));
        if ((rc = dalloc(c, c->d_pairs, (size_t)chunk))) return rc;
        if ((rc = dalloc(c, c->d_wide, (size_t)chunk))) return rc;
        if ((rc = dalloc(c, c->d_big, (size_t)chunk))) return rc;
        c->pair_cap = chunk;
        c->generation++;
    }
    lp->nt = nt;
    lp->max_n = max_n;
    lp->total = total;
    lp->chunk = chunk;
    lp->nchunks = (size_t)((total + chunk - 1) / chunk);
    return PERCIS_OK;
}

// The device buffers one launch runs on: the context's own (ctx_bufs), or
// views into the library's static scratch (the no-allocation entry point).
struct LaunchBufs {
    DevStats* stats = nullptr;            // launch-wide counters
    unsigned long long* work = nullptr;   // [6], as percis_ctx::d_work
    PairRec *pairs = nullptr, *wide = nullptr, *big = nullptr;  // one chunk's lists
    DevSlots slots{};                     // per-node slots
    SamplerShape shape{};
    int nslots = 0;
    DevSlots cslots{};                    // compact slots (ncslots = 0: none)
    SamplerShape cshape{};
    int ncslots = 0;
    WideSlots wslots{};                   // the 128-bit path
    int wide_slots = 0;
};

static LaunchBufs ctx_bufs(const percis_ctx* c) {
    LaunchBufs b;
    b.stats = c->d_stats;
    b.work = c->d_work;
    b.pairs = c->d_pairs;
    b.wide = c->d_wide;
    b.big = c->d_big;
    b.slots = c->slots;
    b.shape = c->shape;
    b.nslots = c->nslots;
    b.cslots = c->cslots;
    b.cshape = c->cshape;
    b.ncslots = c->ncslots;
    b.wslots = c->wslots;
    b.wide_slots = c->wide_slots;
    return b;
}

// Enqueues the launch's kernels on `stream`: task clearing, then per chunk
// the pair kernel, the sampler (compact slots first when they are on), the
// 128-bit path. Kernels only, so that the sequence can be captured; with
// `timed`, per-chunk events bracket the pair kernel and the rest.
static int enqueue_tasks(percis_ctx* c, const LaunchPlan& lp, const DevTask* table, const LaunchBufs& B,
                         hipStream_t stream, bool timed) {
    if (timed) {
        while (c->chunk_ev.size() < 4 * lp.nchunks) {
            hipEvent_t e;
            HIPCHK(c, hipEventCreate(&e));
            c->chunk_ev.push_back(e);
        }
    }
    HIPCHK(c, launch_clear_tasks(table, lp.nt, lp.max_n, stream));
    HIPCHK(c, launch_init_stats(B.stats, B.work, stream));
    SampleLaunch a{};
    a.tasks = table;
    a.ntasks = lp.nt;
    a.pairs = B.pairs;
    a.work = B.work;
    a.npairs = B.work + 1;
    a.stats = B.stats;
    a.balance = c->opt_balance > 0 ? (uint32_t)c->opt_balance : kBalance;
    // the per-node shape of this launch: wider workgroups for a small launch
    // unless the caller fixed the shape
    SamplerShape shape = B.shape;
    int nsl = B.nslots;
    if (B.ncslots == 0 && c->opt_block == 0 && c->opt_slots == 0 && shape.block < kFewBlock &&
        lp.total <= (uint64_t)B.nslots * kFewPerSlot) {
        SamplerShape wide = shape;
        wide.block = kFewBlock;
        wide.lds_bytes = wide.lds_sets ? sampler_table_lds(false, kFewBlock) : 0;
        const int occ = sampler_occupancy(wide);
        if (occ > 0) {
            shape = wide;
            nsl = (int)std::min<int64_t>(B.nslots, (int64_t)std::max(c->cu_count, 1) * occ);
        }
    }
    a.slots = (int)std::min<uint64_t>((uint64_t)nsl, lp.chunk);
    a.wide = B.wide;
    a.nwide = B.work + 2;
    a.big = B.big;
    a.nbig = B.work + 4;
    a.big_work = B.work + 5;
    for (size_t i = 0; i < lp.nchunks; i++) {
        a.base = (uint64_t)i * lp.chunk;
        a.count = std::min<uint64_t>(lp.chunk, lp.total - a.base);
        if (timed) HIPCHK(c, hipEventRecord(c->chunk_ev[4 * i], stream));
        HIPCHK(c, launch_pairs(a, stream));
        if (timed) HIPCHK(c, hipEventRecord(c->chunk_ev[4 * i + 1], stream));
        if (B.ncslots > 0) {
            // compact slots first; the samples they hand on go to the per-node slots
            SampleLaunch ca = a;
            ca.slots = (int)std::min<uint64_t>((uint64_t)B.ncslots, lp.chunk);
            HIPCHK(c, launch_sampler(B.cslots, ca, B.cshape, stream));
            if (timed) HIPCHK(c, hipEventRecord(c->chunk_ev[4 * i + 2], stream));
            SampleLaunch da = a;
            da.pairs = B.big;
            da.npairs = a.nbig;
            da.work = a.big_work;
            da.slots = (int)std::min<uint64_t>((uint64_t)B.nslots, lp.chunk);
            HIPCHK(c, launch_sampler(B.slots, da, B.shape, stream));
        } else {
            HIPCHK(c, launch_sampler(B.slots, a, shape, stream));
            if (timed) HIPCHK(c, hipEventRecord(c->chunk_ev[4 * i + 2], stream));
        }
        HIPCHK(c, launch_wide(a, B.wslots, B.wide_slots, stream));
        if (timed) HIPCHK(c, hipEventRecord(c->chunk_ev[4 * i + 3], stream));
    }
    return PERCIS_OK;
}

// The launch-wide work counters, phase times and device times of a finished
// launch into agg.
static void launch_fields(const percis_ctx* c, const DevStats& hl, double ms, double pair_ms, const double* pass_ms,
                          percis_stats* agg) {
    agg->edges = hl.edges;
    agg->sigma_adds = hl.sigma_adds;
    agg->vertices_expanded = hl.vexp;
    agg->vertices_discovered = hl.vdisc;
    agg->spilled = hl.spills;
    agg->deferred = hl.deferred;
    agg->kernel_ms = ms;
    agg->pair_ms = pair_ms;
    if (pass_ms) {
        agg->pass_ms[0] = pass_ms[0];
        agg->pass_ms[1] = pass_ms[1];
    }
    for (int i = 0; i < 5; i++) agg->phase_ms[i] = c->wall_hz > 0 ? (double)hl.phase_ticks[i] / c->wall_hz * 1e3 : 0.0;
}

// The status of a finished launch: a broken walk, then overflow.
static int launch_status(percis_ctx* c, const DevStats& hl, const percis_stats& agg) {
    if (hl.walk_errors)
        return fail(c, PERCIS_E_DEVICE,
                    "%llu sample(s) whose path walk found no predecessor (a search invariant broke); they added no hits",
                    (unsigned long long)hl.walk_errors);
    if (agg.overflow)
        return fail(c, PERCIS_E_SIGMA_OVERFLOW, "%llu sample(s) with sigma_st >= 2^64, first index %llu",
                    (unsigned long long)agg.overflow, (unsigned long long)agg.first_overflow);
    return PERCIS_OK;
}

// Reads a finished launch's statistics (`tstats`, per task, and the
// launch-wide counters) and checks that every task ran all its samples.
static int tally_tasks(percis_ctx* c, const std::vector<TaskSpec>& tasks, const DevStats* hts, const DevStats& hl,
                       double ms, double pair_ms, const double* pass_ms, std::vector<percis_stats>* out,
                       percis_stats* launch);

static int collect_tasks(percis_ctx* c, const std::vector<TaskSpec>& tasks, const DevStats* tstats,
                         const DevStats* lstats, double ms, double pair_ms, const double* pass_ms,
                         std::vector<percis_stats>* out, percis_stats* launch) {
    const int nt = (int)tasks.size();
    std::vector<DevStats> hts(nt);
    DevStats hl{};
    HIPCHK(c, hipMemcpyAsync(hts.data(), tstats, sizeof(DevStats) * nt, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(&hl, lstats, sizeof hl, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return tally_tasks(c, tasks, hts.data(), hl, ms, pair_ms, pass_ms, out, launch);
}

// The statistics of a finished launch, already on the host: per task (hts)
// and launch-wide (hl).
static int tally_tasks(percis_ctx* c, const std::vector<TaskSpec>& tasks, const DevStats* hts, const DevStats& hl,
                       double ms, double pair_ms, const double* pass_ms, std::vector<percis_stats>* out,
                       percis_stats* launch) {
    const int nt = (int)tasks.size();
    percis_stats agg{};
    agg.first_overflow = ~0ull;
    if (out) out->resize(nt);
    for (int i = 0; i < nt; i++) {
        percis_stats st;
        stats_from_dev(hts[i], &st);
        st.kernel_ms = ms;
        st.pair_ms = pair_ms;
        if (out) (*out)[i] = st;
        if (st.samples != tasks[i].count)
            return fail(c, PERCIS_E_DEVICE, "task %d: sampler processed %llu of %llu samples", i,
                        (unsigned long long)st.samples, (unsigned long long)tasks[i].count);
        agg.samples += st.samples;
        agg.reachable += st.reachable;
        agg.sum_I += st.sum_I;
        agg.sum_I2 += st.sum_I2;
        agg.overflow += st.overflow;
        agg.first_overflow = std::min(agg.first_overflow, st.first_overflow);
    }
    launch_fields(c, hl, ms, pair_ms, pass_ms, &agg);
    if (launch) *launch = agg;
    return launch_status(c, hl, agg);
}

// Runs `tasks` in one persistent launch on the context's stream and waits for
// it. `out` (optional) receives each task's sample statistics; `launch`
// (optional) their sums with the launch-wide work counters, phase times and
// kernel time.
int run_tasks(percis_ctx* c, const std::vector<TaskSpec>& tasks, std::vector<percis_stats>* out, percis_stats* launch) {
    const int nt = (int)tasks.size();
    int rc = set_device(c);
    if (rc) return rc;
    if (nt > c->task_cap) {
        if (c->stream) HIPCHK(c, hipStreamSynchronize(c->stream));
        if ((rc = dalloc(c, c->d_tasks, (size_t)nt))) return rc;
        if ((rc = dalloc(c, c->d_task_stats, (size_t)nt))) return rc;
        c->task_cap = nt;
    }
    LaunchPlan lp;
    std::vector<DevTask> ht;
    if ((rc = plan_tasks(c, tasks, c->d_tasks, c->d_task_stats, ht, &lp))) return rc;
    if ((rc = enqueue_tasks(c, lp, c->d_tasks, ctx_bufs(c), c->stream, true))) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double ms = 0.0, pair_ms = 0.0, pass_ms[2] = {0.0, 0.0};
    for (size_t i = 0; i < lp.nchunks; i++) {
        float a_ms = 0.f, b_ms = 0.f, c_ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&a_ms, c->chunk_ev[4 * i], c->chunk_ev[4 * i + 1]));
        HIPCHK(c, hipEventElapsedTime(&b_ms, c->chunk_ev[4 * i + 1], c->chunk_ev[4 * i + 2]));
        HIPCHK(c, hipEventElapsedTime(&c_ms, c->chunk_ev[4 * i + 2], c->chunk_ev[4 * i + 3]));
        pair_ms += a_ms;
        pass_ms[0] += b_ms;
        pass_ms[1] += c_ms;
        ms += b_ms + c_ms;
    }
    return collect_tasks(c, tasks, c->d_task_stats, c->d_stats, ms, pair_ms, pass_ms, out, launch);
}

int async_launch_init(percis_ctx* c, AsyncLaunch* a, int cap) {
    *a = AsyncLaunch{};
    a->cap = cap;
    int rc;
    if ((rc = dalloc(c, a->d_tasks, (size_t)cap)) || (rc = dalloc(c, a->d_tstats, (size_t)cap)) ||
        (rc = dalloc(c, a->d_lstats, 1)))
        return rc;
    if (hipHostMalloc((void**)&a->h_tstats, sizeof(DevStats) * cap) != hipSuccess ||
        hipHostMalloc((void**)&a->h_lstats, sizeof(DevStats)) != hipSuccess)
        return fail(c, PERCIS_E_NOMEM, "cannot allocate pinned statistics buffers");
    HIPCHK(c, hipEventCreate(&a->start));
    HIPCHK(c, hipEventCreate(&a->end));
    HIPCHK(c, hipEventCreate(&a->done));
    return PERCIS_OK;
}

void async_launch_free(AsyncLaunch* a) {
    dfree(a->d_tasks);
    dfree(a->d_tstats);
    dfree(a->d_lstats);
    if (a->h_tstats) (void)hipHostFree(a->h_tstats);
    if (a->h_lstats) (void)hipHostFree(a->h_lstats);
    a->h_tstats = a->h_lstats = nullptr;
    for (hipEvent_t* e : {&a->start, &a->end, &a->done})
        if (*e) (void)hipEventDestroy(*e), *e = nullptr;
}

// Enqueues a launch of `tasks` on the context's stream and returns at once:
// the kernels, then copies of the statistics into the pinned buffers, then
// the `done` event. Launches on one stream run one after the other.
int launch_tasks_async(percis_ctx* c, const std::vector<TaskSpec>& tasks, AsyncLaunch* a) {
    const int nt = (int)tasks.size();
    if (nt < 1 || nt > a->cap) return fail(c, PERCIS_E_INVAL, "%d tasks in one launch (1 .. %d)", nt, a->cap);
    int rc = set_device(c);
    if (rc) return rc;
    a->tasks = tasks;
    LaunchPlan lp;
    if ((rc = plan_tasks(c, tasks, a->d_tasks, a->d_tstats, a->table, &lp))) return rc;
    LaunchBufs B = ctx_bufs(c);
    B.stats = a->d_lstats;
    HIPCHK(c, hipEventRecord(a->start, c->stream));
    if ((rc = enqueue_tasks(c, lp, a->d_tasks, B, c->stream, false))) return rc;
    HIPCHK(c, hipEventRecord(a->end, c->stream));
    HIPCHK(c, hipMemcpyAsync(a->h_tstats, a->d_tstats, sizeof(DevStats) * nt, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(a->h_lstats, a->d_lstats, sizeof(DevStats), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipEventRecord(a->done, c->stream));
    return PERCIS_OK;
}

// Waits for a launch of launch_tasks_async and reads its statistics (as
// run_tasks reports them).
int finish_tasks_async(percis_ctx* c, AsyncLaunch* a, std::vector<percis_stats>* out, percis_stats* launch) {
    HIPCHK(c, hipEventSynchronize(a->done));
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, a->start, a->end));
    return tally_tasks(c, a->tasks, a->h_tstats, *a->h_lstats, ms, 0.0, nullptr, out, launch);
}

GraphData* get_graph(percis_ctx* c, int32_t id) {
    if (id < 0 || id >= (int32_t)c->graphs.size() || !c->graphs[id]) return nullptr;
    return c->graphs[id];
}

// Algorithm 1 on graph `id`: D, phase 1, the bounds, phase 2, the estimate.
// Algorithm 1 (di = false), or PercIS-DI (di = true: no phase 1, rho_hat = D,
// v_hat = d_hat^2 / 4).
static int estimate_graph(percis_ctx* c, int32_t id, double eps, double delta, uint64_t seed, double* p_out,
                          percis_estimate_info* info, bool di = false) {
    GraphData* G = get_graph(c, id);
    if (!G) return fail(c, PERCIS_E_INVAL, "no graph %d", id);
    if (!G->has_graph || !G->has_states) return fail(c, PERCIS_E_STATE, "load a graph and set states first");
    if (!(eps > 0 && eps < 1) || !(delta > 0 && delta < 1) || !p_out)
        return fail(c, PERCIS_E_INVAL, "need 0 < eps < 1, 0 < delta < 1 and an output array");
    int rc = graph_upload(c, *G, true);
    if (rc) return rc;
    auto t0 = std::chrono::steady_clock::now();
    percis_estimate_info I{};
    if ((rc = vertex_diam_ub(c, *G, &I.D))) return rc;
    I.d_hat = G->d_hat;
    std::vector<TaskSpec> one(1);
    percis_stats s1{};
    if (di) {
        I.rho_hat = (double)I.D;
        I.v_hat = I.d_hat * I.d_hat / 4.0;
        auto tb = std::chrono::steady_clock::now();
        const double lb = sample_size_sup(I.d_hat, I.rho_hat, I.v_hat, eps, delta, &I.x_hat);
        I.l = lb < 4294967295.0 ? (uint64_t)std::ceil(lb) : ~0ull;
        I.bounds_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tb).count();
    } else {
        I.l1 = (uint64_t)std::ceil(std::max(1000.0, std::log(1.0 / delta) / eps));
        std::vector<percis_stats> ts;
        one[0] = TaskSpec{id, 1, 0, I.l1, seed, G->d_hits, false};
        rc = run_tasks(c, one, &ts, &s1);
        if (rc != PERCIS_OK) {
            I.overflow = s1.overflow;
            if (info) *info = I;
            return rc;
        }
        I.phase1_ms = s1.kernel_ms;
        auto tb = std::chrono::steady_clock::now();
        if ((rc = phase1_bounds(c, *G, I.l1, ts[0].sum_I, ts[0].sum_I2, G->d_hits, eps, delta, &I, c->stream)))
            return rc;
        auto te = std::chrono::steady_clock::now();
        I.bounds_ms = std::chrono::duration<double, std::milli>(te - tb).count();
    }
    if (I.l >= 4294967295ull) {
        if (info) *info = I;
        return fail(c, PERCIS_E_TOO_LARGE, "phase-2 sample size exceeds 2^32 - 1");
    }

    one[0] = TaskSpec{id, 2, 0, I.l, seed, G->d_hits, false};
    percis_stats s2{};
    rc = run_tasks(c, one, nullptr, &s2);
    I.overflow = s1.overflow + s2.overflow;
    I.phase2_ms = s2.kernel_ms;
    if (rc != PERCIS_OK) {
        if (info) *info = I;
        return rc;
    }
    if ((rc = estimates_to_host(c, *G, G->d_hits, I.l, p_out, c->stream))) return rc;
    I.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = I;
    return PERCIS_OK;
}

static int sync_ctx(percis_ctx* c) {
    if (c->host_only) return PERCIS_OK;
    int rc = set_device(c);
    if (rc) return rc;
    if (c->stream) HIPCHK(c, hipStreamSynchronize(c->stream)); else HIPCHK(c, hipDeviceSynchronize());
    return PERCIS_OK;
}

static int64_t max_active(const percis_ctx* c) {
    int64_t act = 0;
    for (const GraphData* G : c->graphs)
        if (G && G->has_graph) act = std::max<int64_t>(act, G->n_act);
    return act;
}

}  // namespace percis

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
    percis_ctx* c = nullptr;
    if (device == PERCIS_HOST_ONLY) {
        c = new (std::nothrow) percis_ctx();
        if (!c) return PERCIS_E_NOMEM;
        c->host_only = true;
        c->device = -1;
    } else {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return PERCIS_E_DEVICE;
        if (device < 0 || device >= ndev) return PERCIS_E_INVAL;
        c = new (std::nothrow) percis_ctx();
        if (!c) return PERCIS_E_NOMEM;
        c->device = device;
        c->stream = (hipStream_t)hip_stream;
        hipDeviceProp_t prop;
        if (hipSetDevice(device) != hipSuccess || hipGetDeviceProperties(&prop, device) != hipSuccess) {
            delete c;
            return PERCIS_E_DEVICE;
        }
        c->cu_count = prop.multiProcessorCount;
        int wall_khz = 0;
        if (hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, device) == hipSuccess)
            c->wall_hz = wall_khz * 1e3;
        if (hipMalloc((void**)&c->d_stats, sizeof(DevStats)) != hipSuccess ||
            hipMalloc((void**)&c->d_work, 6 * sizeof(unsigned long long)) != hipSuccess ||
            hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
            percis_destroy(c);
            return PERCIS_E_DEVICE;
        }
        // the no-allocation call's scratch: its address on this device, once
        // (if the lookup fails here, that call repeats it and reports why)
        if (noalloc_scratch(c, &c->noalloc) != PERCIS_OK) {
            (void)hipGetLastError();
            c->noalloc = nullptr;
            c->err.clear();
        }
    }
    c->graphs.push_back(new (std::nothrow) GraphData());
    if (!c->graphs[0]) {
        percis_destroy(c);
        return PERCIS_E_NOMEM;
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
    for (GraphData* G : c->graphs) {
        if (G) {
            graph_clear(*G);
            delete G;
        }
    }
    c->graphs.clear();
    free_slots(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    c->cap_stream = nullptr;
    dfree(c->d_stats);
    dfree(c->d_work);
    dfree(c->d_pairs);
    dfree(c->d_wide);
    dfree(c->d_big);
    dfree(c->d_wdbg);
    for (hipEvent_t e : c->chunk_ev) (void)hipEventDestroy(e);
    c->chunk_ev.clear();
    dfree(c->d_dbg);
    dfree(c->d_tasks);
    dfree(c->d_task_stats);
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
    int rc = sync_ctx(c);
    if (rc) return rc;
    GraphData* tmp = new (std::nothrow) GraphData();
    if (!tmp) return fail(c, PERCIS_E_NOMEM, "out of host memory");
    rc = graph_load(c, *tmp, n, m, row_ptr, col, flags);
    if (rc) {
        graph_clear(*tmp);
        delete tmp;
        return rc;
    }
    tmp->D_override = c->graphs[0]->D_override;
    c->generation++;
    graph_clear(*c->graphs[0]);
    delete c->graphs[0];
    c->graphs[0] = tmp;
    return PERCIS_OK;
}

int percis_set_states(percis_ctx* c, const uint16_t* k, uint32_t flags) {
    if (!c) return PERCIS_E_INVAL;
    int rc = sync_ctx(c);
    if (rc) return rc;
    return graph_set_states(c, *c->graphs[0], k, flags);
}

int percis_add_graph(percis_ctx* c, int32_t n, int64_t m, const int32_t* row_ptr, const int32_t* col,
                     const uint16_t* k, uint32_t flags, int32_t* graph_id) {
    if (!c || !graph_id) return PERCIS_E_INVAL;
    GraphData* G = new (std::nothrow) GraphData();
    if (!G) return fail(c, PERCIS_E_NOMEM, "out of host memory");
    int rc = graph_load(c, *G, n, m, row_ptr, col, flags);
    if (!rc) rc = graph_set_states(c, *G, k, flags & PERCIS_DEVICE_PTRS);
    if (rc) {
        graph_clear(*G);
        delete G;
        return rc;
    }
    c->graphs.push_back(G);
    *graph_id = (int32_t)c->graphs.size() - 1;
    return PERCIS_OK;
}

int percis_graph_info(percis_ctx* c, int32_t graph, int32_t* n, int64_t* m, int32_t* n_active) {
    if (!c) return PERCIS_E_INVAL;
    GraphData* G = get_graph(c, graph);
    if (!G || !G->has_graph) return fail(c, PERCIS_E_INVAL, "no graph %d", graph);
    if (n) *n = G->n;
    if (m) *m = G->m;
    if (n_active) *n_active = G->n_act;
    return PERCIS_OK;
}

int percis_sample_range(percis_ctx* c, uint64_t first, uint64_t count, uint64_t seed, uint32_t phase, uint32_t* hits,
                        uint32_t flags, percis_stats* st) {
    if (!c) return PERCIS_E_INVAL;
    GraphData& G = *c->graphs[0];
    if (!G.has_graph || !G.has_states) return fail(c, PERCIS_E_STATE, "load a graph and set states first");
    if (!hits) return fail(c, PERCIS_E_INVAL, "null hits");
    if (count >= (1ull << 32)) return fail(c, PERCIS_E_TOO_LARGE, "at most 2^32 - 1 samples per call");
    int rc = graph_upload(c, G, true);
    if (rc) return rc;
    const bool dev = (flags & PERCIS_DEVICE_PTRS) != 0;
    const bool acc = (flags & PERCIS_ACCUMULATE) != 0;
    uint32_t* dh = dev ? hits : G.d_hits;
    if (!dev && acc) HIPCHK(c, hipMemcpyAsync(dh, hits, sizeof(uint32_t) * G.n, hipMemcpyHostToDevice, c->stream));
    std::vector<TaskSpec> one(1);
    one[0] = TaskSpec{0, phase, first, count, seed, dh, acc};
    percis_stats launch{};
    rc = run_tasks(c, one, nullptr, &launch);
    if (rc != PERCIS_OK && rc != PERCIS_E_SIGMA_OVERFLOW) return rc;
    if (st) *st = launch;
    if (!dev) {
        HIPCHK(c, hipMemcpyAsync(hits, dh, sizeof(uint32_t) * G.n, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return rc;
}

// percis_sample_range without allocating: every buffer of the launch is a
// view into the library's static device scratch (kNoAllocScratchBytes per
// GPU), laid out for this call's graph: the task table and counters, the
// pair lists of one chunk of at most kNoAllocChunk samples, one slot of the
// 128-bit path, compact slots when the per-node slots cannot fill the device,
// and per-node slots (at least one) for the rest. The used part is cleared by
// fill kernels first; the kernels are those of percis_sample_range.
int percis_sample_range_noalloc(percis_ctx* c, uint64_t first, uint64_t count, uint64_t seed, uint32_t phase,
                                uint32_t* hits, uint32_t flags, percis_stats* st) {
    if (!c) return PERCIS_E_INVAL;
    if (c->host_only) return fail(c, PERCIS_E_STATE, "host-only context: no device work possible");
    if (!hits) return fail(c, PERCIS_E_INVAL, "null hits");
    if (!(flags & PERCIS_DEVICE_PTRS))
        return fail(c, PERCIS_E_INVAL, "hits must be device memory (PERCIS_DEVICE_PTRS): host hits need a staging buffer");
    if (flags & ~(uint32_t)(PERCIS_DEVICE_PTRS | PERCIS_ACCUMULATE)) return fail(c, PERCIS_E_INVAL, "unknown flags");
    if (count >= (1ull << 32)) return fail(c, PERCIS_E_TOO_LARGE, "at most 2^32 - 1 samples per call");
    GraphData& G = *c->graphs[0];
    if (!G.has_graph || !G.has_states || !G.graph_on_device || !G.states_on_device)
        return fail(c, PERCIS_E_STATE, "load a graph and set its states first (those calls allocate, this one does not)");
    int rc = set_device(c);
    if (rc) return rc;
    if (!c->noalloc && (rc = noalloc_scratch(c, &c->noalloc))) return rc;
    char* base = (char*)c->noalloc;

    // layout
    const int64_t act = std::max<int64_t>(G.n_act, 1);
    const int64_t stride = (act + 63) / 64 * 64;
    const int64_t words = bitmap_words(act);
    const int64_t per_node = node_slot_bytes(stride, words);
    const int64_t wide_one = stride * kWideBytesPerNode;
    const uint64_t chunk = std::max<uint64_t>(1, std::min<uint64_t>(count, kNoAllocChunk));
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        const int64_t at = off;
        off = (off + bytes + 255) / 256 * 256;
        return at;
    };
    const int64_t o_task = take(sizeof(DevTask)), o_tstats = take(sizeof(DevStats)), o_stats = take(sizeof(DevStats));
    const int64_t o_work = take(6 * sizeof(unsigned long long));
    const int64_t o_pairs = take((int64_t)chunk * sizeof(PairRec)), o_wide = take((int64_t)chunk * sizeof(PairRec));
    const int64_t o_big = take((int64_t)chunk * sizeof(PairRec));
    const int64_t o_clear = off;  // from here on the scratch must be cleared before use
    const int64_t o_wslot = take(wide_one);
    const int64_t avail = kNoAllocScratchBytes - off;
    if (avail < per_node) {
        const int64_t lim = (kNoAllocScratchBytes - off - kArcsPerSlot * (int64_t)sizeof(DagArc)) /
                            (kSlotBytesPerNode + kWideBytesPerNode + 1);
        return fail(c, PERCIS_E_TOO_LARGE,
                    "the graph has %d nodes with arcs; the no-allocation call's %lld MiB scratch holds graphs of "
                    "up to about %lld",
                    G.n_act, (long long)(kNoAllocScratchBytes >> 20), (long long)lim);
    }
    SamplerShape sh{};
    int occ = 0;
    if ((rc = pick_shape(c, act, &sh, &occ))) return rc;
    const int64_t cu = std::max(c->cu_count, 1);
    const int64_t want = c->opt_slots > 0 ? c->opt_slots : cu * occ;
    LaunchBufs B;
    B.shape = sh;
    int64_t np = std::min<int64_t>(want, avail / per_node), nc = 0;
    if (sh.lds_sets && (c->opt_compact == 2 || (c->opt_compact == 0 && np < want))) {
        SamplerShape cs = sh, big = sh;
        cs.compact = true;
        if (c->opt_block == 0) cs.block = kCompactBlock;
        cs.lds_bytes = sampler_table_lds(true, cs.block);
        const int cocc = sampler_occupancy(cs);
        big.block = c->opt_defer_block > 0 ? (int)c->opt_defer_block : kDeferBlock;
        big.lds_bytes = sampler_table_lds(false, big.block);
        const int bocc = sampler_occupancy(big);
        if (bocc <= 0) big = sh;
        const int64_t cper = compact_slot_bytes();
        // one per-node slot at least; the compact slots take the rest up to
        // the device's fill, more per-node slots what is left after them
        nc = cocc > 0 ? std::min<int64_t>(c->opt_slots > 0 ? c->opt_slots : cu * cocc, (avail - per_node) / cper) : 0;
        if (nc >= 1) {
            np = std::max<int64_t>(1, std::min<int64_t>(cu * std::max(bocc, 1), (avail - nc * cper) / per_node));
            B.cshape = cs;
            B.shape = big;
        } else {
            nc = 0;
        }
    }
    const int64_t o_nodes = take(np * per_node);
    const int64_t o_cslots = take(nc * compact_slot_bytes());
    if (off > kNoAllocScratchBytes) return fail(c, PERCIS_E_DEVICE, "no-allocation scratch layout overflow");
    B.stats = (DevStats*)(base + o_stats);
    B.work = (unsigned long long*)(base + o_work);
    B.pairs = (PairRec*)(base + o_pairs);
    B.wide = (PairRec*)(base + o_wide);
    B.big = (PairRec*)(base + o_big);
    B.slots = node_slots_at(base + o_nodes, np, stride, words);
    B.nslots = (int)np;
    if (nc > 0) B.cslots = compact_slots_at(base + o_cslots, nc);
    B.ncslots = (int)nc;
    B.wslots = wide_slots_at(base + o_wslot, 1, stride, B.work + 3);
    B.wide_slots = 1;

    // the task, then a cleared scratch (the slots' between-sample state)
    DevTask t{};
    t.g = dev_graph(G);
    t.cdf = dev_cdf(G);
    t.first = first;
    t.count = count;
    t.seed = seed;
    t.phase = phase;
    t.hits = hits;
    t.stats = (DevStats*)(base + o_tstats);
    t.offset = 0;
    t.clear_hits = (flags & PERCIS_ACCUMULATE) ? 0u : 1u;
    DevTask* table = (DevTask*)(base + o_task);
    HIPCHK(c, hipMemcpyAsync(table, &t, sizeof t, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, launch_fill_u8(base + o_clear, off - o_clear, c->stream));
    HIPCHK(c, launch_fill_u32((uint32_t*)B.wslots.dist, 0xFFFFFFFFu, stride, c->stream));
    LaunchPlan lp;
    lp.nt = 1;
    lp.max_n = G.n;
    lp.total = count;
    lp.chunk = chunk;
    lp.nchunks = (size_t)((count + chunk - 1) / chunk);
    HIPCHK(c, hipEventRecord(c->ev0, c->stream));
    if ((rc = enqueue_tasks(c, lp, table, B, c->stream, false))) return rc;
    HIPCHK(c, hipEventRecord(c->ev1, c->stream));
    DevStats ht{}, hl{};
    HIPCHK(c, hipMemcpyAsync(&ht, t.stats, sizeof ht, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(&hl, B.stats, sizeof hl, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
    percis_stats agg;
    stats_from_dev(ht, &agg);
    launch_fields(c, hl, ms, 0.0, nullptr, &agg);
    if (st) *st = agg;
    if (agg.samples != count)
        return fail(c, PERCIS_E_DEVICE, "sampler processed %llu of %llu samples", (unsigned long long)agg.samples,
                    (unsigned long long)count);
    return launch_status(c, hl, agg);
}

int percis_sample(percis_ctx* c, uint64_t n_samples, uint64_t seed, uint32_t* hits, uint32_t flags, percis_stats* st) {
    return percis_sample_range(c, 0, n_samples, seed, 0, hits, flags, st);
}

int percis_sample_tasks(percis_ctx* c, int32_t ntasks, const percis_task* tasks, percis_stats* launch_stats) {
    if (!c) return PERCIS_E_INVAL;
    if (ntasks < 1 || !tasks) return fail(c, PERCIS_E_INVAL, "need at least one task");
    std::vector<TaskSpec> specs(ntasks);
    for (int32_t i = 0; i < ntasks; i++) {
        const percis_task& t = tasks[i];
        GraphData* G = get_graph(c, t.graph);
        if (!G) return fail(c, PERCIS_E_INVAL, "task %d: no graph %d", i, t.graph);
        if (!G->has_graph || !G->has_states) return fail(c, PERCIS_E_STATE, "task %d: graph %d has no states", i, t.graph);
        if (!t.hits) return fail(c, PERCIS_E_INVAL, "task %d: null hits", i);
        if (t.count >= (1ull << 32)) return fail(c, PERCIS_E_TOO_LARGE, "task %d: at most 2^32 - 1 samples", i);
        specs[i] = TaskSpec{t.graph, t.phase, t.first, t.count, t.seed, t.hits, (t.flags & PERCIS_ACCUMULATE) != 0};
    }
    std::vector<percis_stats> ts;
    const int rc = run_tasks(c, specs, &ts, launch_stats);
    if (rc != PERCIS_OK && rc != PERCIS_E_SIGMA_OVERFLOW) return rc;
    for (int32_t i = 0; i < ntasks; i++)
        if (tasks[i].stats) *tasks[i].stats = ts[i];
    return rc;
}

}  // extern "C"

struct percis_batch {
    percis_ctx* ctx = nullptr;
    std::vector<TaskSpec> tasks;
    std::vector<percis_stats*> task_stats;   // host, from the capture's task list (may be null)
    DevTask* d_tasks = nullptr;
    DevStats* d_task_stats = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t generation = 0;
};

static void batch_free(percis_batch* b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    dfree(b->d_tasks);
    dfree(b->d_task_stats);
    delete b;
}

extern "C" {

int percis_batch_capture(percis_ctx* c, int32_t ntasks, const percis_task* tasks, percis_batch** out) {
    if (!c || !out) return PERCIS_E_INVAL;
    *out = nullptr;
    if (ntasks < 1 || !tasks) return fail(c, PERCIS_E_INVAL, "need at least one task");
    int rc = set_device(c);
    if (rc) return rc;
    percis_batch* b = new (std::nothrow) percis_batch();
    if (!b) return fail(c, PERCIS_E_NOMEM, "out of host memory");
    b->ctx = c;
    for (int32_t i = 0; i < ntasks; i++) {
        const percis_task& t = tasks[i];
        GraphData* G = get_graph(c, t.graph);
        rc = !G ? fail(c, PERCIS_E_INVAL, "task %d: no graph %d", i, t.graph)
           : (!G->has_graph || !G->has_states) ? fail(c, PERCIS_E_STATE, "task %d: graph %d has no states", i, t.graph)
           : !t.hits ? fail(c, PERCIS_E_INVAL, "task %d: null hits", i)
           : t.count >= (1ull << 32) ? fail(c, PERCIS_E_TOO_LARGE, "task %d: at most 2^32 - 1 samples", i)
                                     : PERCIS_OK;
        if (rc) {
            batch_free(b);
            return rc;
        }
        b->tasks.push_back(TaskSpec{t.graph, t.phase, t.first, t.count, t.seed, t.hits, (t.flags & PERCIS_ACCUMULATE) != 0});
        b->task_stats.push_back(t.stats);
    }
    if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        c->cap_stream = nullptr;
        batch_free(b);
        return fail(c, PERCIS_E_DEVICE, "cannot create the capture stream");
    }
    LaunchPlan lp;
    std::vector<DevTask> ht;
    if ((rc = dalloc(c, b->d_tasks, (size_t)ntasks)) || (rc = dalloc(c, b->d_task_stats, (size_t)ntasks)) ||
        (rc = plan_tasks(c, b->tasks, b->d_tasks, b->d_task_stats, ht, &lp))) {
        batch_free(b);
        return rc;
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess ||
        hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
        batch_free(b);
        return fail(c, PERCIS_E_DEVICE, "cannot begin a stream capture");
    }
    rc = enqueue_tasks(c, lp, b->d_tasks, ctx_bufs(c), c->cap_stream, false);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
    if (rc == PERCIS_OK && e != hipSuccess) rc = fail(c, PERCIS_E_DEVICE, "stream capture: %s", hipGetErrorString(e));
    if (rc == PERCIS_OK && hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        b->exec = nullptr;
        rc = fail(c, PERCIS_E_DEVICE, "cannot instantiate the captured launch");
    }
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    if (rc) {
        batch_free(b);
        return rc;
    }
    b->generation = c->generation;
    *out = b;
    return PERCIS_OK;
}

int percis_batch_replay(percis_batch* b, percis_stats* launch_stats) {
    if (!b || !b->ctx) return PERCIS_E_INVAL;
    percis_ctx* c = b->ctx;
    if (b->generation != c->generation)
        return fail(c, PERCIS_E_STATE, "graphs, states, options or buffers changed since the capture; capture again");
    for (size_t i = 0; i < b->tasks.size(); i++) {
        const GraphData* G = get_graph(c, b->tasks[i].graph);
        if (!G || !G->has_graph || !G->has_states || !G->states_on_device)
            return fail(c, PERCIS_E_STATE, "task %zu: graph %d has no states; set them and capture again", i,
                        b->tasks[i].graph);
    }
    int rc = set_device(c);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipEventRecord(c->ev0, c->cap_stream));
    HIPCHK(c, hipGraphLaunch(b->exec, c->cap_stream));
    HIPCHK(c, hipEventRecord(c->ev1, c->cap_stream));
    HIPCHK(c, hipStreamSynchronize(c->cap_stream));
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
    std::vector<percis_stats> ts;
    rc = collect_tasks(c, b->tasks, b->d_task_stats, c->d_stats, ms, 0.0, nullptr, &ts, launch_stats);
    if (rc != PERCIS_OK && rc != PERCIS_E_SIGMA_OVERFLOW) return rc;
    for (size_t i = 0; i < b->task_stats.size() && i < ts.size(); i++)
        if (b->task_stats[i]) *b->task_stats[i] = ts[i];
    return rc;
}

void percis_batch_destroy(percis_batch* b) {
    if (!b) return;
    if (b->ctx && !b->ctx->host_only) {
        (void)hipSetDevice(b->ctx->device);
        if (b->ctx->cap_stream) (void)hipStreamSynchronize(b->ctx->cap_stream);
    }
    batch_free(b);
}

int percis_set_vertex_diameter(percis_ctx* c, int64_t D) {
    if (!c) return PERCIS_E_INVAL;
    c->graphs[0]->D_override = D;
    return PERCIS_OK;
}

int percis_graph_set_vertex_diameter(percis_ctx* c, int32_t graph, int64_t D) {
    if (!c) return PERCIS_E_INVAL;
    GraphData* G = get_graph(c, graph);
    if (!G) return fail(c, PERCIS_E_INVAL, "no graph %d", graph);
    G->D_override = D;
    return PERCIS_OK;
}

int percis_graph_vertex_diameter(percis_ctx* c, int32_t graph, int64_t* D) {
    if (!c || !D) return PERCIS_E_INVAL;
    GraphData* G = get_graph(c, graph);
    if (!G || !G->has_graph) return fail(c, PERCIS_E_INVAL, "no graph %d", graph);
    return vertex_diam_ub(c, *G, D);
}

int percis_debug_states(percis_ctx* c, int32_t graph, int32_t* perm, uint32_t* kr, uint64_t* W, uint64_t* P,
                        double* d_v, double* S_v, uint64_t* C, double* d_hat) {
    if (!c) return PERCIS_E_INVAL;
    GraphData* G = get_graph(c, graph);
    if (!G || !G->has_graph || !G->has_states) return fail(c, PERCIS_E_STATE, "graph %d has no states", graph);
    int rc = graph_upload(c, *G, true);
    if (rc) return rc;
    const int32_t n = G->n;
    if (perm) {
        HIPCHK(c, hipMemcpyAsync(perm, G->d_perm, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (int32_t i = 1; i <= n; i++) perm[i] = G->h_orig[perm[i]];
    }
    if (kr) HIPCHK(c, hipMemcpyAsync(kr, G->d_kr, sizeof(uint32_t) * (n + 2), hipMemcpyDeviceToHost, c->stream));
    if (W) HIPCHK(c, hipMemcpyAsync(W, G->d_W, sizeof(uint64_t) * (n + 2), hipMemcpyDeviceToHost, c->stream));
    if (P) HIPCHK(c, hipMemcpyAsync(P, G->d_P, sizeof(uint64_t) * (n + 1), hipMemcpyDeviceToHost, c->stream));
    if (d_v) HIPCHK(c, hipMemcpyAsync(d_v, G->d_dv, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    if (S_v) HIPCHK(c, hipMemcpyAsync(S_v, G->d_Sv, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (C) *C = G->C;
    if (d_hat) *d_hat = G->d_hat;
    return PERCIS_OK;
}

int percis_estimate(percis_ctx* c, double eps, double delta, uint64_t seed, double* p_out, percis_estimate_info* info) {
    if (!c) return PERCIS_E_INVAL;
    return estimate_graph(c, 0, eps, delta, seed, p_out, info);
}

int percis_graph_estimate_di(percis_ctx* c, int32_t graph, double eps, double delta, uint64_t seed, double* p_out,
                             percis_estimate_info* info) {
    if (!c) return PERCIS_E_INVAL;
    return estimate_graph(c, graph, eps, delta, seed, p_out, info, true);
}

int percis_graph_estimate(percis_ctx* c, int32_t graph, double eps, double delta, uint64_t seed, double* p_out,
                          percis_estimate_info* info) {
    if (!c) return PERCIS_E_INVAL;
    return estimate_graph(c, graph, eps, delta, seed, p_out, info);
}

int percis_debug_path(percis_ctx* c, int32_t s, int32_t t, uint64_t r, int32_t* path, int32_t cap, int32_t* L,
                      uint64_t* sigma, int32_t* overflow) {
    if (!c) return PERCIS_E_INVAL;
    GraphData& G = *c->graphs[0];
    if (!G.has_graph) return fail(c, PERCIS_E_STATE, "load a graph first");
    if (s < 0 || s >= G.n || t < 0 || t >= G.n || s == t || cap < 0 || (cap > 0 && !path))
        return fail(c, PERCIS_E_INVAL, "bad debug_path arguments");
    int rc = graph_upload(c, G, false);  // the path needs the graph only
    if (rc) return rc;
    if ((rc = ensure_slots(c, std::max<int64_t>(G.n_act, max_active(c))))) return rc;
    const int32_t need = std::max<int32_t>(cap, 1);
    if (need > c->dbg_cap) {
        dfree(c->d_dbg);
        void* p = nullptr;
        HIPCHK(c, hipMalloc(&p, sizeof(DebugOut) + sizeof(int32_t) * need));
        c->d_dbg = (DebugOut*)p;
        c->dbg_cap = need;
    }
    HIPCHK(c, launch_fill_u8(c->d_dbg, sizeof(DebugOut) + sizeof(int32_t) * need, c->stream));
    HIPCHK(c, launch_debug_path(dev_graph(G), c->slots, G.h_newid[s], G.h_newid[t], r, c->d_dbg, cap, c->shape,
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
        for (int32_t i = 0; i <= o->L; i++) path[i] = G.h_orig[o->path[i]];
    return PERCIS_OK;
}

int percis_debug_path_wide(percis_ctx* c, int32_t s, int32_t t, uint64_t r_lo, uint64_t r_hi, int32_t* path,
                           int32_t cap, int32_t* L, uint64_t* sigma_lo, uint64_t* sigma_hi, int32_t* overflow) {
    if (!c) return PERCIS_E_INVAL;
    GraphData& G = *c->graphs[0];
    if (!G.has_graph) return fail(c, PERCIS_E_STATE, "load a graph first");
    if (s < 0 || s >= G.n || t < 0 || t >= G.n || s == t || cap < 0 || (cap > 0 && !path))
        return fail(c, PERCIS_E_INVAL, "bad debug_path_wide arguments");
    int rc = graph_upload(c, G, false);
    if (rc) return rc;
    if ((rc = ensure_slots(c, std::max<int64_t>(G.n_act, max_active(c))))) return rc;
    const int32_t need = std::max<int32_t>(cap, 1);
    if (need > c->wdbg_cap) {
        dfree(c->d_wdbg);
        void* p = nullptr;
        HIPCHK(c, hipMalloc(&p, sizeof(WideDebug) + sizeof(int32_t) * need));
        c->d_wdbg = (WideDebug*)p;
        c->wdbg_cap = need;
    }
    WideDebug req{};
    req.s = G.h_newid[s];
    req.t = G.h_newid[t];
    req.r = (unsigned __int128)r_lo | ((unsigned __int128)r_hi << 64);
    req.cap = cap;
    req.path = (int32_t*)(c->d_wdbg + 1);
    HIPCHK(c, hipMemcpyAsync(c->d_wdbg, &req, sizeof req, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, launch_wide_debug(dev_graph(G), c->wslots, c->d_wdbg, c->stream));
    std::vector<int32_t> dpath(need);
    HIPCHK(c, hipMemcpyAsync(&req, c->d_wdbg, sizeof req, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(dpath.data(), c->d_wdbg + 1, sizeof(int32_t) * need, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (L) *L = req.L;
    if (sigma_lo) *sigma_lo = (uint64_t)req.sigma;
    if (sigma_hi) *sigma_hi = (uint64_t)(req.sigma >> 64);
    if (overflow) *overflow = req.overflow;
    if (req.overflow == 2) return fail(c, PERCIS_E_DEVICE, "canonical walk found no predecessor");
    if (path && req.L >= 0 && !req.overflow && req.r < req.sigma && req.L + 1 <= cap)
        for (int32_t i = 0; i <= req.L; i++) path[i] = G.h_orig[dpath[i]];
    return PERCIS_OK;
}

int percis_set_option(percis_ctx* c, int option, int64_t value) {
    if (!c) return PERCIS_E_INVAL;
    if (value < 0) return fail(c, PERCIS_E_INVAL, "negative option value");
    switch (option) {
        case PERCIS_OPT_SLOTS: c->opt_slots = value; break;
        case PERCIS_OPT_SCRATCH_MB: c->opt_scratch_mb = value; break;
        case PERCIS_OPT_BLOCK:
            if (value != 0 && value != 64 && value != 128 && value != 256 && value != 512 && value != 1024)
                return fail(c, PERCIS_E_INVAL, "block must be 64, 128, 256, 512 or 1024");
            c->opt_block = value;
            break;
        case PERCIS_OPT_BITMAPS:
            if (value > 2) return fail(c, PERCIS_E_INVAL, "bitmaps option is 0 (auto), 1 (device bitmaps) or 2 (LDS tables)");
            c->opt_bitmaps = value;
            break;
        case PERCIS_OPT_COMPACT:
            if (value > 2) return fail(c, PERCIS_E_INVAL, "compact option is 0 (auto), 1 (off) or 2 (on)");
            c->opt_compact = value;
            break;
        case PERCIS_OPT_DEFER_BLOCK:
            if (value != 0 && value != 64 && value != 128 && value != 256 && value != 512 && value != 1024)
                return fail(c, PERCIS_E_INVAL, "block must be 64, 128, 256, 512 or 1024");
            c->opt_defer_block = value;
            break;
        case PERCIS_OPT_PAIR_CHUNK:
            if ((uint64_t)value > kMaxPairChunk) return fail(c, PERCIS_E_INVAL, "pair chunk must be at most 2^30 samples");
            c->opt_pair_chunk = value;
            break;
        case PERCIS_OPT_BALANCE:
            if (value != 0 && (value < kMinBalance || value > kMaxBalance))
                return fail(c, PERCIS_E_INVAL, "balance must be 0 (auto) or %d .. %d", kMinBalance, kMaxBalance);
            // the rule only steers the search, so slots stay valid; a captured
            // launch keeps the rule it was captured with
            c->opt_balance = value;
            return PERCIS_OK;
        default: return fail(c, PERCIS_E_INVAL, "unknown option %d", option);
    }
    if (!c->host_only && sync_ctx(c) == PERCIS_OK) free_slots(c);
    return PERCIS_OK;
}

int percis_get_option(percis_ctx* c, int option, int64_t* value) {
    if (!c || !value) return PERCIS_E_INVAL;
    if (option == PERCIS_OPT_SCRATCH_MB) {
        *value = c->opt_scratch_mb;
        return PERCIS_OK;
    }
    if (option == PERCIS_OPT_PAIR_CHUNK) {
        *value = c->opt_pair_chunk > 0 ? c->opt_pair_chunk : (int64_t)kPairChunk;
        return PERCIS_OK;
    }
    if (option == PERCIS_OPT_BALANCE) {
        *value = c->opt_balance > 0 ? c->opt_balance : (int64_t)kBalance;
        return PERCIS_OK;
    }
    if (option != PERCIS_OPT_SLOTS && option != PERCIS_OPT_BLOCK && option != PERCIS_OPT_BITMAPS &&
        option != PERCIS_OPT_COMPACT && option != PERCIS_OPT_DEFER_BLOCK)
        return fail(c, PERCIS_E_INVAL, "unknown option %d", option);
    const int64_t act = max_active(c);
    if (c->host_only || act == 0) {
        *value = option == PERCIS_OPT_SLOTS     ? c->opt_slots
               : option == PERCIS_OPT_BLOCK     ? c->opt_block
               : option == PERCIS_OPT_BITMAPS   ? c->opt_bitmaps
               : option == PERCIS_OPT_COMPACT   ? c->opt_compact
                                                : c->opt_defer_block;
        return PERCIS_OK;
    }
    int rc = set_device(c);
    if (rc) return rc;
    if ((rc = ensure_slots(c, act))) return rc;
    const bool cm = c->ncslots > 0;
    *value = option == PERCIS_OPT_SLOTS     ? (cm ? c->ncslots : c->nslots)
           : option == PERCIS_OPT_BLOCK     ? (cm ? c->cshape.block : c->shape.block)
           : option == PERCIS_OPT_BITMAPS   ? (c->shape.lds_sets ? 2 : 1)
           : option == PERCIS_OPT_COMPACT   ? (cm ? 2 : 1)
                                            : (cm ? c->shape.block : c->opt_defer_block);
    return PERCIS_OK;
}

int percis_exact(percis_ctx* c, int32_t graph, double* p_out, double* kernel_ms) {
    if (!c) return PERCIS_E_INVAL;
    GraphData* G = get_graph(c, graph);
    if (!G) return fail(c, PERCIS_E_INVAL, "no graph %d", graph);
    if (!G->has_graph || !G->has_states) return fail(c, PERCIS_E_STATE, "graph %d has no states", graph);
    if (!p_out) return fail(c, PERCIS_E_INVAL, "null output");
    int rc = graph_upload(c, *G, true);
    if (rc) return rc;
    const int32_t n = G->n, na = std::max<int32_t>(G->n_act, 1);
    const int64_t stride = ((int64_t)na + 63) / 64 * 64;
    uint16_t* d_k = nullptr;
    double* d_out = nullptr;
    void* scratch = nullptr;
    size_t free_b = 0, total_b = 0;
    HIPCHK(c, hipMemGetInfo(&free_b, &total_b));
    int slots = std::max(1, c->cu_count * 2);
    while (slots > 1 && exact_scratch_bytes(stride, slots) > (int64_t)(free_b * 0.5)) slots /= 2;
    const int64_t bytes = exact_scratch_bytes(stride, slots);
    auto cleanup = [&]() {
        dfree(d_k);
        dfree(d_out);
        if (scratch) (void)hipFree(scratch);
        scratch = nullptr;
    };
    if ((rc = dalloc(c, d_k, (size_t)n)) || (rc = dalloc(c, d_out, (size_t)na))) {
        cleanup();
        return rc;
    }
    if (hipMalloc(&scratch, (size_t)bytes) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        return fail(c, PERCIS_E_NOMEM, "cannot allocate %lld bytes of scratch", (long long)bytes);
    }
    hipError_t e = launch_states_internal(G->d_k, G->d_newid, n, d_k, c->stream);
    if (e == hipSuccess) e = launch_fill_u8(scratch, bytes, c->stream);
    if (e == hipSuccess) e = launch_init_stats(c->d_stats, c->d_work, c->stream);
    if (e == hipSuccess) e = hipEventRecord(c->ev0, c->stream);
    if (e == hipSuccess) e = launch_exact(dev_graph(*G), d_k, scratch, stride, slots, c->d_work, d_out, c->stream);
    if (e == hipSuccess) e = hipEventRecord(c->ev1, c->stream);
    if (e == hipSuccess) e = launch_exact_finish(d_out, G->d_Sv, G->d_newid, n, G->n_act, G->d_p, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(p_out, G->d_p, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, c->ev0, c->ev1);
    cleanup();
    if (e != hipSuccess) return fail(c, PERCIS_E_DEVICE, "exact centrality: %s", hipGetErrorString(e));
    if (kernel_ms) *kernel_ms = ms;
    return PERCIS_OK;
}

int percis_autotune(percis_ctx* c, int32_t graph, uint64_t probe_samples, uint64_t seed, percis_tuning* result) {
    if (!c) return PERCIS_E_INVAL;
    if (c->host_only) return fail(c, PERCIS_E_STATE, "host-only context");
    if (probe_samples < 1 || probe_samples >= (1ull << 32)) return fail(c, PERCIS_E_INVAL, "bad probe size");
    // the probe: stream phase 3 of the one graph, or an equal share of every
    // graph with states (graph -1), as one launch
    std::vector<int32_t> ids;
    if (graph == -1) {
        for (int32_t i = 0; i < (int32_t)c->graphs.size(); i++) {
            const GraphData* G = c->graphs[i];
            if (G && G->has_graph && G->has_states) ids.push_back(i);
        }
        if (ids.empty()) return fail(c, PERCIS_E_STATE, "no graph has states");
    } else {
        GraphData* G = get_graph(c, graph);
        if (!G) return fail(c, PERCIS_E_INVAL, "no graph %d", graph);
        if (!G->has_graph || !G->has_states) return fail(c, PERCIS_E_STATE, "graph %d has no states", graph);
        ids.push_back(graph);
    }
    int rc;
    std::vector<TaskSpec> probe;
    const uint64_t share = std::max<uint64_t>(1, probe_samples / ids.size());
    uint64_t total = 0;
    for (int32_t id : ids) {
        GraphData* G = get_graph(c, id);
        if ((rc = graph_upload(c, *G, true))) return rc;
        probe.push_back(TaskSpec{id, 3, 0, share, seed, G->d_hits, false});
        total += share;
    }
    const int64_t act = std::max<int64_t>(1, max_active(c));
    struct Knobs {
        int64_t block, bitmaps, compact, slots, balance;
    };
    const Knobs saved{c->opt_block, c->opt_bitmaps, c->opt_compact, c->opt_slots, c->opt_balance};
    auto apply = [&](const Knobs& k) -> int {
        const bool shape = k.block != c->opt_block || k.bitmaps != c->opt_bitmaps || k.compact != c->opt_compact ||
                           k.slots != c->opt_slots;
        c->opt_block = k.block;
        c->opt_bitmaps = k.bitmaps;
        c->opt_compact = k.compact;
        c->opt_slots = k.slots;
        c->opt_balance = k.balance;
        int r = sync_ctx(c);
        if (r == PERCIS_OK && shape) free_slots(c);
        return r;
    };
    // one untimed launch, then the faster of two timed ones; a shape that
    // cannot run (no memory for its slots, no occupancy) rates 0
    int timed = 0;
    auto rate_of = [&](const Knobs& k, double* rate) -> int {
        *rate = 0.0;
        int r = apply(k);
        if (r) return r;
        percis_stats st{};
        double best_ms = 0.0;
        for (int rep = 0; rep < 3; rep++) {
            r = run_tasks(c, probe, nullptr, &st);
            if (r != PERCIS_OK && r != PERCIS_E_SIGMA_OVERFLOW) return PERCIS_OK;
            if (rep > 0 && st.kernel_ms > 0 && (best_ms == 0.0 || st.kernel_ms < best_ms)) best_ms = st.kernel_ms;
        }
        timed++;
        if (best_ms > 0) *rate = (double)total / best_ms * 1e3;
        return PERCIS_OK;
    };
    Knobs best{0, 0, 0, 0, 0};
    double best_rate = 0.0, auto_rate = 0.0;
    auto consider = [&](const Knobs& k) -> int {
        double r = 0.0;
        int e = rate_of(k, &r);
        if (e) return e;
        if (r > best_rate) {
            best_rate = r;
            best = k;
        }
        return PERCIS_OK;
    };
    auto restore = [&]() { (void)apply(saved); };
    // stage 1: the automatic shape, then threads per sample x where the
    // visited sets live (device bitmaps, LDS tables, LDS tables on compact slots)
    if ((rc = consider(best))) return restore(), rc;
    auto_rate = best_rate;
    for (int64_t b : {128, 256, 512, 1024}) {
        if (sampler_table_lds(false, (int)b) + sampler_static_lds() <= kLdsPerCu) {
            if ((rc = consider(Knobs{b, 2, 1, 0, 0}))) return restore(), rc;
            if ((rc = consider(Knobs{b, 2, 2, 0, 0}))) return restore(), rc;
        }
        if ((rc = consider(Knobs{b, 1, 1, 0, 0}))) return restore(), rc;
    }
    if (best_rate <= 0.0) {
        restore();
        return fail(c, PERCIS_E_DEVICE, "no launch shape could run");
    }
    // stage 2: fewer concurrent samples than fill the device (less pressure on
    // the L2 and on the memory system)
    if ((rc = apply(best))) return restore(), rc;
    if ((rc = ensure_slots(c, act))) return restore(), rc;
    const int64_t full = c->ncslots > 0 ? c->ncslots : c->nslots;
    // a slot count turns the automatic choices off: pin what they chose
    const int64_t chose_compact = c->ncslots > 0 ? 2 : 1, chose_bitmaps = c->shape.lds_sets ? 2 : 1;
    for (int64_t num : {3, 2}) {
        const int64_t s = full * num / 4;
        if (s < 1) continue;
        Knobs k = best;
        k.slots = s;
        k.compact = chose_compact;
        k.bitmaps = chose_bitmaps;
        if ((rc = consider(k))) return restore(), rc;
    }
    // stage 3: the side rule of the bidirectional search
    for (int64_t bal : {50, 200}) {
        Knobs k = best;
        k.balance = bal;
        if ((rc = consider(k))) return restore(), rc;
    }
    if ((rc = apply(best))) return restore(), rc;
    if ((rc = ensure_slots(c, act))) return rc;
    if (result) {
        const bool cm = c->ncslots > 0;
        result->block = (int32_t)(cm ? c->cshape.block : c->shape.block);
        result->bitmaps = c->shape.lds_sets ? 2 : 1;
        result->slots = (int32_t)(cm ? c->ncslots : c->nslots);
        result->candidates = timed;
        result->samples_per_s = best_rate;
        result->compact = cm ? 2 : 1;
        result->balance = (int32_t)(c->opt_balance > 0 ? c->opt_balance : kBalance);
        result->defer_block = cm ? (int32_t)c->shape.block : 0;
        result->auto_samples_per_s = auto_rate;
    }
    return PERCIS_OK;
}

}  // extern "C"
