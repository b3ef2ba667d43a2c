// Library-internal declarations of the device-side setup and reductions
// (percis_setup.hip). Nothing here is part of the ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace percis {

// Device arrays of the pair distribution of one graph (Algorithm 2's
// preprocessing in units of 1/65535) and the per-node weights; all owned by
// the graph. Ranks i = 1..n are sorted by (k non-increasing, caller id
// increasing).
struct StateArrays {
    int32_t n;
    const uint16_t* k;      // [n]   states by caller id (input)
    const int32_t* newid;   // [n]   caller id -> internal id
    int32_t* perm;          // [n+1] perm[i] = internal id of rank i, perm[0] = -1
    uint32_t* kr;           // [n+2] k of rank i, kr[0] = kr[n+1] = 0
    uint64_t* W;            // [n+2] W[i] = sum_{j >= i} kr[j], W[0] = W[n+1] = 0
    uint64_t* P;            // [n+1] P[i] = sum_{j <= i} ((n-j+1) kr[j] - W[j]), P[0] = 0; C = P[n]
    double* d_v;            // [n]   C / S_v by caller id, 0 where S_v = 0
    double* S_v;            // [n]   S_v by caller id (units of 1/65535)
};

// Scratch of the state build, sized by state_build_bytes(n).
int64_t state_build_bytes(int32_t n);

// Builds every output array of `a` from a.k on `stream`. `scratch` holds
// state_build_bytes(a.n) bytes. On completion result[0] = C and result[1] =
// the bit pattern of max_v d_v (a non-negative double), both device memory
// inside the scratch: *result_dev points at them.
hipError_t launch_state_build(const StateArrays& a, void* scratch, const uint64_t** result_dev, hipStream_t stream);

// VertexDiamUB: connected components of the active nodes (weakly connected for
// directed graphs), their sizes and, for undirected graphs, the eccentricity
// of each component's node of smallest caller id (orig: internal id -> caller
// id). Scratch holds diam_scratch_bytes(n_act, m) bytes; m = rp[n_act] arcs.
// The host drives the hooking rounds and the BFS levels, so the call
// synchronises `stream`.
int64_t diam_scratch_bytes(int32_t n_act, int64_t m);
hipError_t run_vertex_diam_ub(const int32_t* rp, const int32_t* col, const int32_t* orig, int32_t n_act, int64_t m,
                              bool directed, void* scratch, int64_t* D_out, int32_t* levels_out, int32_t* rounds_out,
                              hipStream_t stream);

// *out := max(*out, bits of max_v d_v h_v) over v < n (non-negative doubles
// order like their bit patterns). *out must be initialised by the caller.
hipError_t launch_hit_weight_max(const double* d_v, const uint32_t* hits, int32_t n, unsigned long long* out,
                                 hipStream_t stream);
// p[v] = d_v h_v / l.
hipError_t launch_estimates(const double* d_v, const uint32_t* hits, int32_t n, uint64_t l, double* p,
                            hipStream_t stream);
// p[v] = num[newid[v]] / S_v where newid[v] < n_act and S_v > 0, else 0.
hipError_t launch_exact_finish(const double* num, const double* S_v, const int32_t* newid, int32_t n, int32_t n_act,
                               double* p, hipStream_t stream);
// kint[newid[v]] = k[v].
hipError_t launch_states_internal(const uint16_t* k, const int32_t* newid, int32_t n, uint16_t* kint,
                                  hipStream_t stream);

}  // namespace percis
