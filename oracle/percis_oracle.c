/*
 * PercIS CPU oracle -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * A plain, slow, single-threaded C implementation of what the PercIS hot path
 * computes (Cruciani & Pellegrina, "Fast Percolation Centrality Approximation
 * with Importance Sampling"). It exists only to check the HIP library: only the
 * test suite, the package smoke check and the CPU-baseline leg of the benchmark
 * may load it. It shares no code, header, table or helper with the HIP library.
 *
 * Functions and the passages they follow:
 *   orc_philox4x64_10   Philox4x64-10 block function (Salmon, Moraes, Dror, Shaw,
 *                       "Parallel Random Numbers: As Easy as 1, 2, 3", SC'11).
 *   orc_bounded         Uniform integer in [0,N) by multiply-and-reject
 *                       (Lemire, "Fast Random Integer Generation in an Interval",
 *                       ACM TOMACS 2019), each attempt a fresh Philox block.
 *   orc_states_new      Preprocessing of Algorithm 2 (ImportanceSampler, appendix):
 *                       states sorted non-increasingly (Section II-A), then the
 *                       suffix sums w_i, the per-rank weights c_i, the suffix sums
 *                       r_i of c and the total c -- all in integer units of 1/65535.
 *   orc_draw_pair       The two binary searches of Algorithm 2 (sampling part),
 *                       with u = (U+1)/C read as an exact integer comparison.
 *   orc_path            RandomSP (Section III-B): BFS from s expanded until t is
 *                       found, shortest-path counts sigma (Section II-A), and one
 *                       shortest path chosen by the canonical backward walk.
 *   orc_path_bidir128,  RandomSP through the balanced bidirectional BFS that
 *   orc_sample_range_   Section III-B recommends: two balls grown from s and t,
 *   bidir               the sigma_s counts carried through the t side, the same
 *                       canonical walk. A speed path for the largest graphs,
 *                       proved equal to the truncated BFS by the CPU tests.
 *   orc_bounded128      Lemire's method at 128 bits, for r when sigma_st >= 2^64.
 *   orc_sample_range    The sampling loop of Algorithm 2 with RandomSP, reporting
 *                       per-node counts of internal-node hits (estimator of
 *                       Section III-A) and the |I(tau)| statistics used by Alg. 1.
 *   orc_exact           Percolation centrality of Definition 1 (Eq. 1) by the
 *                       Brandes-style dependency accumulation the paper uses for
 *                       its exact values (Section IV-A).
 *   orc_vertex_diam_ub  VertexDiamUB of Algorithm 1 (Section III-B).
 *   orc_estimate        Algorithm 1 (PercIS): two sampling phases and the bounds
 *                       of Proposition 2 (rho-hat), Proposition 3 (v-hat) and
 *                       Theorem 1 (sample size), with the constants of Alg. 1.
 *   orc_estimate_di     PercIS-DI (Section IV, sample size bound experiment):
 *                       Algorithm 1 without its first phase, with rho-hat = D
 *                       and v-hat = d-hat^2 / 4 in Theorem 1's sample size.
 *
 * Parity status: every function above is pinned by a CPU test (brute force on
 * tiny graphs, closed forms, an independent Philox implementation, exhaustive
 * boundary checks and statistical checks); none is "parity unpinned".
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------------- */
/* Philox4x64-10 (SC'11). Multipliers and Weyl key increments as published.   */
/* ------------------------------------------------------------------------- */
#define PHILOX_M0 0xD2E7470EE14C6C93ULL
#define PHILOX_M1 0xCA5A826395121157ULL
#define PHILOX_W0 0x9E3779B97F4A7C15ULL
#define PHILOX_W1 0xBB67AE8584CAA73BULL

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) { k0 += PHILOX_W0; k1 += PHILOX_W1; }
        u128 p0 = (u128)PHILOX_M0 * x0;
        u128 p1 = (u128)PHILOX_M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* The random stream: key = (seed, phase), counter = (sample index, variate,
 * attempt, 0); each variate uses word 0 of its block. Variates: 0 = the draw
 * that picks s, 1 = the draw that picks t, 2 = the draw that picks the path. */
uint64_t orc_word(uint64_t seed, uint64_t phase, uint64_t idx, uint64_t variate, uint64_t attempt)
{
    uint64_t ctr[4] = { idx, variate, attempt, 0 };
    uint64_t key[2] = { seed, phase };
    uint64_t out[4];
    orc_philox4x64_10(ctr, key, out);
    return out[0];
}

/* Lemire's method: m = x*N as 128 bits; the high word is the result unless the
 * low word falls in the biased zone [0, 2^64 mod N), then draw again. N >= 1. */
uint64_t orc_bounded(uint64_t seed, uint64_t phase, uint64_t idx, uint64_t variate,
                     uint64_t N, uint64_t* attempts_used)
{
    uint64_t attempt = 0;
    for (;;) {
        uint64_t x = orc_word(seed, phase, idx, variate, attempt);
        u128 m = (u128)x * N;
        uint64_t low = (uint64_t)m;
        int reject = 0;
        if (low < N) {
            uint64_t threshold = (uint64_t)(0 - N) % N; /* 2^64 mod N */
            if (low < threshold) reject = 1;
        }
        if (!reject) {
            if (attempts_used) *attempts_used = attempt + 1;
            return (uint64_t)(m >> 64);
        }
        attempt++;
    }
}

/* ------------------------------------------------------------------------- */
/* Graph: out-adjacency and in-adjacency, each row sorted ascending.          */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t n;
    int64_t m;
    int directed;
    int64_t* rp;  int32_t* col;   /* out-neighbours */
    int64_t* irp; int32_t* icol;  /* in-neighbours  */
} orc_graph;

static int cmp_i32(const void* a, const void* b)
{
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/* Copies a CSR (row_ptr[n+1], col[m]); rows are sorted here. For an undirected
 * graph the caller passes both arcs of every edge and in == out. */
orc_graph* orc_graph_new(int32_t n, int64_t m, const int32_t* row_ptr, const int32_t* col, int directed)
{
    orc_graph* g = (orc_graph*)calloc(1, sizeof(orc_graph));
    g->n = n; g->m = m; g->directed = directed;
    g->rp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    g->col = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    for (int32_t v = 0; v <= n; v++) g->rp[v] = row_ptr[v];
    for (int64_t e = 0; e < m; e++) g->col[e] = col[e];
    for (int32_t v = 0; v < n; v++)
        qsort(g->col + g->rp[v], (size_t)(g->rp[v + 1] - g->rp[v]), sizeof(int32_t), cmp_i32);
    /* in-adjacency by transposition; scanning sources in increasing order
     * leaves every in-row sorted ascending */
    g->irp = (int64_t*)calloc((size_t)(n + 1), sizeof(int64_t));
    g->icol = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    for (int64_t e = 0; e < m; e++) g->irp[g->col[e] + 1]++;
    for (int32_t v = 0; v < n; v++) g->irp[v + 1] += g->irp[v];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    memcpy(fill, g->irp, sizeof(int64_t) * (size_t)(n + 1));
    for (int32_t u = 0; u < n; u++)
        for (int64_t e = g->rp[u]; e < g->rp[u + 1]; e++) g->icol[fill[g->col[e]]++] = u;
    free(fill);
    return g;
}

void orc_graph_free(orc_graph* g)
{
    if (!g) return;
    free(g->rp); free(g->col); free(g->irp); free(g->icol); free(g);
}

/* ------------------------------------------------------------------------- */
/* States and the preprocessing of Algorithm 2.                               */
/* x_v = k_v / 65535; every quantity below is kept in units of 1/65535, so    */
/* that all sums are exact integers.                                          */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t n;
    uint16_t* k;     /* k[v], by node id */
    int32_t* perm;   /* perm[i] = node of rank i, i = 1..n (rank 0 unused) */
    uint64_t* x;     /* x[i] = k of rank i, i = 1..n */
    uint64_t* w;     /* w[i] = sum_{j>=i} x[j], i = 1..n+1 */
    uint64_t* c;     /* c[i] = sum_{j>=i} R(x[i]-x[j]) */
    uint64_t* r;     /* r[i] = sum_{j>=i} c[j], i = 1..n+1 */
    uint64_t C;      /* total weight sum_{u != w} R(x_u - x_w) */
    double* S;       /* S[v] = sum over pairs (u,w) with u != v != w of R(x_u - x_w) */
} orc_states;

static const uint16_t* g_sort_keys;
static int cmp_rank(const void* a, const void* b)
{
    int32_t u = *(const int32_t*)a, v = *(const int32_t*)b;
    /* non-increasing state; ties by increasing node id */
    if (g_sort_keys[u] != g_sort_keys[v]) return g_sort_keys[u] > g_sort_keys[v] ? -1 : 1;
    return (u > v) - (u < v);
}

orc_states* orc_states_new(int32_t n, const uint16_t* k)
{
    orc_states* st = (orc_states*)calloc(1, sizeof(orc_states));
    st->n = n;
    st->k = (uint16_t*)malloc(sizeof(uint16_t) * (size_t)n);
    memcpy(st->k, k, sizeof(uint16_t) * (size_t)n);
    st->perm = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 2));
    st->x = (uint64_t*)calloc((size_t)(n + 2), sizeof(uint64_t));
    st->w = (uint64_t*)calloc((size_t)(n + 2), sizeof(uint64_t));
    st->c = (uint64_t*)calloc((size_t)(n + 2), sizeof(uint64_t));
    st->r = (uint64_t*)calloc((size_t)(n + 2), sizeof(uint64_t));
    st->S = (double*)calloc((size_t)n, sizeof(double));

    /* relabel so that states are non-increasing (Section II-A) */
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t v = 0; v < n; v++) order[v] = v;
    g_sort_keys = st->k;
    qsort(order, (size_t)n, sizeof(int32_t), cmp_rank);
    st->perm[0] = -1;
    for (int32_t i = 1; i <= n; i++) { st->perm[i] = order[i - 1]; st->x[i] = st->k[order[i - 1]]; }
    free(order);

    /* Algorithm 2, preprocessing: a single pass from the last rank to the first */
    uint64_t Csum = 0;
    st->w[n + 1] = 0; st->r[n + 1] = 0;
    for (int32_t i = n; i >= 1; i--) {
        st->w[i] = st->w[i + 1] + st->x[i];
        st->c[i] = (uint64_t)(n - i + 1) * st->x[i] - st->w[i];
        st->r[i] = st->r[i + 1] + st->c[i];
        Csum += st->c[i];
    }
    st->C = Csum;

    /* S_v: the pairs that avoid v. Pairs (u,w) that involve v contribute
     * R(x_v - x_w) + R(x_u - x_v) summed over the other node, i.e. |x_v - x_u|
     * summed over all u; the rest of the total is S_v. The sum over u is taken
     * from a histogram of the 65536 state values. */
    uint64_t* cnt = (uint64_t*)calloc(65537, sizeof(uint64_t));
    uint64_t* sum = (uint64_t*)calloc(65537, sizeof(uint64_t));
    for (int32_t v = 0; v < n; v++) { cnt[st->k[v] + 1]++; sum[st->k[v] + 1] += st->k[v]; }
    for (int j = 1; j <= 65536; j++) { cnt[j] += cnt[j - 1]; sum[j] += sum[j - 1]; }
    /* cnt[j], sum[j]: count and sum of states with value < j */
    for (int32_t v = 0; v < n; v++) {
        uint64_t kv = st->k[v];
        uint64_t below_cnt = cnt[kv], below_sum = sum[kv];
        uint64_t above_cnt = cnt[65536] - cnt[kv + 1], above_sum = sum[65536] - sum[kv + 1];
        uint64_t A = (below_cnt * kv - below_sum) + (above_sum - above_cnt * kv);
        st->S[v] = (double)(st->C - A);
    }
    free(cnt); free(sum);
    return st;
}

void orc_states_free(orc_states* st)
{
    if (!st) return;
    free(st->k); free(st->perm); free(st->x); free(st->w); free(st->c); free(st->r); free(st->S); free(st);
}

uint64_t orc_states_total(const orc_states* st) { return st->C; }
void orc_states_arrays(const orc_states* st, int32_t* perm, uint64_t* x, uint64_t* w, uint64_t* c, uint64_t* r, double* S)
{
    int32_t n = st->n;
    if (perm) memcpy(perm, st->perm, sizeof(int32_t) * (size_t)(n + 2));
    if (x) memcpy(x, st->x, sizeof(uint64_t) * (size_t)(n + 2));
    if (w) memcpy(w, st->w, sizeof(uint64_t) * (size_t)(n + 2));
    if (c) memcpy(c, st->c, sizeof(uint64_t) * (size_t)(n + 2));
    if (r) memcpy(r, st->r, sizeof(uint64_t) * (size_t)(n + 2));
    if (S) memcpy(S, st->S, sizeof(double) * (size_t)n);
}

/* Algorithm 2, sampling part. Both searches are the paper's loops with
 * u = (U+1)/C (resp. (U+1)/c_s) for an integer U uniform in [0,C) (resp.
 * [0,c_s)), so that "u <= k" is the exact integer test "U < numerator of k".
 * Returns ranks (1-based). Requires C > 0. */
void orc_search_s(const orc_states* st, uint64_t U, int32_t* s_out)
{
    int32_t n = st->n;
    int32_t a = 1, b = n, d = (a + b) / 2;
    while (a <= b) {
        /* k = (c - r_{d+1}) / c */
        if (U < st->C - st->r[d + 1]) b = d - 1; else a = d + 1;
        d = (a + b) / 2;
    }
    *s_out = b + 1;
}

void orc_search_t(const orc_states* st, int32_t s, uint64_t U, int32_t* t_out)
{
    int32_t n = st->n;
    int32_t a = s, b = n, d = (a + b) / 2;
    while (a <= b) {
        /* k = ((d - s + 1) x_s - w_s + w_{d+1}) / c_s */
        uint64_t num = (uint64_t)(d - s + 1) * st->x[s] - st->w[s] + st->w[d + 1];
        if (U < num) b = d - 1; else a = d + 1;
        d = (a + b) / 2;
    }
    *t_out = b + 1;
}

/* Draws the pair of sample `idx`; returns node ids. */
void orc_draw_pair(const orc_states* st, uint64_t seed, uint64_t phase, uint64_t idx,
                   int32_t* s_node, int32_t* t_node, int32_t* s_rank, int32_t* t_rank)
{
    int32_t s, t;
    uint64_t Us = orc_bounded(seed, phase, idx, 0, st->C, NULL);
    orc_search_s(st, Us, &s);
    uint64_t Ut = orc_bounded(seed, phase, idx, 1, st->c[s], NULL);
    orc_search_t(st, s, Ut, &t);
    if (s_rank) *s_rank = s;
    if (t_rank) *t_rank = t;
    *s_node = st->perm[s];
    *t_node = st->perm[t];
}

/* Lemire's method at 128 bits, for ranges N >= 2^64: x = the low two words of
 * the Philox block (word 0 low, word 1 high), m = x*N as 256 bits; the high
 * 128 bits are the result unless the low 128 fall in [0, 2^128 mod N). */
static void mul128(u128 a, u128 b, u128* hi, u128* lo)
{
    const u128 M = ((u128)1 << 64) - 1;
    u128 a0 = a & M, a1 = a >> 64, b0 = b & M, b1 = b >> 64;
    u128 p00 = a0 * b0, p01 = a0 * b1, p10 = a1 * b0, p11 = a1 * b1;
    u128 mid = (p00 >> 64) + (p01 & M) + (p10 & M);
    *lo = (p00 & M) | (mid << 64);
    *hi = p11 + (p01 >> 64) + (p10 >> 64) + (mid >> 64);
}

u128 orc_bounded128(uint64_t seed, uint64_t phase, uint64_t idx, uint64_t variate, u128 N, uint64_t* attempts_used)
{
    for (uint64_t attempt = 0;; attempt++) {
        uint64_t ctr[4] = { idx, variate, attempt, 0 };
        uint64_t key[2] = { seed, phase };
        uint64_t out[4];
        orc_philox4x64_10(ctr, key, out);
        u128 x = (u128)out[0] | ((u128)out[1] << 64);
        u128 hi, lo;
        mul128(x, N, &hi, &lo);
        if (lo < N) {
            u128 threshold = (u128)(0 - N) % N; /* 2^128 mod N */
            if (lo < threshold) continue;
        }
        if (attempts_used) *attempts_used = attempt + 1;
        return hi;
    }
}

/* Python-facing form: N and the result as two 64-bit halves. */
void orc_bounded128_parts(uint64_t seed, uint64_t phase, uint64_t idx, uint64_t variate, uint64_t n_lo,
                          uint64_t n_hi, uint64_t* r_lo, uint64_t* r_hi, uint64_t* attempts_used)
{
    u128 r = orc_bounded128(seed, phase, idx, variate, (u128)n_lo | ((u128)n_hi << 64), attempts_used);
    *r_lo = (uint64_t)r;
    *r_hi = (uint64_t)(r >> 64);
}

/* ------------------------------------------------------------------------- */
/* RandomSP: truncated BFS from s, shortest-path counts, canonical path.      */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t* dist;   /* -1 = not reached */
    u128* sigma;     /* saturates at 2^128 - 1 */
    int32_t* queue;
    int32_t touched; /* nodes the last search reached: queue[0 .. touched) */
} orc_work;

static orc_work* work_new(int32_t n)
{
    orc_work* w = (orc_work*)malloc(sizeof(orc_work));
    w->dist = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    w->sigma = (u128*)calloc((size_t)(n > 0 ? n : 1), sizeof(u128));
    w->queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t v = 0; v < n; v++) w->dist[v] = -1;
    w->touched = 0;
    return w;
}
static void work_free(orc_work* w) { free(w->dist); free(w->sigma); free(w->queue); free(w); }

static u128 add_sat(u128 a, u128 b)
{
    u128 s = a + b;
    return s < a ? ~(u128)0 : s;
}

/* Plain BFS from s in FIFO order; stops when the first node at distance
 * dist(t) is about to be expanded, so that every node at distance < dist(t)
 * has been expanded and sigma[t] is complete. Returns dist(t) or -1. */
static int32_t truncated_bfs(const orc_graph* g, int32_t s, int32_t t, orc_work* wk)
{
    /* forget the previous search: every node it reached is in its queue */
    for (int32_t i = 0; i < wk->touched; i++) { wk->dist[wk->queue[i]] = -1; wk->sigma[wk->queue[i]] = 0; }
    int32_t head = 0, tail = 0;
    wk->dist[s] = 0; wk->sigma[s] = 1; wk->queue[tail++] = s;
    while (head < tail) {
        int32_t u = wk->queue[head++];
        if (wk->dist[t] >= 0 && wk->dist[u] >= wk->dist[t]) break;
        for (int64_t e = g->rp[u]; e < g->rp[u + 1]; e++) {
            int32_t v = g->col[e];
            if (wk->dist[v] < 0) { wk->dist[v] = wk->dist[u] + 1; wk->queue[tail++] = v; }
            if (wk->dist[v] == wk->dist[u] + 1) wk->sigma[v] = add_sat(wk->sigma[v], wk->sigma[u]);
        }
    }
    wk->touched = tail;
    return wk->dist[t];
}

/* Canonical backward walk: from w = t, scan the in-neighbours u of w in
 * ascending id; those with dist(u) = dist(w) - 1 are the predecessors on
 * shortest paths from s. Step to the first predecessor whose sigma exceeds r,
 * subtracting the sigma of every predecessor passed over. This maps
 * r in [0, sigma_st) one-to-one onto the shortest s-t paths, so a uniform r
 * gives a uniform path (Section III-A, distribution q). Writes the path
 * s = path[0], ..., path[L] = t. Requires sigma_st below the saturation value
 * (every count on the walk is at most sigma_st, so none saturated). */
static void canonical_walk(const orc_graph* g, int32_t t, int32_t L, u128 r, const orc_work* wk, int32_t* path)
{
    int32_t w = t;
    path[L] = t;
    for (int32_t pos = L; pos >= 1; pos--) {
        int32_t next = -1;
        for (int64_t e = g->irp[w]; e < g->irp[w + 1]; e++) {
            int32_t u = g->icol[e];
            if (wk->dist[u] != pos - 1) continue;
            u128 su = wk->sigma[u];
            if (r < su) { next = u; break; }
            r -= su;
        }
        path[pos - 1] = next;
        w = next;
    }
}

/* r for a reachable sample with sigma_st = sg (below saturation): the 64-bit
 * draw of variate 2 when sigma_st < 2^64, else the 128-bit one. */
static u128 draw_r(uint64_t seed, uint64_t phase, uint64_t idx, u128 sg)
{
    if ((sg >> 64) == 0) return orc_bounded(seed, phase, idx, 2, (uint64_t)sg, NULL);
    return orc_bounded128(seed, phase, idx, 2, sg, NULL);
}

/* One canonical path for (s, t, r), r = r_lo + 2^64 r_hi; returns L = d(s,t),
 * or -1 if t is not reachable. sigma is returned as two 64-bit halves
 * (saturated at 2^128-1, which counts as overflow). The path is written only
 * if sigma is below saturation, r < sigma and cap >= L+1. */
int32_t orc_path128(const orc_graph* g, int32_t s, int32_t t, uint64_t r_lo, uint64_t r_hi, int32_t* path,
                    int32_t cap, uint64_t* sigma_lo, uint64_t* sigma_hi)
{
    orc_work* wk = work_new(g->n);
    int32_t L = truncated_bfs(g, s, t, wk);
    u128 sg = L >= 0 ? wk->sigma[t] : 0;
    u128 r = (u128)r_lo | ((u128)r_hi << 64);
    if (sigma_lo) *sigma_lo = (uint64_t)sg;
    if (sigma_hi) *sigma_hi = (uint64_t)(sg >> 64);
    if (L >= 0 && sg != ~(u128)0 && r < sg && cap >= L + 1) canonical_walk(g, t, L, r, wk, path);
    work_free(wk);
    return L;
}

/* orc_path128 with r < 2^64. */
int32_t orc_path(const orc_graph* g, int32_t s, int32_t t, uint64_t r, int32_t* path, int32_t cap,
                 uint64_t* sigma_lo, uint64_t* sigma_hi)
{
    return orc_path128(g, s, t, r, 0, path, cap, sigma_lo, sigma_hi);
}

typedef struct {
    uint64_t samples;          /* samples drawn */
    uint64_t reachable;        /* samples whose t is reachable from s */
    uint64_t sum_I;            /* sum of |I(tau)| over the samples */
    uint64_t sum_I2;           /* sum of |I(tau)|^2 */
    uint64_t overflow;         /* samples with sigma_st >= 2^128 - 1 (saturated) */
    uint64_t first_overflow;   /* smallest such sample index, or UINT64_MAX */
    uint64_t edges;            /* adjacency entries examined */
} orc_stats;

/* Samples idx = first .. first+count-1 of stream (seed, phase). hits[v] is
 * incremented once for every sampled path that has v as an internal node.
 * If I_out is not NULL, I_out[idx-first] receives |I(tau)| of each sample.
 * A sample whose sigma_st saturates (>= 2^128 - 1) adds no hits and is
 * counted in overflow. */
void orc_sample_range(const orc_graph* g, const orc_states* st, uint64_t first, uint64_t count,
                      uint64_t seed, uint64_t phase, uint32_t* hits, orc_stats* stats, int32_t* I_out)
{
    orc_work* wk = work_new(g->n);
    int32_t* path = (int32_t*)malloc(sizeof(int32_t) * (size_t)(g->n + 1));
    orc_stats S; memset(&S, 0, sizeof S); S.first_overflow = UINT64_MAX;
    for (uint64_t q = 0; q < count; q++) {
        uint64_t idx = first + q;
        int32_t s, t;
        orc_draw_pair(st, seed, phase, idx, &s, &t, NULL, NULL);
        S.samples++;
        int32_t L = truncated_bfs(g, s, t, wk);
        if (I_out) I_out[q] = 0;
        if (L < 0) continue;
        u128 sg = wk->sigma[t];
        if (sg == ~(u128)0) {
            S.overflow++;
            if (idx < S.first_overflow) S.first_overflow = idx;
            continue;
        }
        canonical_walk(g, t, L, draw_r(seed, phase, idx, sg), wk, path);
        for (int32_t i = 1; i < L; i++) hits[path[i]]++;
        uint64_t I = (uint64_t)(L - 1);
        S.reachable++;
        S.sum_I += I;
        S.sum_I2 += I * I;
        if (I_out) I_out[q] = (int32_t)I;
    }
    if (stats) *stats = S;
    free(path);
    work_free(wk);
}

/* ------------------------------------------------------------------------- */
/* RandomSP by balanced bidirectional BFS (Section III-B): two BFS balls, one  */
/* grown from s along out-arcs and one grown from t along in-arcs, the ball   */
/* whose frontier has fewer arcs to scan growing by one full level at a time. */
/* The canonical path depends only on the graph, s, t and r, so this finds    */
/* exactly the path of the truncated BFS above; the CPU tests check that on   */
/* every (s, t, r) of small graphs and on sample windows of large ones. It is */
/* a speed path of the oracle for graphs where a truncated BFS from s would   */
/* scan most of the graph for every sample.                                   */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t* ds;    /* distance from s, -1 = outside the s-ball */
    int32_t* dt;    /* distance to t, -1 = outside the t-ball */
    u128* gs;       /* shortest s-x path counts in the s-ball */
    u128* gt;       /* shortest x-t path counts in the t-ball */
    u128* gw;       /* t-ball: shortest s-x path counts for x on a shortest s-t path, else 0 */
    int32_t* qs;    /* the s-ball in BFS order (each level contiguous) */
    int32_t* qt;    /* the t-ball in BFS order */
    int32_t* tlev;  /* t-level j is qt[tlev[j] .. tlev[j+1]) */
    int32_t ns, nt; /* ball sizes */
    int32_t a, b;   /* levels each ball has completed */
} orc_bwork;

static orc_bwork* bwork_new(int32_t n)
{
    size_t N = (size_t)(n > 0 ? n : 1);
    orc_bwork* w = (orc_bwork*)calloc(1, sizeof(orc_bwork));
    w->ds = (int32_t*)malloc(sizeof(int32_t) * N);
    w->dt = (int32_t*)malloc(sizeof(int32_t) * N);
    w->gs = (u128*)calloc(N, sizeof(u128));
    w->gt = (u128*)calloc(N, sizeof(u128));
    w->gw = (u128*)calloc(N, sizeof(u128));
    w->qs = (int32_t*)malloc(sizeof(int32_t) * N);
    w->qt = (int32_t*)malloc(sizeof(int32_t) * N);
    w->tlev = (int32_t*)malloc(sizeof(int32_t) * (N + 2));
    for (int32_t v = 0; v < n; v++) { w->ds[v] = -1; w->dt[v] = -1; }
    return w;
}

static void bwork_free(orc_bwork* w)
{
    free(w->ds); free(w->dt); free(w->gs); free(w->gt); free(w->gw); free(w->qs); free(w->qt); free(w->tlev);
    free(w);
}

static u128 mul_sat(u128 x, u128 y)
{
    if (x != 0 && y > ~(u128)0 / x) return ~(u128)0;
    return x * y;
}

/* Grows both balls until a level reaches the other ball. Returns d(s,t), or
 * -1 if a ball stops growing first (t unreachable), and sets *sigma_st
 * (saturated at 2^128 - 1). On return every node at distance <= a from s
 * has ds and gs, and every node at distance <= b to t has dt and gt.
 * If the last level grown is level a of the s-ball, its new nodes that lie
 * in the t-ball are all at distance b to t (an earlier meeting would have
 * stopped the search), so d(s,t) = a + b, and every shortest path crosses
 * t-level b at one of them; the same holds with the sides swapped. Then
 * sigma_st = sum over that meeting layer of gs * gt. */
static int32_t bidir_search(const orc_graph* g, int32_t s, int32_t t, orc_bwork* w, u128* sigma_st)
{
    for (int32_t i = 0; i < w->ns; i++) { w->ds[w->qs[i]] = -1; w->gs[w->qs[i]] = 0; }
    for (int32_t i = 0; i < w->nt; i++) { w->dt[w->qt[i]] = -1; w->gt[w->qt[i]] = 0; w->gw[w->qt[i]] = 0; }
    w->ns = w->nt = 0;
    w->a = w->b = 0;
    *sigma_st = 0;
    w->ds[s] = 0; w->gs[s] = 1; w->qs[w->ns++] = s;
    w->dt[t] = 0; w->gt[t] = 1; w->qt[w->nt++] = t;
    w->tlev[0] = 0; w->tlev[1] = 1;
    if (s == t) { *sigma_st = 1; return 0; }
    int32_t s_lo = 0, t_lo = 0;   /* current frontiers: qs[s_lo .. ns), qt[t_lo .. nt) */
    for (;;) {
        if (s_lo == w->ns || t_lo == w->nt) return -1;
        uint64_t arcs_s = 0, arcs_t = 0;
        for (int32_t i = s_lo; i < w->ns; i++) arcs_s += (uint64_t)(g->rp[w->qs[i] + 1] - g->rp[w->qs[i]]);
        for (int32_t i = t_lo; i < w->nt; i++) arcs_t += (uint64_t)(g->irp[w->qt[i] + 1] - g->irp[w->qt[i]]);
        u128 meet = 0;
        int met = 0;
        if (arcs_s <= arcs_t) {
            int32_t hi = w->ns, lv = w->a + 1;
            for (int32_t i = s_lo; i < hi; i++) {
                int32_t u = w->qs[i];
                for (int64_t e = g->rp[u]; e < g->rp[u + 1]; e++) {
                    int32_t v = g->col[e];
                    if (w->ds[v] < 0) { w->ds[v] = lv; w->qs[w->ns++] = v; }
                    if (w->ds[v] == lv) w->gs[v] = add_sat(w->gs[v], w->gs[u]);
                }
            }
            s_lo = hi;
            w->a = lv;
            for (int32_t i = hi; i < w->ns; i++) {
                int32_t v = w->qs[i];
                if (w->dt[v] >= 0) { met = 1; meet = add_sat(meet, mul_sat(w->gs[v], w->gt[v])); }
            }
        } else {
            int32_t hi = w->nt, lv = w->b + 1;
            for (int32_t i = t_lo; i < hi; i++) {
                int32_t u = w->qt[i];
                for (int64_t e = g->irp[u]; e < g->irp[u + 1]; e++) {
                    int32_t v = g->icol[e];
                    if (w->dt[v] < 0) { w->dt[v] = lv; w->qt[w->nt++] = v; }
                    if (w->dt[v] == lv) w->gt[v] = add_sat(w->gt[v], w->gt[u]);
                }
            }
            t_lo = hi;
            w->b = lv;
            w->tlev[lv + 1] = w->nt;
            for (int32_t i = hi; i < w->nt; i++) {
                int32_t v = w->qt[i];
                if (w->ds[v] >= 0) { met = 1; meet = add_sat(meet, mul_sat(w->gs[v], w->gt[v])); }
            }
        }
        if (met) { *sigma_st = meet; return w->a + w->b; }
    }
}

/* After a meeting: gw[x] for the t-ball. A node x at distance j < b to t lies
 * on a shortest s-t path iff its distance from s is L - j; its shortest
 * predecessors u then lie on shortest s-t paths too, at distance j + 1 to t,
 * so sigma_s(x) = the sum of sigma_s(u) over in-neighbours u at t-level j + 1
 * that lie on shortest s-t paths. At t-level b those are the meeting layer
 * (the t-level-b nodes inside the s-ball), whose sigma_s is gs. Off the
 * shortest paths the sums come out 0. */
static void bidir_carry(const orc_graph* g, orc_bwork* w)
{
    for (int32_t i = w->tlev[w->b]; i < w->tlev[w->b + 1]; i++) {
        int32_t x = w->qt[i];
        if (w->ds[x] >= 0) w->gw[x] = w->gs[x];
    }
    for (int32_t j = w->b - 1; j >= 0; j--) {
        for (int32_t i = w->tlev[j]; i < w->tlev[j + 1]; i++) {
            int32_t x = w->qt[i];
            u128 sum = 0;
            for (int64_t e = g->irp[x]; e < g->irp[x + 1]; e++) {
                int32_t u = g->icol[e];
                if (w->dt[u] == j + 1) sum = add_sat(sum, w->gw[u]);
            }
            w->gw[x] = sum;
        }
    }
}

/* The canonical backward walk of canonical_walk on the two balls: the
 * predecessors of the node at position p + 1 are its in-neighbours at
 * distance p from s, weighed by sigma_s: read from the s-ball while p <= a,
 * from the t-ball (distance L - p to t, weight gw) beyond it. A node with
 * weight 0 is not a predecessor. */
static void bidir_walk(const orc_graph* g, int32_t t, int32_t L, u128 r, const orc_bwork* w, int32_t* path)
{
    int32_t x = t;
    path[L] = t;
    for (int32_t pos = L; pos >= 1; pos--) {
        int32_t p = pos - 1, next = -1;
        for (int64_t e = g->irp[x]; e < g->irp[x + 1]; e++) {
            int32_t u = g->icol[e];
            u128 su;
            if (p <= w->a) su = w->ds[u] == p ? w->gs[u] : 0;
            else su = w->dt[u] == L - p ? w->gw[u] : 0;
            if (su == 0) continue;
            if (r < su) { next = u; break; }
            r -= su;
        }
        path[p] = next;
        x = next;
    }
}

/* orc_path128 through the bidirectional search. */
int32_t orc_path_bidir128(const orc_graph* g, int32_t s, int32_t t, uint64_t r_lo, uint64_t r_hi, int32_t* path,
                          int32_t cap, uint64_t* sigma_lo, uint64_t* sigma_hi)
{
    orc_bwork* w = bwork_new(g->n);
    u128 sg = 0;
    int32_t L = bidir_search(g, s, t, w, &sg);
    u128 r = (u128)r_lo | ((u128)r_hi << 64);
    if (sigma_lo) *sigma_lo = (uint64_t)sg;
    if (sigma_hi) *sigma_hi = (uint64_t)(sg >> 64);
    if (L >= 0 && sg != ~(u128)0 && r < sg && cap >= L + 1) {
        bidir_carry(g, w);
        bidir_walk(g, t, L, r, w, path);
    }
    bwork_free(w);
    return L;
}

/* Scratch of the bidirectional search for graphs of up to n nodes, for
 * callers that run many sample ranges (one per thread at a time). */
orc_bwork* orc_bidir_work_new(int32_t n) { return bwork_new(n); }
void orc_bidir_work_free(orc_bwork* w) { if (w) bwork_free(w); }

/* orc_sample_range through the bidirectional search: the same hits and
 * statistics, sample by sample. w: scratch from orc_bidir_work_new for at
 * least g's nodes, or NULL (then allocated for this call). */
void orc_sample_range_bidir(const orc_graph* g, const orc_states* st, uint64_t first, uint64_t count,
                            uint64_t seed, uint64_t phase, uint32_t* hits, orc_stats* stats, int32_t* I_out,
                            orc_bwork* work)
{
    orc_bwork* w = work ? work : bwork_new(g->n);
    int32_t* path = (int32_t*)malloc(sizeof(int32_t) * (size_t)(g->n + 1));
    orc_stats S; memset(&S, 0, sizeof S); S.first_overflow = UINT64_MAX;
    for (uint64_t q = 0; q < count; q++) {
        uint64_t idx = first + q;
        int32_t s, t;
        orc_draw_pair(st, seed, phase, idx, &s, &t, NULL, NULL);
        S.samples++;
        if (I_out) I_out[q] = 0;
        u128 sg = 0;
        int32_t L = bidir_search(g, s, t, w, &sg);
        if (L < 0) continue;
        if (sg == ~(u128)0) {
            S.overflow++;
            if (idx < S.first_overflow) S.first_overflow = idx;
            continue;
        }
        bidir_carry(g, w);
        bidir_walk(g, t, L, draw_r(seed, phase, idx, sg), w, path);
        for (int32_t i = 1; i < L; i++) hits[path[i]]++;
        uint64_t I = (uint64_t)(L - 1);
        S.reachable++;
        S.sum_I += I;
        S.sum_I2 += I * I;
        if (I_out) I_out[q] = (int32_t)I;
    }
    if (stats) *stats = S;
    free(path);
    if (!work) bwork_free(w);
}

/* ------------------------------------------------------------------------- */
/* Exact percolation centrality (Definition 1) by dependency accumulation.    */
/* For a source s, with R_s(w) = R(x_s - x_w), the dependency                */
/*   delta_s(v) = sum_{t != s, v} sigma_st(v)/sigma_st * R_s(t)               */
/* satisfies delta_s(v) = sum over successors w of v on shortest paths from s */
/* of sigma_sv/sigma_sw * (R_s(w) + delta_s(w)), and                         */
/*   p(v) = sum_{s != v} delta_s(v) / S_v.                                    */
/* p(v) := 0 where S_v = 0 (p is undefined there).                            */
/* ------------------------------------------------------------------------- */
void orc_exact(const orc_graph* g, const orc_states* st, double* p_out)
{
    int32_t n = g->n;
    int32_t* dist = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    double* sigma = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* delta = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    double* num = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    for (int32_t s = 0; s < n; s++) {
        for (int32_t v = 0; v < n; v++) { dist[v] = -1; sigma[v] = 0.0; delta[v] = 0.0; }
        int32_t head = 0, tail = 0;
        dist[s] = 0; sigma[s] = 1.0; queue[tail++] = s;
        while (head < tail) {
            int32_t u = queue[head++];
            for (int64_t e = g->rp[u]; e < g->rp[u + 1]; e++) {
                int32_t v = g->col[e];
                if (dist[v] < 0) { dist[v] = dist[u] + 1; queue[tail++] = v; }
                if (dist[v] == dist[u] + 1) sigma[v] += sigma[u];
            }
        }
        double ks = (double)st->k[s];
        for (int32_t i = tail - 1; i >= 1; i--) {
            int32_t w = queue[i];
            double Rw = ks > st->k[w] ? ks - (double)st->k[w] : 0.0;
            for (int64_t e = g->irp[w]; e < g->irp[w + 1]; e++) {
                int32_t v = g->icol[e];
                if (dist[v] >= 0 && dist[v] == dist[w] - 1)
                    delta[v] += sigma[v] / sigma[w] * (Rw + delta[w]);
            }
        }
        for (int32_t i = 1; i < tail; i++) num[queue[i]] += delta[queue[i]];
    }
    for (int32_t v = 0; v < n; v++) p_out[v] = st->S[v] > 0 ? num[v] / st->S[v] : 0.0;
    free(dist); free(sigma); free(delta); free(queue); free(num);
}

/* ------------------------------------------------------------------------- */
/* VertexDiamUB (Algorithm 1). Undirected: per connected component, a BFS     */
/* from its smallest node u bounds the diameter by 2 ecc(u), so at most       */
/* 2 ecc(u) - 1 nodes are internal to a shortest path; never more than        */
/* |component| - 2. Directed: the component bound alone, on weakly connected  */
/* components.                                                                */
/* ------------------------------------------------------------------------- */
int64_t orc_vertex_diam_ub(const orc_graph* g)
{
    int32_t n = g->n;
    int32_t* dist = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t v = 0; v < n; v++) dist[v] = -1;
    int64_t D = 0;
    for (int32_t u = 0; u < n; u++) {
        if (dist[u] >= 0) continue;
        int32_t head = 0, tail = 0, ecc = 0;
        dist[u] = 0; queue[tail++] = u;
        while (head < tail) {
            int32_t x = queue[head++];
            if (dist[x] > ecc) ecc = dist[x];
            for (int64_t e = g->rp[x]; e < g->rp[x + 1]; e++) {
                int32_t y = g->col[e];
                if (dist[y] < 0) { dist[y] = dist[x] + 1; queue[tail++] = y; }
            }
            if (g->directed) {
                for (int64_t e = g->irp[x]; e < g->irp[x + 1]; e++) {
                    int32_t y = g->icol[e];
                    if (dist[y] < 0) { dist[y] = dist[x] + 1; queue[tail++] = y; }
                }
            }
        }
        int64_t size_bound = (int64_t)tail - 2;
        int64_t Dc = g->directed ? size_bound : (size_bound < 2 * (int64_t)ecc - 1 ? size_bound : 2 * (int64_t)ecc - 1);
        if (Dc > D) D = Dc;
    }
    free(dist); free(queue);
    return D;
}

/* ------------------------------------------------------------------------- */
/* Algorithm 1 (PercIS).                                                      */
/* ------------------------------------------------------------------------- */
typedef struct {
    uint64_t l1, l;           /* phase sizes */
    int64_t D;                /* vertex-diameter bound used */
    double d_hat;             /* max_v C / S_v */
    double rho_tilde, Lambda, rho_hat, v_hat, x_hat;
    uint64_t overflow;        /* overflowed samples over both phases */
} orc_estimate_info;

/* Theorem 1 with the constants of Algorithm 1: the bound on the number of
 * samples at a point x of (0, x_hat], with g(x) = x (d - x) and
 * h(y) = (1+y) ln(1+y) - y. */
static double sample_bound_at(double x, double d, double rho, double eps, double delta)
{
    double gx = x * (d - x);
    double y = eps * d / gx;
    double hy = (1.0 + y) * log1p(y) - y;
    return d * d * log(4.0 * d * rho / (x * delta)) / (gx * hy);
}

/* The supremum over (0, x_hat], read on a log-spaced grid of 200001 points
 * between x_hat * 1e-15 and x_hat (both included). */
double orc_sample_size(double d, double rho, double v, double eps, double delta, double* x_hat_out)
{
    double q = d * d / 4.0;
    double x_hat = d / 2.0 - sqrt(q - (q < v ? q : v));
    if (x_hat_out) *x_hat_out = x_hat;
    const int G = 200001;
    double best = 0.0;
    for (int j = 0; j < G; j++) {
        double x = j == G - 1 ? x_hat : x_hat * pow(10.0, -15.0 * (double)(G - 1 - j) / (double)(G - 1));
        double f = sample_bound_at(x, d, rho, eps, delta);
        if (f > best) best = f;
    }
    return best;
}

/* Estimator of Section III-A for the samples of one phase, written as the
 * paper writes it: every internal node v of every sampled path adds
 * kappa(s,t,v) / kappa~(s,t); the sum is divided by the number of samples. */
static void phase_estimate(const orc_graph* g, const orc_states* st, uint64_t count, uint64_t seed,
                           uint64_t phase, double* p, orc_stats* stats, int32_t* I_out)
{
    orc_work* wk = work_new(g->n);
    int32_t* path = (int32_t*)malloc(sizeof(int32_t) * (size_t)(g->n + 1));
    orc_stats S; memset(&S, 0, sizeof S); S.first_overflow = UINT64_MAX;
    for (int32_t v = 0; v < g->n; v++) p[v] = 0.0;
    for (uint64_t idx = 0; idx < count; idx++) {
        int32_t s, t;
        orc_draw_pair(st, seed, phase, idx, &s, &t, NULL, NULL);
        S.samples++;
        I_out[idx] = 0;
        int32_t L = truncated_bfs(g, s, t, wk);
        if (L < 0) continue;
        u128 sg = wk->sigma[t];
        if (sg == ~(u128)0) { S.overflow++; if (idx < S.first_overflow) S.first_overflow = idx; continue; }
        canonical_walk(g, t, L, draw_r(seed, phase, idx, sg), wk, path);
        double R = (double)st->k[s] - (double)st->k[t];
        double kappa_tilde = R / (double)st->C;
        for (int32_t i = 1; i < L; i++) {
            int32_t v = path[i];
            double kappa = R / st->S[v];
            p[v] += kappa / kappa_tilde;
        }
        S.reachable++;
        S.sum_I += (uint64_t)(L - 1);
        S.sum_I2 += (uint64_t)(L - 1) * (uint64_t)(L - 1);
        I_out[idx] = L - 1;
    }
    for (int32_t v = 0; v < g->n; v++) p[v] /= (double)count;
    if (stats) *stats = S;
    free(path);
    work_free(wk);
}

/* Runs Algorithm 1 with l1 = ceil(max(1000, ln(1/delta)/eps)) (Section III-B).
 * D < 0 asks for VertexDiamUB. Phase 1 uses stream phase 1, phase 2 uses
 * stream phase 2. Returns 0, or -1 if C = 0 (percolation centrality
 * undefined), or -2 if a sample overflowed. p_out receives phase 2. */
int orc_estimate(const orc_graph* g, const orc_states* st, double eps, double delta, uint64_t seed,
                 int64_t D, double* p_out, orc_estimate_info* info)
{
    orc_estimate_info I; memset(&I, 0, sizeof I);
    if (st->C == 0) return -1;
    int32_t n = g->n;
    I.D = D >= 0 ? D : orc_vertex_diam_ub(g);
    double d_hat = 1.0;
    for (int32_t v = 0; v < n; v++)
        if (st->S[v] > 0 && (double)st->C / st->S[v] > d_hat) d_hat = (double)st->C / st->S[v];
    I.d_hat = d_hat;
    double l1d = log(1.0 / delta) / eps;
    I.l1 = (uint64_t)ceil(l1d > 1000.0 ? l1d : 1000.0);

    double* p1 = (double*)malloc(sizeof(double) * (size_t)n);
    int32_t* Is = (int32_t*)malloc(sizeof(int32_t) * (size_t)I.l1);
    orc_stats S1;
    phase_estimate(g, st, I.l1, seed, 1, p1, &S1, Is);
    double l1 = (double)I.l1;
    double sumI = 0.0;
    for (uint64_t i = 0; i < I.l1; i++) sumI += Is[i];
    I.rho_tilde = sumI / l1;
    /* Proposition 2: Lambda = 1/(l(l-1)) * sum_{i<j} (|I_i| - |I_j|)^2 */
    double pair_sum = 0.0;
    for (uint64_t i = 0; i < I.l1; i++)
        for (uint64_t j = i + 1; j < I.l1; j++) {
            double dd = (double)(Is[i] - Is[j]);
            pair_sum += dd * dd;
        }
    I.Lambda = pair_sum / (l1 * (l1 - 1.0));
    double L8 = log(8.0 / delta), L4 = log(4.0 / delta);
    I.rho_hat = I.rho_tilde + sqrt(2.0 * I.Lambda * L8 / l1) + 7.0 * (double)I.D * L8 / (3.0 * (l1 - 1.0));
    double vmax = 0.0;
    for (int32_t v = 0; v < n; v++) {
        double b = p1[v] + sqrt(2.0 * p1[v] * L4 / l1) + L4 / (3.0 * l1);
        if (b > vmax) vmax = b;
    }
    I.v_hat = d_hat * d_hat * vmax;
    double lbound = orc_sample_size(d_hat, I.rho_hat, I.v_hat, eps, delta, &I.x_hat);
    I.l = (uint64_t)ceil(lbound);

    orc_stats S2;
    int32_t* Is2 = (int32_t*)malloc(sizeof(int32_t) * (size_t)(I.l > 0 ? I.l : 1));
    phase_estimate(g, st, I.l, seed, 2, p_out, &S2, Is2);
    I.overflow = S1.overflow + S2.overflow;
    if (info) *info = I;
    free(p1); free(Is); free(Is2);
    return I.overflow ? -2 : 0;
}

/* PercIS-DI: the data-independent variant the paper compares its bound with.
 * There is no first phase; the vertex-diameter bound D stands for rho-hat and
 * the largest possible value d-hat^2 / 4 for v-hat (so x-hat = d-hat / 2);
 * the l samples of phase 2 give p as in Algorithm 1. */
int orc_estimate_di(const orc_graph* g, const orc_states* st, double eps, double delta, uint64_t seed,
                    int64_t D, double* p_out, orc_estimate_info* info)
{
    orc_estimate_info I; memset(&I, 0, sizeof I);
    if (st->C == 0) return -1;
    int32_t n = g->n;
    I.D = D >= 0 ? D : orc_vertex_diam_ub(g);
    double d_hat = 1.0;
    for (int32_t v = 0; v < n; v++)
        if (st->S[v] > 0 && (double)st->C / st->S[v] > d_hat) d_hat = (double)st->C / st->S[v];
    I.d_hat = d_hat;
    I.rho_hat = (double)I.D;
    I.v_hat = d_hat * d_hat / 4.0;
    I.l = (uint64_t)ceil(orc_sample_size(d_hat, I.rho_hat, I.v_hat, eps, delta, &I.x_hat));
    orc_stats S2;
    int32_t* Is2 = (int32_t*)malloc(sizeof(int32_t) * (size_t)(I.l > 0 ? I.l : 1));
    phase_estimate(g, st, I.l, seed, 2, p_out, &S2, Is2);
    I.overflow = S2.overflow;
    if (info) *info = I;
    free(Is2);
    return I.overflow ? -2 : 0;
}
