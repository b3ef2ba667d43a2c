/*
 * Seeded synthetic graph generators (inputs only: no part of the PercIS
 * method lives here). Used by the tests and the benchmark to build the same
 * inputs for the oracle and for the HIP library.
 *
 *   wl_rmat   R-MAT edge draws (Chakrabarti, Zhan, Faloutsos, SDM 2004):
 *             every edge picks one of the four quadrants at each of `scale`
 *             levels with probabilities (a, b, c, 1-a-b-c).
 *   wl_ba     Barabasi-Albert preferential attachment (Science 1999): a seed
 *             clique on m+1 nodes, then every new node links to m distinct
 *             earlier nodes picked with probability proportional to degree.
 *   wl_csr    CSR from an edge list: drops self-loops, optionally adds the
 *             reverse of every edge, removes duplicates, sorts every row.
 *
 * The random source is splitmix64 (Steele, Lea, Flood, OOPSLA 2014), seeded
 * per generator call and, for the threaded R-MAT, per block of edges.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

static inline uint64_t splitmix64(uint64_t* s)
{
    uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline double unit(uint64_t* s) { return (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0); }

typedef struct {
    int scale; int64_t lo, hi; double a, b, c; uint64_t seed; int32_t* src; int32_t* dst;
} rmat_job;

static void* rmat_worker(void* arg)
{
    rmat_job* j = (rmat_job*)arg;
    const int64_t BLOCK = 1 << 16;
    for (int64_t base = j->lo; base < j->hi; base += BLOCK) {
        uint64_t s = j->seed ^ (0xD1B54A32D192ED03ULL * (uint64_t)(base / BLOCK + 1));
        int64_t end = base + BLOCK < j->hi ? base + BLOCK : j->hi;
        for (int64_t e = base; e < end; e++) {
            uint32_t u = 0, v = 0;
            for (int l = 0; l < j->scale; l++) {
                double r = unit(&s);
                u <<= 1; v <<= 1;
                if (r < j->a) { }
                else if (r < j->a + j->b) { v |= 1; }
                else if (r < j->a + j->b + j->c) { u |= 1; }
                else { u |= 1; v |= 1; }
            }
            j->src[e] = (int32_t)u; j->dst[e] = (int32_t)v;
        }
    }
    return NULL;
}

/* ne edge draws into src/dst; node ids are then relabelled by a seeded
 * Fisher-Yates permutation so that degree does not follow the id. */
void wl_rmat(int scale, int64_t ne, double a, double b, double c, uint64_t seed, int nthreads,
             int32_t* src, int32_t* dst)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 64) nthreads = 64;
    pthread_t th[64]; rmat_job jobs[64];
    const int64_t BLOCK = 1 << 16;
    int64_t nblocks = (ne + BLOCK - 1) / BLOCK;
    for (int i = 0; i < nthreads; i++) {
        int64_t b0 = nblocks * i / nthreads, b1 = nblocks * (i + 1) / nthreads;
        jobs[i] = (rmat_job){ scale, b0 * BLOCK, b1 * BLOCK < ne ? b1 * BLOCK : ne, a, b, c, seed, src, dst };
        pthread_create(&th[i], NULL, rmat_worker, &jobs[i]);
    }
    for (int i = 0; i < nthreads; i++) pthread_join(th[i], NULL);
    int64_t n = (int64_t)1 << scale;
    int32_t* perm = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    for (int64_t i = 0; i < n; i++) perm[i] = (int32_t)i;
    uint64_t s = seed ^ 0x5851F42D4C957F2DULL;
    for (int64_t i = n - 1; i > 0; i--) {
        int64_t j = (int64_t)(splitmix64(&s) % (uint64_t)(i + 1));
        int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
    for (int64_t e = 0; e < ne; e++) { src[e] = perm[src[e]]; dst[e] = perm[dst[e]]; }
    free(perm);
}

/* BA graph with n nodes (n > m), m links per new node; writes the edge list
 * (n_edges = m(m+1)/2 + (n-m-1) m edges) into src/dst. */
int64_t wl_ba(int32_t n, int32_t m, uint64_t seed, int32_t* src, int32_t* dst)
{
    int64_t ne = 0;
    int64_t cap_ends = (int64_t)m * (m + 1) + 2 * (int64_t)(n - m - 1) * m;
    int32_t* ends = (int32_t*)malloc(sizeof(int32_t) * (size_t)(cap_ends > 0 ? cap_ends : 1));
    int64_t nends = 0;
    for (int32_t u = 0; u <= m; u++)
        for (int32_t v = u + 1; v <= m; v++) {
            src[ne] = u; dst[ne] = v; ne++;
            ends[nends++] = u; ends[nends++] = v;
        }
    uint64_t s = seed;
    int32_t* pick = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
    for (int32_t v = m + 1; v < n; v++) {
        int32_t got = 0;
        while (got < m) {
            int32_t u = ends[splitmix64(&s) % (uint64_t)nends];
            int dup = 0;
            for (int32_t i = 0; i < got; i++) if (pick[i] == u) { dup = 1; break; }
            if (!dup) pick[got++] = u;
        }
        for (int32_t i = 0; i < m; i++) {
            src[ne] = v; dst[ne] = pick[i]; ne++;
            ends[nends++] = v; ends[nends++] = pick[i];
        }
    }
    free(pick); free(ends);
    return ne;
}

static int cmp_i32(const void* x, const void* y)
{
    int32_t a = *(const int32_t*)x, b = *(const int32_t*)y;
    return (a > b) - (a < b);
}

/* Pass 1: counts arcs per row (row_cnt[n], zeroed by the caller) and returns
 * the number of arcs before deduplication. */
int64_t wl_csr_count(int32_t n, int64_t ne, const int32_t* src, const int32_t* dst, int undirected, int64_t* row_cnt)
{
    int64_t tot = 0;
    for (int64_t e = 0; e < ne; e++) {
        if (src[e] == dst[e]) continue;
        row_cnt[src[e]]++; tot++;
        if (undirected) { row_cnt[dst[e]]++; tot++; }
    }
    (void)n;
    return tot;
}

/* Pass 2: fills col (capacity = pass-1 total) using row_ptr (exclusive prefix
 * of row_cnt, n+1 entries, rewritten in place with the deduplicated row
 * offsets); returns the final number of arcs. */
int64_t wl_csr_fill(int32_t n, int64_t ne, const int32_t* src, const int32_t* dst, int undirected,
                    int64_t* row_ptr, int32_t* col)
{
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    memcpy(fill, row_ptr, sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t e = 0; e < ne; e++) {
        if (src[e] == dst[e]) continue;
        col[fill[src[e]]++] = dst[e];
        if (undirected) col[fill[dst[e]]++] = src[e];
    }
    free(fill);
    int64_t out = 0;
    for (int32_t v = 0; v < n; v++) {
        int64_t b = row_ptr[v], e = row_ptr[v + 1];
        qsort(col + b, (size_t)(e - b), sizeof(int32_t), cmp_i32);
        row_ptr[v] = out;
        for (int64_t i = b; i < e; i++)
            if (i == b || col[i] != col[i - 1]) col[out++] = col[i];
    }
    row_ptr[n] = out;
    return out;
}
