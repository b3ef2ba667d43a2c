"""Seeded synthetic inputs for the PercIS hot path (graphs and states).

This module holds no part of the method: it only builds graphs (CSR) and
quantised percolation states k_v in 0..65535 (x_v = k_v / 65535). Both the
oracle and the HIP library consume what it returns, so that their results can
be compared element by element.

The graphs stand in for the paper's SNAP networks (Table I), which are not
available here: R-MAT and Barabasi-Albert graphs give power-law degrees like
the web and social graphs of the paper, Erdos-Renyi graphs are the control.
State generators mirror the paper's settings (Section IV-A): uniform states
(UN), random seeds (RS), random seeds spread (RSS) and the isolated component
(IC), plus the skewed and Beta(1/2, 1/2) mixes used by the benchmarks.
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libworkloads.so")
_lib = None

K = 65535


def build(force=True):
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-shared", "-fPIC", "-pthread", "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = C.CDLL(_LIB)
        P = C.c_void_p
        lib.wl_rmat.argtypes = [C.c_int, C.c_int64, C.c_double, C.c_double, C.c_double, C.c_uint64, C.c_int, P, P]
        lib.wl_rmat.restype = None
        lib.wl_ba.argtypes = [C.c_int32, C.c_int32, C.c_uint64, P, P]
        lib.wl_ba.restype = C.c_int64
        lib.wl_csr_count.argtypes = [C.c_int32, C.c_int64, P, P, C.c_int, P]
        lib.wl_csr_count.restype = C.c_int64
        lib.wl_csr_fill.argtypes = [C.c_int32, C.c_int64, P, P, C.c_int, P, P]
        lib.wl_csr_fill.restype = C.c_int64
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


class Graph:
    """CSR graph: row_ptr int32[n+1], col int32[m]; rows sorted, no loops or
    duplicates; an undirected graph stores both arcs of every edge."""

    def __init__(self, n, row_ptr, col, directed, name=""):
        self.n = int(n)
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.m = int(self.col.size)
        self.directed = bool(directed)
        self.name = name

    def degrees(self):
        return np.diff(self.row_ptr.astype(np.int64))

    def edges(self):
        src = np.repeat(np.arange(self.n, dtype=np.int32), self.degrees())
        return src, self.col


def csr_from_edges(n, src, dst, directed, name=""):
    lib = _load()
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    ne = int(src.size)
    cnt = np.zeros(n + 1, np.int64)
    tot = lib.wl_csr_count(n, ne, _p(src), _p(dst), int(not directed), _p(cnt))
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(cnt[:n], out=rp[1:])
    col = np.empty(max(int(tot), 1), np.int32)
    m = lib.wl_csr_fill(n, ne, _p(src), _p(dst), int(not directed), _p(rp), _p(col))
    if m >= 2 ** 31:
        raise ValueError("graph has %d arcs; int32 CSR holds at most 2^31-1" % m)
    return Graph(n, rp.astype(np.int32), col[:m].copy(), directed, name)


# ----------------------------------------------------------------- families
def er_graph(n, m, seed):
    """G(n, m): m distinct unordered non-loop pairs drawn uniformly with
    numpy default_rng(seed); both arcs stored."""
    rng = np.random.default_rng(seed)
    keys = set()
    chosen = []
    while len(chosen) < m:
        u, v = rng.integers(0, n, size=2)
        if u == v:
            continue
        a, b = (int(u), int(v)) if u < v else (int(v), int(u))
        if (a, b) in keys:
            continue
        keys.add((a, b))
        chosen.append((a, b))
    e = np.array(chosen, dtype=np.int32).reshape(-1, 2)
    return csr_from_edges(n, e[:, 0], e[:, 1], directed=False, name="er_%d_%d" % (n, m))


def rmat_graph(scale, edge_factor=16, a=0.57, b=0.19, c=0.19, seed=1, directed=False, threads=None):
    n = 1 << scale
    ne = n * edge_factor
    src = np.empty(ne, np.int32)
    dst = np.empty(ne, np.int32)
    thr = threads or min(16, os.cpu_count() or 1)
    _load().wl_rmat(scale, ne, a, b, c, seed, thr, _p(src), _p(dst))
    g = csr_from_edges(n, src, dst, directed,
                       name="rmat%d_%s" % (scale, "dir" if directed else "undir"))
    del src, dst
    return g


def ba_graph(n, m, seed):
    ne = m * (m + 1) // 2 + (n - m - 1) * m
    src = np.empty(ne, np.int32)
    dst = np.empty(ne, np.int32)
    got = _load().wl_ba(n, m, seed, _p(src), _p(dst))
    assert got == ne
    return csr_from_edges(n, src, dst, directed=False, name="ba_%d_%d" % (n, m))


def from_edge_list(n, edges, directed=False, name=""):
    e = np.array(edges, dtype=np.int32).reshape(-1, 2)
    return csr_from_edges(n, e[:, 0], e[:, 1], directed, name)


def path_graph(n):
    return from_edge_list(n, [(i, i + 1) for i in range(n - 1)], name="path%d" % n)


def star_graph(n):
    return from_edge_list(n, [(0, i) for i in range(1, n)], name="star%d" % n)


def cycle_graph(n):
    return from_edge_list(n, [(i, (i + 1) % n) for i in range(n)], name="cycle%d" % n)


def complete_graph(n):
    return from_edge_list(n, [(i, j) for i in range(n) for j in range(i + 1, n)], name="K%d" % n)


def grid_graph(a, b):
    """a x b grid; node (i, j) has id i*b + j."""
    e = []
    for i in range(a):
        for j in range(b):
            if i + 1 < a:
                e.append((i * b + j, (i + 1) * b + j))
            if j + 1 < b:
                e.append((i * b + j, i * b + j + 1))
    return from_edge_list(a * b, e, name="grid%dx%d" % (a, b))


def diamond_chain(k):
    """k diamonds in a row: hubs h_0..h_k (ids 0..k), between h_i and h_{i+1}
    two middle nodes (ids k+1+2i, k+2+2i). sigma(h_0, h_k) = 2^k."""
    e = []
    for i in range(k):
        a, b = k + 1 + 2 * i, k + 2 + 2 * i
        e += [(i, a), (i, b), (a, i + 1), (b, i + 1)]
    return from_edge_list(k + 1 + 2 * k, e, name="diamonds%d" % k)


def layered_graph(sizes, directed=False):
    """Layers of the given sizes, consecutive layers completely joined (arcs
    from each layer to the next if directed); ids layer by layer. Between the
    first node and the last, sigma is the product of the inner layer sizes."""
    starts = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    e = []
    for i in range(len(sizes) - 1):
        for u in range(starts[i], starts[i + 1]):
            for v in range(starts[i + 1], starts[i + 2]):
                e.append((u, v))
    return from_edge_list(int(starts[-1]), e, directed=directed,
                          name="layers%s%s" % ("-".join(map(str, sizes)), "d" if directed else ""))


def complete_bipartite(a, b):
    return from_edge_list(a + b, [(i, a + j) for i in range(a) for j in range(b)], name="K%d,%d" % (a, b))


def prop7_instance(n):
    """Directed instance of the lower-bound proposition (Section III-D):
    path a->b->c (ids 0,1,2); H = ids 3..n-1 strongly connected by a directed
    cycle; an arc from node 3 (in H) to a. States: x_a = 1, x_b = 0,
    x_c = 1/2 (quantised to k = 32768 by rint), H at 0."""
    e = [(0, 1), (1, 2)]
    H = list(range(3, n))
    for i, u in enumerate(H):
        e.append((u, H[(i + 1) % len(H)]))
    e.append((3, 0))
    g = from_edge_list(n, e, directed=True, name="prop7_%d" % n)
    k = np.zeros(n, np.uint16)
    k[0] = K
    k[2] = quantise(np.array([0.5]))[0]
    return g, k


def random_small_graph(n, p, seed, directed=False):
    rng = np.random.default_rng(seed)
    e = []
    for u in range(n):
        for v in range(n):
            if u == v or (not directed and v <= u):
                continue
            if rng.random() < p:
                e.append((u, v))
    return from_edge_list(n, e if e else [(0, 1)], directed=directed, name="rand%d" % n)


# ------------------------------------------------------------------- states
def quantise(x):
    """k = rint(65535 x) (round half to even), clipped to [0, 65535]."""
    return np.clip(np.rint(np.asarray(x, dtype=np.float64) * K), 0, K).astype(np.uint16)


def uniform_states(n, rng):
    """UN setting: k uniform on {0..65535}."""
    return rng.integers(0, K + 1, size=n, dtype=np.int64).astype(np.uint16)


def skewed_states(n, rng, zero_frac=0.95):
    """k = 0 with probability zero_frac, else uniform on {0..65535}."""
    k = rng.integers(0, K + 1, size=n, dtype=np.int64)
    k[rng.random(n) < zero_frac] = 0
    return k.astype(np.uint16)


def beta_states(n, rng, a=0.5, b=0.5):
    return quantise(rng.beta(a, b, size=n))


def rs_states(n, rng, seeds=50):
    """RS setting: `seeds` random nodes at state 1, all others at 0."""
    k = np.zeros(n, np.uint16)
    k[rng.choice(n, size=min(seeds, n), replace=False)] = K
    return k


def rss_states(g, rng):
    """RSS setting: log n random seeds; x_v = max over seeds of 4^-d(seed, v)."""
    n = g.n
    ns = max(1, int(np.log(n)))
    seeds = rng.choice(n, size=ns, replace=False)
    x = np.zeros(n)
    rp, col = g.row_ptr, g.col
    for s in seeds:
        dist = np.full(n, -1, np.int64)
        dist[s] = 0
        frontier = [int(s)]
        while frontier:
            nxt = []
            for u in frontier:
                for v in col[rp[u]:rp[u + 1]]:
                    if dist[v] < 0:
                        dist[v] = dist[u] + 1
                        nxt.append(int(v))
            frontier = nxt
        reach = dist >= 0
        x[reach] = np.maximum(x[reach], 4.0 ** (-dist[reach].astype(np.float64)))
    return quantise(x)


def with_isolated_component(g, length=50, directed=None):
    """IC setting: appends a path of `length` nodes (bidirectional arcs);
    undirected graphs keep it isolated, directed ones get one arc from node 0
    to its first node. Returns (graph, k) with the first half of the path at
    state 1 and everything else at 0."""
    directed = g.directed if directed is None else directed
    n0 = g.n
    src, dst = g.edges()
    extra = []
    for i in range(length - 1):
        extra.append((n0 + i, n0 + i + 1))
        extra.append((n0 + i + 1, n0 + i))
    if directed:
        extra.append((0, n0))
    e = np.array(extra, dtype=np.int32).reshape(-1, 2)
    src2 = np.concatenate([src, e[:, 0]])
    dst2 = np.concatenate([dst, e[:, 1]])
    h = csr_from_edges(n0 + length, src2, dst2, directed, name=g.name + "+ic")
    k = np.zeros(n0 + length, np.uint16)
    k[n0:n0 + length // 2] = K
    return h, k


# ------------------------------------------------------ benchmark workloads
def workload_er1000(seed=1):
    """ER G(n=1000, m=5000), undirected; k uniform; numpy default_rng(seed)."""
    rng = np.random.default_rng(seed)
    g = er_graph(1000, 5000, rng)
    k = uniform_states(g.n, rng)
    return g, k


def workload_rmat18(seed=1):
    """R-MAT scale 18, edge factor 16, (0.57, 0.19, 0.19, 0.05), undirected;
    95% of states 0, the rest uniform."""
    g = rmat_graph(18, 16, seed=seed, directed=False)
    k = skewed_states(g.n, np.random.default_rng(seed), 0.95)
    return g, k


def workload_rmat24_directed(seed=1):
    """R-MAT scale 24, edge factor 16, directed; x ~ Beta(1/2, 1/2)."""
    g = rmat_graph(24, 16, seed=seed, directed=True)
    k = beta_states(g.n, np.random.default_rng(seed))
    return g, k


def workload_ba_batch(count=64, m=4, seed=1, lo=1e4, hi=1e6):
    """`count` BA graphs with n log-uniform on [lo, hi], each with its own
    uniform states; seeds from SeedSequence(seed).spawn(count)."""
    out = []
    for child in np.random.SeedSequence(seed).spawn(count):
        rng = np.random.default_rng(child)
        n = int(round(10 ** (np.log10(lo) + (np.log10(hi) - np.log10(lo)) * rng.random())))
        g = ba_graph(n, m, int(rng.integers(0, 2 ** 63)))
        out.append((g, uniform_states(n, rng)))
    return out
