"""GPU parity: the HIP library against the CPU oracle, through the C ABI.

Integer outputs (hit counts, sample statistics, paths, shortest-path counts,
overflow flags) must be bit-identical. Floating outputs of percis_estimate
are compared with the tolerances stated next to each check."""
import math

import numpy as np
import pytest

import brute as B
import oracle as O
import workloads as W
from gpu_common import gpu_context, gpu_hits, oracle_hits, oracle_objects, same_stats

pytestmark = pytest.mark.gpu


def small_graphs():
    out = [W.path_graph(7), W.star_graph(6), W.cycle_graph(8), W.cycle_graph(7), W.complete_graph(5),
           W.grid_graph(3, 4), W.diamond_chain(3), W.complete_bipartite(3, 4)]
    for sd in range(6):
        out.append(W.random_small_graph(9 + sd % 3, 0.3, sd, directed=False))
        out.append(W.random_small_graph(8 + sd % 4, 0.25, 100 + sd, directed=True))
    return out


def test_debug_path_exhaustive_small_graphs():
    """Every (s, t, r) on 20 small graphs: L, sigma and the path equal the
    oracle's, which the CPU suite pins to the sorted enumeration."""
    from paper_2509_11454_amd import percis as P
    for g in small_graphs():
        c = P.Context(0)
        c.load_csr(g.n, g.row_ptr, g.col, directed=g.directed)
        og = O.Graph(g.n, g.row_ptr, g.col, g.directed)
        for s in range(g.n):
            for t in range(g.n):
                if s == t:
                    continue
                L0, sig0, _ = O.path(og, s, t, 0)
                rs = range(sig0) if L0 >= 0 else [0]
                for r in rs:
                    L, sig, ovf, p = c.debug_path(s, t, r)
                    assert ovf == 0
                    assert L == L0, (g.name, s, t)
                    if L0 < 0:
                        continue
                    assert sig == sig0
                    assert p == O.path(og, s, t, r)[2], (g.name, s, t, r)
        c.close()


def test_debug_path_sigma_extremes():
    from paper_2509_11454_amd import percis as P
    # 34 x 35 grid: sigma = C(67, 33) < 2^64, walk with r at both ends
    g = W.grid_graph(34, 35)
    c = P.Context(0)
    c.load_csr(g.n, g.row_ptr, g.col)
    og = O.Graph(g.n, g.row_ptr, g.col)
    sig = math.comb(67, 33)
    for r in [0, 1, sig // 2, sig - 2, sig - 1]:
        L, s2, ovf, p = c.debug_path(0, g.n - 1, r)
        assert (L, s2, ovf) == (67, sig, 0)
        assert p == O.path(og, 0, g.n - 1, r)[2]
    # 35 x 35: sigma = C(68, 34) >= 2^64 -> overflow flagged
    g = W.grid_graph(35, 35)
    c.load_csr(g.n, g.row_ptr, g.col)
    L, s2, ovf, p = c.debug_path(0, g.n - 1, 0)
    assert L == 68 and ovf == 1 and p is None
    # diamond chains: 2^63 ok, 2^64 overflows
    for k, want in [(63, 0), (64, 1)]:
        g = W.diamond_chain(k)
        c.load_csr(g.n, g.row_ptr, g.col)
        og = O.Graph(g.n, g.row_ptr, g.col)
        L, s2, ovf, p = c.debug_path(0, k, 2 ** 63 - 1 if k == 63 else 0)
        assert L == 2 * k and ovf == want
        if not want:
            assert s2 == 2 ** 63 and p == O.path(og, 0, k, 2 ** 63 - 1)[2]
    c.close()


def test_walk_many_predecessors_and_arc_overflow():
    """Nodes with more than 64 DAG predecessors (radix selection over the arc
    list), and searches that record more DAG arcs than a slot keeps (16384 in
    a per-node slot; [1, 150, 150, 1] records 22650, of which the level into
    distance 2 alone 22500), which make the walk scan in-rows instead for
    those steps, while steps whose own segment of the list is complete still
    use it; the paths still equal the oracle's."""
    from paper_2509_11454_amd import percis as P
    for g in [W.layered_graph([1, 100, 100, 1]), W.layered_graph([1, 150, 150, 1]), W.layered_graph([1, 3, 70, 2, 1]),
              W.layered_graph([1, 90, 60, 1], directed=True), W.layered_graph([1, 65, 1])]:
        c = P.Context(0)
        c.load_csr(g.n, g.row_ptr, g.col, directed=g.directed)
        og = O.Graph(g.n, g.row_ptr, g.col, g.directed)
        s, t = 0, g.n - 1
        L0, sig0, _ = O.path(og, s, t, 0)
        assert L0 > 0
        for r in sorted({0, 1, sig0 // 3, sig0 // 2, sig0 - 2, sig0 - 1}):
            L, sig, ovf, p = c.debug_path(s, t, r)
            assert (L, sig, ovf) == (L0, sig0, 0), g.name
            assert p == O.path(og, s, t, r)[2], (g.name, r)
        c.close()


@pytest.mark.parametrize("k,directed", [(40, False), (70, False), (300, False), (300, True), (5000, False)])
def test_walk_predecessor_order_is_caller_order(k, directed):
    """s -> k middle nodes -> t, each middle node with 0..6 pendant leaves,
    every id shuffled: the library numbers nodes by degree, so t's
    predecessors sit in another order internally than by caller id. Every
    walk step must still take them in caller id order: up to 64 predecessors
    from the arc list in LDS, 65..4096 by radix selection on their caller
    ids, more by the in-row scan in caller order. Paths for r across
    [0, sigma) equal the oracle's."""
    from paper_2509_11454_amd import percis as P
    rng = np.random.default_rng(1000 + k + directed)
    pend = rng.integers(0, 7, size=k)
    n = 2 + k + int(pend.sum())
    edges, leaf = [], 2 + k
    for i in range(k):
        m = 2 + i
        edges += [(0, m), (m, 1)]
        for _ in range(int(pend[i])):
            edges.append((m, leaf))
            leaf += 1
    lab = rng.permutation(n)
    g = W.from_edge_list(n, [(int(lab[a]), int(lab[b])) for a, b in edges], directed=directed)
    s, t = int(lab[0]), int(lab[1])
    c = P.Context(0)
    c.load_csr(g.n, g.row_ptr, g.col, directed=g.directed)
    og = O.Graph(g.n, g.row_ptr, g.col, g.directed)
    L0, sig0, _ = O.path(og, s, t, 0)
    assert (L0, sig0) == (2, k)
    rs = {0, 1, k // 3, k // 2, k - 2, k - 1} | {int(x) for x in rng.integers(0, k, size=24)}
    for r in sorted(rs):
        L, sig, ovf, p = c.debug_path(s, t, r)
        assert (L, sig, ovf) == (L0, sig0, 0)
        assert p == O.path(og, s, t, r)[2], (k, directed, r)
    c.close()


@pytest.mark.parametrize("directed,compact", [(False, 1), (False, 2), (True, 1), (True, 2)])
def test_walk_caller_order_sampling(directed, compact):
    """Sampling parity where walk steps pick among 300 predecessors of mixed
    degree: 40 sources joined to 300 middle nodes (0..6 pendant leaves each),
    all joined to t, ids shuffled; t has state 0 and every other node 65535,
    so every pair ends at t and the pairs from a source walk through t's 300
    predecessors. 2e4 samples on per-node and on compact slots."""
    rng = np.random.default_rng(77 + directed)
    q, k = 40, 300
    pend = rng.integers(0, 7, size=k)
    n = 1 + q + k + int(pend.sum())
    t0, edges, leaf = 0, [], 1 + q + k
    for i in range(k):
        m = 1 + q + i
        edges += [(src, m) for src in range(1, 1 + q)] + [(m, t0)]
        for _ in range(int(pend[i])):
            edges.append((m, leaf))
            leaf += 1
    lab = rng.permutation(n)
    g = W.from_edge_list(n, [(int(lab[a]), int(lab[b])) for a, b in edges], directed=directed)
    kk = np.full(n, 65535, np.uint16)
    kk[lab[t0]] = 0
    og, st = oracle_objects(g, kk)
    ho, so = oracle_hits(og, st, 0, 20000, 3)
    from paper_2509_11454_amd import percis as P
    c = gpu_context(g, kk)
    c.set_option(P.OPT_COMPACT, compact)
    hg, sg = gpu_hits(c, 0, 20000, 3)
    assert np.array_equal(ho, hg)
    same_stats(so, sg)
    c.close()


@pytest.mark.parametrize("sizes,directed", [([1, 3, 70, 2, 1], False), ([5, 40, 80, 40, 5], False),
                                             ([2, 90, 60, 3], True)])
def test_layered_sampling_parity(sizes, directed):
    """Sampling on layered graphs (walk steps over many predecessors, DAGs
    with more arcs than a slot records): bit-identical to the oracle."""
    g = W.layered_graph(sizes, directed=directed)
    k = W.uniform_states(g.n, np.random.default_rng(len(sizes)))
    og, st = oracle_objects(g, k)
    ho, so = oracle_hits(og, st, 0, 3000, 21)
    c = gpu_context(g, k)
    hg, sg = gpu_hits(c, 0, 3000, 21)
    assert np.array_equal(ho, hg)
    same_stats(so, sg)


def test_er1000_parity():
    """ER G(1000, 5000), uniform states, 10^4 samples, seed 1: bit-identical."""
    g, k = W.workload_er1000()
    og, st = oracle_objects(g, k)
    ho, so = oracle_hits(og, st, 0, 10000, 1)
    c = gpu_context(g, k)
    hg, sg = gpu_hits(c, 0, 10000, 1)
    assert np.array_equal(ho, hg)
    same_stats(so, sg)
    assert int(hg.sum()) == sg["sum_I"]


@pytest.mark.parametrize("slots,block,bitmaps", [(1, 0, 0), (3, 256, 1), (37, 512, 2), (0, 1024, 1),
                                                  (0, 256, 2), (5, 1024, 2), (0, 128, 1), (7, 128, 2),
                                                  (0, 64, 2), (9, 64, 1), (1, 64, 2)])
def test_launch_shape_invariance(slots, block, bitmaps):
    """Hit counts and statistics do not depend on the number of slots, the
    threads per sample or where the visited bitmaps live."""
    from paper_2509_11454_amd import percis as P
    g, k = W.workload_er1000()
    c0 = gpu_context(g, k)
    h0, s0 = gpu_hits(c0, 0, 3000, 7)
    c = P.Context(0)
    c.set_option(P.OPT_SLOTS, slots)
    c.set_option(P.OPT_BLOCK, block)
    c.set_option(P.OPT_BITMAPS, bitmaps)
    c.load_csr(g.n, g.row_ptr, g.col)
    c.set_states(k)
    h, s = gpu_hits(c, 0, 3000, 7)
    assert np.array_equal(h0, h)
    same_stats(s0, s)
    if block:
        assert c.get_option(P.OPT_BLOCK) == block
    if bitmaps:
        assert c.get_option(P.OPT_BITMAPS) == bitmaps


def test_rmat18_shapes_agree():
    """On the benchmark graph, LDS and device-memory bitmaps and different
    block sizes give identical hits on a window of samples."""
    from paper_2509_11454_amd import percis as P
    g, k = W.workload_rmat18()
    ref = None
    for block, bitmaps in [(1024, 2), (512, 1), (256, 2), (128, 1), (64, 2), (64, 1)]:
        c = P.Context(0)
        c.set_option(P.OPT_BLOCK, block)
        c.set_option(P.OPT_BITMAPS, bitmaps)
        c.load_csr(g.n, g.row_ptr, g.col)
        c.set_states(k)
        h, s = gpu_hits(c, 5000, 20000, 3)
        if ref is None:
            ref = (h, s)
        else:
            assert np.array_equal(ref[0], h)
            same_stats(ref[1], s)
        c.close()


def test_ranges_add_up_and_accumulate():
    g, k = W.workload_er1000()
    c = gpu_context(g, k)
    h_all, _ = gpu_hits(c, 0, 5000, 3, phase=1)
    h_a, _ = gpu_hits(c, 0, 1234, 3, phase=1)
    h_b, _ = gpu_hits(c, 1234, 5000 - 1234, 3, phase=1)
    assert np.array_equal(h_all, h_a + h_b)
    acc = h_a.copy()
    c.sample_range(1234, 5000 - 1234, 3, 1, hits=acc, accumulate=True)
    assert np.array_equal(acc, h_all)


def special_cases():
    rng = np.random.default_rng(5)
    cases = []
    for g in [W.path_graph(40), W.star_graph(30), W.cycle_graph(31), W.cycle_graph(32),
              W.complete_bipartite(6, 9), W.grid_graph(12, 17), W.diamond_chain(20), W.complete_graph(12)]:
        cases.append((g, W.uniform_states(g.n, rng)))
    for sd in range(3):
        g = W.random_small_graph(60, 0.06, 300 + sd, directed=True)
        cases.append((g, W.uniform_states(g.n, rng)))
    g0 = W.er_graph(300, 700, 9)
    cases.append(W.with_isolated_component(g0, 50))
    g1 = W.random_small_graph(80, 0.05, 17, directed=True)
    cases.append(W.with_isolated_component(g1, 20))
    cases.append(W.prop7_instance(40))
    g2 = W.er_graph(400, 1200, 3)
    cases.append((g2, W.rs_states(g2.n, rng, 10)))
    cases.append((g2, W.rss_states(g2, rng)))
    g3 = W.ba_graph(2000, 4, 11)
    cases.append((g3, W.skewed_states(g3.n, rng)))
    return cases


@pytest.mark.parametrize("ci", range(17))
def test_special_graph_parity(ci):
    g, k = special_cases()[ci]
    og, st = oracle_objects(g, k)
    ho, so = oracle_hits(og, st, 0, 4000, 11 + ci)
    c = gpu_context(g, k)
    hg, sg = gpu_hits(c, 0, 4000, 11 + ci)
    assert np.array_equal(ho, hg), g.name
    same_stats(so, sg)


def test_wide_sigma_parity():
    """35 x 35 grid with the corner pair likely: the pair (0, far corner) has
    C(68, 34) >= 2^64 shortest paths, so its samples take the 128-bit path (r
    drawn at 128 bits); hits and statistics are bit-identical to the oracle,
    and nothing overflows."""
    g = W.grid_graph(35, 35)
    k = np.full(g.n, 32768, np.uint16)
    k[0], k[g.n - 1] = 65535, 0
    og, st = oracle_objects(g, k)
    ho, so = oracle_hits(og, st, 0, 6000, 2)
    assert so["overflow"] == 0
    # the corner pair is among the samples
    assert any(O.draw_pair(st, 2, 0, i)[:2] in ((0, g.n - 1), (g.n - 1, 0)) for i in range(6000))
    c = gpu_context(g, k)
    hg, sg = gpu_hits(c, 0, 6000, 2)
    assert np.array_equal(ho, hg)
    same_stats(so, sg)


def test_overflow_parity():
    """70 x 70 grid with the corner pair likely: C(138, 69) >= 2^128 shortest
    paths saturate even the 128-bit counts; those samples are counted, add no
    hits, and the call reports PERCIS_E_SIGMA_OVERFLOW with the first index."""
    from paper_2509_11454_amd import percis as P
    g = W.grid_graph(70, 70)
    k = np.full(g.n, 32768, np.uint16)
    k[0], k[g.n - 1] = 65535, 0
    og, st = oracle_objects(g, k)
    ho, so = oracle_hits(og, st, 0, 1500, 2)
    assert so["overflow"] > 0
    c = gpu_context(g, k)
    h = np.zeros(g.n, np.uint32)
    with pytest.raises(P.PercisError) as e:
        c.sample_range(0, 1500, 2, 0, hits=h)
    assert e.value.status == P.E_SIGMA_OVERFLOW
    hg, sg = gpu_hits(c, 0, 1500, 2, allow_overflow=True)
    assert np.array_equal(ho, hg)
    same_stats(so, sg)


def diamond_path(k, r):
    out = [0]
    for i in range(k):
        out.append(k + 1 + 2 * i + ((r >> i) & 1))
        out.append(i + 1)
    return out


def test_debug_path_wide():
    """The 128-bit path: diamond chains (sigma = 2^k, the path is the binary
    expansion of r, k up to 127; k = 128 saturates), grid corners on both
    sides of 2^128 against the oracle, and agreement with the 64-bit path
    below 2^64."""
    from paper_2509_11454_amd import percis as P
    rng = np.random.default_rng(17)
    c = P.Context(0)
    for k in (64, 100, 127, 128):
        g = W.diamond_chain(k)
        c.load_csr(g.n, g.row_ptr, g.col)
        if k == 128:
            L, sig, ovf, p = c.debug_path_wide(0, k, 0)
            assert L == 256 and ovf == 1 and p is None
            continue
        for r in [0, 1, 2 ** k - 1, 2 ** (k - 1)] + [int(rng.integers(0, 2 ** 62)) << (k - 62) for _ in range(4)]:
            L, sig, ovf, p = c.debug_path_wide(0, k, r)
            assert (L, sig, ovf) == (2 * k, 2 ** k, 0)
            assert p == diamond_path(k, r)
    for a in (35, 66, 70):
        g = W.grid_graph(a, a)
        c.load_csr(g.n, g.row_ptr, g.col)
        og = O.Graph(g.n, g.row_ptr, g.col)
        L0, sig0, _ = O.path(og, 0, g.n - 1, 0)
        if sig0 == O.SIGMA_SATURATED:
            L, sig, ovf, p = c.debug_path_wide(0, g.n - 1, 0)
            assert (L, ovf, p) == (L0, 1, None)
            continue
        for r in (0, 1, sig0 // 3, sig0 - 1):
            L, sig, ovf, p = c.debug_path_wide(0, g.n - 1, r)
            assert (L, sig, ovf) == (L0, sig0, 0)
            assert p == O.path(og, 0, g.n - 1, r)[2]
    for g in small_graphs()[:6]:
        c.load_csr(g.n, g.row_ptr, g.col, directed=g.directed)
        for s_, t_ in ((0, g.n - 1), (1, 2), (g.n - 1, 0)):
            a64 = c.debug_path(s_, t_, 0)
            a128 = c.debug_path_wide(s_, t_, 0)
            assert a64 == a128
    c.close()


def test_estimate_parity():
    """percis_estimate against the oracle's Algorithm 1. Integer quantities
    (l1, D) and the phase-1 statistics are exact; d_hat, rho_hat, v_hat agree to
    1e-12 relative (same formulas, different summation order); l agrees up to
    the resolution of the two supremum searches (1e-6 relative, +1). The
    phase-2 hits of the oracle's l are bit-identical on the device."""
    g, k = W.workload_er1000()
    og, st = oracle_objects(g, k)
    c = gpu_context(g, k)
    for eps, delta, seed in [(0.01, 0.1, 1), (0.05, 0.05, 2)]:
        rc, po, io = O.estimate(og, st, eps, delta, seed)
        assert rc == 0
        pg, ig = c.estimate(eps, delta, seed)
        assert ig["l1"] == io["l1"] and ig["D"] == io["D"]
        for key in ("d_hat", "rho_tilde", "Lambda", "rho_hat", "v_hat", "x_hat"):
            assert abs(ig[key] - io[key]) <= 1e-12 * max(1.0, abs(io[key])), key
        assert abs(ig["l"] - io["l"]) <= 1 + 1e-6 * io["l"]
        h2o, _ = O.sample_range(og, st, 0, io["l"], seed, 2)
        h2g, _ = gpu_hits(c, 0, io["l"], seed, phase=2)
        assert np.array_equal(h2o, h2g)
        if ig["l"] == io["l"]:
            assert np.allclose(pg, po, rtol=1e-12, atol=1e-15)
        p_exact = O.exact(og, st)
        assert np.abs(pg - p_exact).max() <= eps


def test_estimate_di_parity():
    """PercIS-DI against the oracle: D and the data-independent rho_hat, v_hat,
    x_hat agree (d_hat to 1e-12 relative), l up to the resolution of the two
    supremum searches; the phase-2 hits of the oracle's l are bit-identical,
    and with equal l so is the estimate (to the double formula's rounding)."""
    g, k = W.workload_er1000()
    og, st = oracle_objects(g, k)
    c = gpu_context(g, k)
    for eps, delta, seed in [(0.05, 0.1, 5), (0.1, 0.05, 6)]:
        rc, po, io = O.estimate_di(og, st, eps, delta, seed)
        assert rc == 0
        pg, ig = c.graph_estimate_di(0, eps, delta, seed)
        assert ig["l1"] == 0 and ig["D"] == io["D"] and ig["rho_hat"] == io["rho_hat"]
        for key in ("d_hat", "v_hat", "x_hat"):
            assert abs(ig[key] - io[key]) <= 1e-12 * max(1.0, abs(io[key])), key
        assert abs(ig["l"] - io["l"]) <= 1 + 1e-6 * io["l"]
        h2o, _ = O.sample_range(og, st, 0, io["l"], seed, 2)
        h2g, _ = gpu_hits(c, 0, io["l"], seed, phase=2)
        assert np.array_equal(h2o, h2g)
        if ig["l"] == io["l"]:
            assert np.allclose(pg, po, rtol=1e-12, atol=1e-15)
        # the data-dependent bound is the smaller one
        _, i2 = c.estimate(eps, delta, seed)
        assert i2["l"] <= ig["l"]


def test_device_pointer_inputs():
    import torch
    from paper_2509_11454_amd import percis as P
    g, k = W.workload_er1000()
    c = P.Context(0)
    c.load_csr(g.n, torch.from_numpy(g.row_ptr).cuda(), torch.from_numpy(g.col).cuda())
    c.set_states(torch.from_numpy(k.view(np.int16)).cuda())
    hits, st = c.sample(2000, 5)
    torch.cuda.synchronize()
    og, sto = oracle_objects(g, k)
    ho, so = oracle_hits(og, sto, 0, 2000, 5)
    assert np.array_equal(hits.cpu().numpy().view(np.uint32), ho)
    same_stats(so, st)


def test_directed_prop7_estimate():
    """Directed instance of Proposition 7 with a caller-supplied D: the
    estimate of p(b) meets eps and every other node stays at 0."""
    g, k = W.prop7_instance(30)
    c = gpu_context(g, k)
    c.set_vertex_diameter(g.n - 2)
    p, info = c.estimate(0.05, 0.1, 3)
    og, st = oracle_objects(g, k)
    pe = O.exact(og, st)
    assert np.abs(p - pe).max() <= 0.05
    assert np.all(p[[0] + list(range(2, g.n))] == 0.0)


def test_tasks_many_graphs_one_launch():
    """Tasks on five graphs (undirected, directed, tiny, with isolated nodes)
    in one launch: every task's hits and statistics equal the oracle's for
    its own graph, range, seed and phase, whatever the mix."""
    import torch
    from paper_2509_11454_amd import percis as P
    rng = np.random.default_rng(21)
    graphs = [W.workload_er1000(), (W.ba_graph(3000, 4, 5), None), (W.random_small_graph(70, 0.05, 8, True), None),
              (W.path_graph(30), None), W.with_isolated_component(W.er_graph(200, 500, 4), 30)]
    graphs = [(g, k if k is not None else W.uniform_states(g.n, rng)) for g, k in graphs]
    c = P.Context(0)
    g0, k0 = graphs[0]
    c.load_csr(g0.n, g0.row_ptr, g0.col)
    c.set_states(k0)
    ids = [0] + [c.add_graph(g.n, g.row_ptr, g.col, k, directed=g.directed) for g, k in graphs[1:]]
    assert c.graph_info(ids[1])[0] == graphs[1][0].n
    tasks = []
    for i, (gid, (g, k)) in enumerate(zip(ids, graphs)):
        for j, (first, count) in enumerate([(0, 700), (5000 + 13 * i, 300)]):
            tasks.append(dict(graph=gid, first=first, count=count, seed=40 + i, phase=j,
                              hits=torch.zeros(g.n, dtype=torch.int32, device="cuda")))
    stats, launch = c.sample_tasks(tasks)
    assert launch["samples"] == sum(t["count"] for t in tasks)
    for t, st in zip(tasks, stats):
        g, k = graphs[ids.index(t["graph"])]
        og, sto = oracle_objects(g, k)
        ho, so = O.sample_range(og, sto, t["first"], t["count"], t["seed"], t["phase"])
        assert np.array_equal(t["hits"].cpu().numpy().view(np.uint32), ho), (g.name, t["first"])
        same_stats(so, st)
    # graph estimate on an added graph meets eps against the exact values
    p, info = c.graph_estimate(ids[1], 0.05, 0.1, 9)
    og, sto = oracle_objects(*graphs[1])
    assert np.abs(p - O.exact(og, sto)).max() <= 0.05


def test_autotune_keeps_results():
    """The staged search times the automatic shape, 4 block sizes on device
    bitmaps, LDS tables and compact slots, two slot counts and two side
    rules; the knobs it keeps are the context's options and leave every
    result unchanged, on one graph and over all resident graphs (-1)."""
    import torch
    from paper_2509_11454_amd import percis as P
    g, k = W.workload_er1000()
    c = gpu_context(g, k)
    h0, s0 = gpu_hits(c, 0, 4000, 17)
    t = c.autotune(0, 5000)
    print("autotune:", t, flush=True)
    assert t["candidates"] >= 12 and t["block"] in (64, 128, 256, 512, 1024) and t["bitmaps"] in (1, 2)
    assert t["compact"] in (1, 2) and t["balance"] in (50, 100, 200)
    assert t["samples_per_s"] >= t["auto_samples_per_s"] > 0
    assert c.get_option(P.OPT_BLOCK) == t["block"] and c.get_option(P.OPT_BALANCE) == t["balance"]
    assert c.get_option(P.OPT_COMPACT) == t["compact"] and c.get_option(P.OPT_SLOTS) == t["slots"]
    h1, s1 = gpu_hits(c, 0, 4000, 17)
    assert np.array_equal(h0, h1)
    same_stats(s0, s1)
    g2, k2 = special_cases()[4]
    gid = c.add_graph(g2.n, g2.row_ptr, g2.col, k2)
    t2 = c.autotune(-1, 8000)
    assert t2["candidates"] >= 12
    h2, s2 = gpu_hits(c, 0, 4000, 17)
    assert np.array_equal(h0, h2)
    same_stats(s0, s2)
    og, st = oracle_objects(g2, k2)
    ho, so = oracle_hits(og, st, 0, 3000, 5)
    hits = torch.zeros(g2.n, dtype=torch.int32, device="cuda")
    (sg,), _ = c.sample_tasks([dict(graph=gid, first=0, count=3000, seed=5, phase=0, hits=hits)])
    assert np.array_equal(ho, hits.cpu().numpy().view(np.uint32))
    same_stats(so, sg)


@pytest.mark.parametrize("compact", [1, 2])
def test_side_rule_keeps_results(compact):
    """PERCIS_OPT_BALANCE only changes which ball grows: hits and sample
    statistics equal the oracle's under the rules 25, 100 and 400, on a
    skewed R-MAT graph and on a directed one, per-node and compact slots."""
    from paper_2509_11454_amd import percis as P
    rng = np.random.default_rng(31)
    cases = [W.rmat_graph(12, 8, seed=3), W.rmat_graph(11, 8, seed=4, directed=True)]
    for g in cases:
        k = W.skewed_states(g.n, rng, zero_frac=0.5)
        og, st = oracle_objects(g, k)
        ho, so = oracle_hits(og, st, 0, 6000, 23)
        c = gpu_context(g, k)
        c.set_option(P.OPT_COMPACT, compact)
        for bal in (25, 100, 400):
            c.set_option(P.OPT_BALANCE, bal)
            hg, sg = gpu_hits(c, 0, 6000, 23)
            assert np.array_equal(ho, hg), (g.name, bal)
            same_stats(so, sg)
        c.close()


@pytest.mark.parametrize("ci", [0, 4, 6, 8, 11, 13, 15])
def test_exact_centrality_on_device(ci):
    """percis_exact against the oracle's exact centrality (both sum in
    double in different orders: relative 1e-9, absolute 1e-12)."""
    g, k = special_cases()[ci]
    c = gpu_context(g, k)
    p, ms = c.exact(0)
    og, st = oracle_objects(g, k)
    pe = O.exact(og, st)
    assert np.allclose(p, pe, rtol=1e-9, atol=1e-12), (g.name, np.abs(p - pe).max())


def test_exact_er1000_and_estimate_within_eps():
    g, k = W.workload_er1000()
    c = gpu_context(g, k)
    p, ms = c.exact(0)
    og, st = oracle_objects(g, k)
    assert np.allclose(p, O.exact(og, st), rtol=1e-9, atol=1e-12)
    pe, info = c.estimate(0.01, 0.1, 5)
    assert np.abs(pe - p).max() <= 0.01
