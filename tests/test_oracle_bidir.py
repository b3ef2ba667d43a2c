"""The oracle's bidirectional search mode against its truncated BFS.

RandomSP (Section III-B) may find the shortest paths with a truncated BFS
from s or with a balanced bidirectional BFS; the canonical path of (s, t, r)
depends on neither. The oracle's bidirectional mode is its speed path for
the largest graphs, so it must return exactly what the truncated BFS returns:
the same d(s,t), sigma_st and path for every (s, t, r) of small graphs, and
the same hits and statistics, sample by sample, on windows of larger ones.
The truncated BFS itself is pinned to brute-force enumeration elsewhere."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def small_graphs():
    out = [W.path_graph(7), W.star_graph(6), W.cycle_graph(8), W.cycle_graph(7), W.complete_graph(5),
           W.grid_graph(3, 4), W.diamond_chain(3), W.complete_bipartite(3, 4),
           W.layered_graph([1, 3, 2, 4, 1]), W.layered_graph([2, 3, 3, 2], directed=True)]
    for sd in range(6):
        out.append(W.random_small_graph(9 + sd % 3, 0.3, sd, directed=False))
        out.append(W.random_small_graph(8 + sd % 4, 0.25, 100 + sd, directed=True))
    out.append(W.prop7_instance(7)[0])
    return out


def oracle_graph(g):
    return O.Graph(g.n, g.row_ptr, g.col, g.directed)


def test_every_path_of_small_graphs():
    """Every (s, t, r), s != t, r < sigma_st, on 21 small graphs; also s == t."""
    checked = 0
    for g in small_graphs():
        og = oracle_graph(g)
        for s in range(g.n):
            assert O.path(og, s, s, 0, bidir=True) == O.path(og, s, s, 0)
            for t in range(g.n):
                if s == t:
                    continue
                L, sig, _ = O.path(og, s, t, 0)
                assert O.path(og, s, t, 0, bidir=True)[:2] == (L, sig), (g.name, s, t)
                if L < 0:
                    continue
                for r in range(sig):
                    assert O.path(og, s, t, r, bidir=True) == O.path(og, s, t, r), (g.name, s, t, r)
                    checked += 1
    assert checked > 2000


def test_sigma_extremes():
    """Grid corners with sigma just below and above 2^64, diamond chains up
    to the 128-bit saturation, with r at both ends and inside."""
    cases = [(W.grid_graph(34, 35), 0, 34 * 35 - 1), (W.grid_graph(35, 35), 0, 35 * 35 - 1)]
    for k in (63, 64, 127, 128):
        cases.append((W.diamond_chain(k), 0, k))
    for g, s, t in cases:
        og = oracle_graph(g)
        L, sig, _ = O.path(og, s, t, 0)
        assert O.path(og, s, t, 0, bidir=True)[:2] == (L, sig)
        if sig == O.SIGMA_SATURATED:
            continue
        for r in (0, 1, sig // 3, sig - 2, sig - 1):
            assert O.path(og, s, t, r, bidir=True) == O.path(og, s, t, r), (g.name, r)
    assert O.path(oracle_graph(W.grid_graph(35, 35)), 0, 35 * 35 - 1)[1] == math.comb(68, 34)


def same_range(og, st, first, count, seed, phase=0, work=None):
    h0, s0, i0 = O.sample_range(og, st, first, count, seed, phase, with_I=True)
    h1, s1, i1 = O.sample_range(og, st, first, count, seed, phase, with_I=True, bidir=True, work=work)
    assert np.array_equal(h0, h1)
    assert s0 == s1
    assert np.array_equal(i0, i1)
    return s0


def test_sample_windows_er_and_special_graphs():
    g, k = W.workload_er1000()
    s = same_range(oracle_graph(g), O.States(k), 0, 3000, 1)
    assert s["reachable"] > 1000
    rng = np.random.default_rng(3)
    for g in (W.ba_graph(3000, 4, 5), W.layered_graph([1, 40, 70, 40, 1]), W.grid_graph(20, 30)):
        same_range(oracle_graph(g), O.States(W.uniform_states(g.n, rng)), 0, 2000, 7)
    gi, ki = W.with_isolated_component(W.er_graph(500, 2000, 4), directed=False)
    same_range(oracle_graph(gi), O.States(ki), 0, 2000, 2)
    gd, kd = W.with_isolated_component(W.random_small_graph(60, 0.06, 9, directed=True))
    same_range(oracle_graph(gd), O.States(kd), 0, 2000, 2)
    # pairs of 2^64 and more shortest paths: the 128-bit draws and the
    # saturated samples land in the same places (diamond chains of 80 and 130
    # diamonds; pairs of hubs 128 or more apart saturate at 2^128 - 1)
    for kd_ in (80, 130):
        gc = W.diamond_chain(kd_)
        kc = np.zeros(gc.n, np.uint16)
        kc[0] = 65535
        kc[kd_] = 1000
        s = same_range(oracle_graph(gc), O.States(kc), 0, 400, 3)
        if kd_ == 130:
            assert s["overflow"] > 0


@pytest.mark.parametrize("directed", [False, True])
def test_sample_windows_rmat16(directed):
    """R-MAT scale 16 (the benchmark generators at a smaller scale): skewed
    states undirected, Beta(1/2, 1/2) directed, as in the benchmarks."""
    g = W.rmat_graph(16, 16, seed=3, directed=directed)
    rng = np.random.default_rng(3)
    k = W.beta_states(g.n, rng) if directed else W.skewed_states(g.n, rng)
    og, st = oracle_graph(g), O.States(k)
    s = same_range(og, st, 0, 1200, 1)
    assert s["reachable"] > 200
    same_range(og, st, 10 ** 6, 600, 2, phase=1)


def test_workspace_reused_across_graphs():
    """One workspace serves graphs of different sizes one after another."""
    work = O.BidirWork(5000)
    g1, k1 = W.workload_er1000()
    g2 = W.ba_graph(4000, 4, 1)
    k2 = W.uniform_states(g2.n, np.random.default_rng(1))
    for g, k in ((g1, k1), (g2, k2), (g1, k1)):
        same_range(oracle_graph(g), O.States(k), 500, 1500, 4, work=work)
