"""Pins of RandomSP and of the exact centrality in the oracle: shortest-path
counts against enumeration and textbook counts, the canonical walk against
the sorted enumeration of all shortest paths, exact percolation centrality
against Definition 1 in rationals and the paper's closed forms."""
import json
import os
from math import comb

import numpy as np
import pytest

import brute as B
import oracle as O
import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def small_graphs():
    out = [W.path_graph(7), W.star_graph(6), W.cycle_graph(8), W.cycle_graph(7), W.complete_graph(5),
           W.grid_graph(3, 4), W.diamond_chain(3), W.complete_bipartite(3, 4)]
    for sd in range(6):
        out.append(W.random_small_graph(9 + sd % 3, 0.3, sd, directed=False))
        out.append(W.random_small_graph(8 + sd % 4, 0.25, 100 + sd, directed=True))
    return out


@pytest.mark.parametrize("gi", range(20))
def test_sigma_and_canonical_walk_vs_enumeration(gi):
    g = small_graphs()[gi]
    og = O.Graph(g.n, g.row_ptr, g.col, g.directed)
    dist = B.floyd_warshall(g)
    for s in range(g.n):
        for t in range(g.n):
            if s == t:
                continue
            paths = B.canonical_order(B.shortest_paths(g, s, t, dist))
            L, sigma, _ = O.path(og, s, t, 0)
            if not paths:
                assert L == -1
                continue
            assert L == dist[s][t]
            assert sigma == len(paths)
            for r in range(sigma):
                _, _, p = O.path(og, s, t, r)
                assert p == paths[r], (s, t, r)


def test_grid_sigma_closed_form_and_overflow():
    """Corner-to-corner counts C(a+b-2, a-1), exact below 2^128 - 1 (a path is
    given at both ends of r), saturated (overflow) beyond."""
    cases = [(a, b, int(want)) for a, b, want in GOLD["grid_sigma"]["cases"]]
    cases += [(66, 66, comb(130, 65)), (70, 70, comb(138, 69))]
    for a, b, want in cases:
        g = W.grid_graph(a, b)
        og = O.Graph(g.n, g.row_ptr, g.col)
        L, sigma, p = O.path(og, 0, a * b - 1, 0)
        assert L == a + b - 2
        assert want == comb(a + b - 2, a - 1)
        if want < O.SIGMA_SATURATED:
            assert sigma == want and p is not None
            # walking back from t, r = 0 keeps the smallest-id predecessor
            # (the node above), so the path runs along row 0 first; r = sigma - 1
            # keeps the largest (the node to the left): down column 0 first
            assert p[:b] == list(range(b))
            q = O.path(og, 0, a * b - 1, want - 1)[2]
            assert q[:a] == [i * b for i in range(a)]
        else:
            assert sigma == O.SIGMA_SATURATED and p is None


def diamond_path(k, r):
    """The canonical path of r in a chain of k diamonds: walking back from
    h_k, bit i of r picks the second middle node of diamond i."""
    out = [0]
    for i in range(k):
        out.append(k + 1 + 2 * i + ((r >> i) & 1))
        out.append(i + 1)
    return out


def test_diamond_chain_sigma():
    ks = list(GOLD["diamond_sigma"]["cases"]) + [100, 127, 128]
    rng = np.random.default_rng(9)
    for k in ks:
        g = W.diamond_chain(k)
        og = O.Graph(g.n, g.row_ptr, g.col)
        L, sigma, p = O.path(og, 0, k, 0)
        assert L == 2 * k
        if k < 128:
            assert sigma == 2 ** k
            rs = {0, 2 ** k - 1, 2 ** (k - 1)} | {int(rng.integers(0, 2 ** 62)) << max(0, k - 62) for _ in range(5)}
            for r in rs:
                r %= 2 ** k
                assert O.path(og, 0, k, r)[2] == diamond_path(k, r), (k, r)
        else:
            assert sigma == O.SIGMA_SATURATED and p is None


def test_simple_sigmas():
    g = W.cycle_graph(10)
    og = O.Graph(g.n, g.row_ptr, g.col)
    assert O.path(og, 0, 5, 0)[:2] == (5, 2)
    g = W.complete_bipartite(3, 5)
    og = O.Graph(g.n, g.row_ptr, g.col)
    assert O.path(og, 0, 1, 0)[:2] == (2, 5)
    assert O.path(og, 3, 4, 0)[:2] == (2, 3)


def test_unreachable_directed():
    g = W.from_edge_list(4, [(0, 1), (1, 2)], directed=True)
    og = O.Graph(g.n, g.row_ptr, g.col, True)
    assert O.path(og, 2, 0, 0)[0] == -1
    assert O.path(og, 0, 3, 0)[0] == -1
    assert O.path(og, 0, 2, 0)[:3] == (2, 1, [0, 1, 2])


def state_sets(n, seed):
    rng = np.random.default_rng(seed)
    return [W.uniform_states(n, rng), rng.integers(0, 3, size=n).astype(np.uint16) * 30000,
            W.rs_states(n, rng, seeds=2)]


@pytest.mark.parametrize("gi", range(20))
def test_exact_vs_definition(gi):
    g = small_graphs()[gi]
    if g.n > 11:
        pytest.skip("enumeration too slow")
    og = O.Graph(g.n, g.row_ptr, g.col, g.directed)
    for k in state_sets(g.n, gi):
        st = O.States(k)
        if st.C == 0:
            continue
        want = B.exact_percolation(g, k)
        got = O.exact(og, st)
        for v in range(g.n):
            assert abs(got[v] - float(want[v])) < 1e-12, (v, got[v], want[v])


def test_star_path_complete_closed_forms():
    rng = np.random.default_rng(3)
    # star: the centre is internal to every pair of leaves, so p(centre) = 1
    g = W.star_graph(7)
    k = W.uniform_states(7, rng)
    p = O.exact(O.Graph(g.n, g.row_ptr, g.col), O.States(k))
    assert abs(p[0] - 1.0) < 1e-12 and np.all(np.abs(p[1:]) < 1e-15)
    # complete graph: no internal nodes
    g = W.complete_graph(6)
    p = O.exact(O.Graph(g.n, g.row_ptr, g.col), O.States(W.uniform_states(6, rng)))
    assert np.all(p == 0.0)
    # path: p(v) = sum over s, t on opposite sides of v of R(x_s - x_t) / S_v
    n = 8
    g = W.path_graph(n)
    k = W.uniform_states(n, rng)
    st = O.States(k)
    p = O.exact(O.Graph(g.n, g.row_ptr, g.col), st)
    S = st.arrays()["S"]
    for v in range(n):
        num = sum(max(0, int(k[s]) - int(k[t])) for s in range(n) for t in range(n)
                  if (s < v < t) or (t < v < s))
        assert abs(p[v] - (num / S[v] if S[v] else 0.0)) < 1e-12


def test_prop7_instance():
    gold = GOLD["prop7_p_b"]
    K = 65535
    for n in gold["n_values"]:
        g, k = W.prop7_instance(n)
        og = O.Graph(g.n, g.row_ptr, g.col, True)
        p = O.exact(og, O.States(k))
        kc = int(k[2])
        want = (K - kc) / ((K - kc) + (n - 3) * (K + kc))
        assert abs(p[1] - want) < 1e-15
        assert np.all(np.abs(np.delete(p, 1)) < 1e-15)
        # the definition, not the printed (1/2)/(n-3+1/2), e.g. 1/4 not 1/3 at n = 4
        if n == 4:
            assert abs(p[1] - 0.25) < 1e-4


def test_vertex_diam_ub():
    # (directed graphs: test_oracle_bounds.test_vertex_diam_ub_directed)
    for g in small_graphs():
        if g.directed:
            continue
        og = O.Graph(g.n, g.row_ptr, g.col)
        D = O.vertex_diam_ub(og)
        dist = B.floyd_warshall(g)
        true = max([d - 1 for row in dist for d in row if d != B.INF and d >= 1] + [0])
        assert D >= true
    og = O.Graph(9, W.path_graph(9).row_ptr, W.path_graph(9).col)
    assert O.vertex_diam_ub(og) == 7
    og = O.Graph(2, W.path_graph(2).row_ptr, W.path_graph(2).col)
    assert O.vertex_diam_ub(og) == 0
