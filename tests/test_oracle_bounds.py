"""Pins of the data-dependent bounds of Algorithm 1 in the oracle.

- rho_hat (Proposition 2) is an empirical Bernstein upper bound on
  rho = E|I(tau)| at confidence delta/4: its deviation term is the Gaussian
  tail quantile at delta/8 to leading order, so on a sample whose |I| is a
  fair coin its miss rate over many seeds is Phi(-sqrt(2 ln(8/delta))).
- v_hat (Proposition 3) is d_hat^2 times an upper confidence bound on p(v)
  at delta/4 taken from the weighted phase-1 estimate: on a node whose
  per-sample term has variance d_v p(v) - p(v)^2 = p(v) (d_v = 2, q_v = 1/2)
  its miss rate is Phi(-sqrt(2 ln(4/delta))).
- Both hold at the paper's settings against exact rho and exact per-node
  variances, on states whose likelihood ratio d_hat is far above 1.
- v_hat follows from the integer phase-1 hits and the weights d_v.
- VertexDiamUB bounds the internal nodes of every shortest path of a
  directed graph (all-pairs distances by Floyd-Warshall).
The simulations use the oracle's own Algorithm 1 end to end (stream phase 1
for the bounds); a plausible slip in either bound (a logarithm's constant, a
dropped factor 2 or d_hat^2, a misplaced square root) moves a miss rate far
outside the band."""
import math
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
from scipy import stats

import brute as B
import oracle as O
import workloads as W

THREADS = 8


def three_path():
    """Path 0 - 1 - 2 with k = (65535, 32767, 0): the pairs (0,1), (0,2),
    (1,2) weigh 32768, 65535, 32767, so |I| = 1 (the pair (0,2), through
    node 1) with probability exactly 1/2, else 0. S_1 = 65535 and C = 131070
    give d_1 = 2 and p(1) = 1; node 1 is the only node ever internal."""
    g = W.path_graph(3)
    k = np.array([65535, 32767, 0], np.uint16)
    return g, k


def estimates(og, st, eps, delta, seeds, D=-1):
    def one(seed):
        rc, _, info = O.estimate(og, st, eps, delta, seed, D=D)
        assert rc == 0
        return info
    with ThreadPoolExecutor(THREADS) as ex:
        return list(ex.map(one, seeds))


def band(M, p, lattice):
    """Counts of misses compatible with rate p over M runs: 4 binomial
    standard deviations plus the probability of one lattice step of the
    phase-1 count (the Gaussian rate ignores that the count is an integer)."""
    return 4 * math.sqrt(M * p * (1 - p)) + M * lattice


def test_three_path_exact_values():
    g, k = three_path()
    assert B.rho(g, k) == B.pair_weights(k)[0][(0, 2)] / B.pair_weights(k)[1] == 0.5
    assert [float(x) for x in B.exact_percolation(g, k)] == [0.0, 1.0, 0.0]
    assert float(B.likelihood_ratios(k)[1]) == 2.0
    assert float(B.hit_expectation(g, k)[1]) == 0.5


def test_deviation_terms_by_simulation():
    """6000 runs of Algorithm 1 on the three-node path at delta = 0.99 (the
    largest miss rates, so the sharpest test), D forced to 0 so that rho_hat
    is rho_tilde plus its deviation term alone. Misses: rho_hat < rho = 1/2,
    and v_hat < d_hat^2 p(1) (the confidence bound of p(1) = E p~(1)
    missed). Expected rates Phi(-sqrt(2 ln(8/delta))) = 2.05% and
    Phi(-sqrt(2 ln(4/delta))) = 4.73%; the phase-1 count moves in steps of
    phi(z)/sqrt(l1/4) probability. With ln(4/delta) and ln(8/delta) swapped
    the rates would be 4.7% and 2.3%; without the 2 under the roots, 7.7%
    and 12%."""
    g, k = three_path()
    og, st = O.Graph(g.n, g.row_ptr, g.col), O.States(k)
    M, delta = 6000, 0.99
    infos = estimates(og, st, 0.5, delta, range(1, M + 1), D=0)
    assert all(i["l1"] == 1000 and i["D"] == 0 for i in infos)
    sd_count = math.sqrt(1000 * 0.25)
    for name, miss, c in (("rho_hat", lambda i: i["rho_hat"] < 0.5, 8.0),
                          ("v_hat", lambda i: i["v_hat"] < i["d_hat"] ** 2 * 1.0, 4.0)):
        z = math.sqrt(2 * math.log(c / delta))
        p = stats.norm.cdf(-z)
        lattice = stats.norm.pdf(z) / sd_count
        got = sum(1 for i in infos if miss(i))
        assert abs(got - M * p) <= band(M, p, lattice), (name, got, M * p)


def test_rho_hat_range_term_when_I_is_constant():
    """A star whose centre holds the top state and whose leaves share one
    lower state: every positive-weight pair has the centre as an end, so
    |I| = 0 on every sample, Lambda = 0 and
    rho_tilde = 0 exactly, and rho_hat is the range term of the empirical
    Bernstein bound (Maurer and Pontil's Theorem 4 for values in [0, D],
    l1 samples, confidence delta/4): 7 D ln(2/(delta/4)) / (3 (l1 - 1))."""
    g = W.star_graph(9)
    k = np.zeros(9, np.uint16)
    k[0] = 65535
    k[1:] = 7000
    og, st = O.Graph(g.n, g.row_ptr, g.col), O.States(k)
    for D, delta in ((0, 0.1), (1, 0.1), (5, 0.3), (40, 0.02)):
        rc, _, I = O.estimate(og, st, 0.2, delta, 3, D=D)
        assert rc == 0 and I["rho_tilde"] == 0.0 and I["Lambda"] == 0.0
        conf = delta / 4
        assert I["rho_hat"] == pytest.approx(7 * D * math.log(2 / conf) / (3 * (I["l1"] - 1)), rel=1e-13, abs=0)


def coverage_graph():
    """8 nodes, directed; two nodes at the top state and one at 20000 out of
    65535: d_hat = 4.66 and the largest per-node variance is 4.4 times the
    largest p(v)."""
    g = W.random_small_graph(8, 0.35, 305, directed=True)
    rng = np.random.default_rng(5)
    k = np.zeros(g.n, np.uint16)
    k[rng.choice(g.n, 2, replace=False)] = 65535
    k[rng.integers(g.n)] = 20000
    return g, k


def test_bounds_cover_exact_values():
    """Propositions 2 and 3 at delta = 0.1 over 300 seeds: rho <= rho_hat
    (and so sum p <= d_hat rho_hat, Lemma 3) and max_v Var <= v_hat, where
    the per-sample term d_v 1[v in I(tau)] has variance d_v^2 q_v (1 - q_v)
    with q_v the exact probability that v is internal. Each may fail with
    probability delta/4; the counts must stay below what Binomial(300,
    0.025) exceeds with probability 1e-4. The variance bound is far from
    the d_v-free one: max_v Var is 4.4 times max_v p(v)."""
    g, k = coverage_graph()
    d = [float(x) for x in B.likelihood_ratios(k)]
    q = [float(x) for x in B.hit_expectation(g, k)]
    p = [float(x) for x in B.exact_percolation(g, k)]
    rho = float(B.rho(g, k))
    var = max(d[v] ** 2 * q[v] * (1 - q[v]) for v in range(g.n))
    assert max(d) > 4.5 and var > 4 * max(p)
    og, st = O.Graph(g.n, g.row_ptr, g.col, g.directed), O.States(k)
    infos = estimates(og, st, 0.05, 0.1, range(100, 400))
    limit = stats.binom.isf(1e-4, 300, 0.025)
    assert all(abs(i["d_hat"] - max(d)) < 1e-12 for i in infos)
    assert sum(i["rho_hat"] < rho for i in infos) <= limit
    assert sum(i["d_hat"] * i["rho_hat"] < sum(p) for i in infos) <= limit
    assert sum(i["v_hat"] < var for i in infos) <= limit


def test_v_hat_from_phase1_hits():
    """v_hat recomputed from the integer phase-1 hits of the plain sampler
    (stream phase 1, l1 samples) and the weights d_v = C / S_v, with the
    upper confidence bound at delta/4 of Proposition 3."""
    g, k = coverage_graph()
    og, st = O.Graph(g.n, g.row_ptr, g.col, g.directed), O.States(k)
    d = np.array([float(x) for x in B.likelihood_ratios(k)])
    for eps, delta, seed in ((0.05, 0.1, 7), (0.002, 0.3, 8)):
        rc, _, I = O.estimate(og, st, eps, delta, seed)
        assert rc == 0
        l1 = I["l1"]
        assert l1 == math.ceil(max(1000, math.log(1 / delta) / eps))
        h1, _ = O.sample_range(og, st, 0, l1, seed, 1)
        pt = d * h1 / l1
        conf = delta / 4
        ucb = pt + np.sqrt(2 * pt * math.log(1 / conf) / l1) + math.log(1 / conf) / (3 * l1)
        assert I["v_hat"] == pytest.approx(I["d_hat"] ** 2 * ucb.max(), rel=1e-12)


def directed_graphs():
    out = [W.random_small_graph(8 + sd % 4, 0.25, 100 + sd, directed=True) for sd in range(6)]
    out += [W.random_small_graph(10, 0.12, 500 + sd, directed=True) for sd in range(6)]
    out += [W.prop7_instance(9)[0], W.layered_graph([2, 3, 1, 2], directed=True)]
    # a path whose arcs point towards node 0: a search along out-arcs from
    # the smallest node sees one node
    out.append(W.from_edge_list(7, [(i + 1, i) for i in range(6)], directed=True))
    return out


def test_vertex_diam_ub_directed():
    """VertexDiamUB on directed graphs is at least max |I| = max d(s,t) - 1
    over reachable pairs (Floyd-Warshall), and equal to it on a directed path
    whose arcs point towards the smallest id."""
    for g in directed_graphs():
        dist = B.floyd_warshall(g)
        worst = max((dist[s][t] - 1 for s in range(g.n) for t in range(g.n)
                     if s != t and dist[s][t] != B.INF), default=0)
        D = O.vertex_diam_ub(O.Graph(g.n, g.row_ptr, g.col, True))
        assert D >= worst, (g.name, D, worst)
    rev = directed_graphs()[-1]
    assert O.vertex_diam_ub(O.Graph(rev.n, rev.row_ptr, rev.col, True)) == 5
    # two weakly connected components of 5 and 9 nodes: the larger bounds D
    e = [(1, 0), (2, 1), (2, 3), (4, 3)] + [(5 + i, 6 + i) for i in range(8)]
    g2 = W.from_edge_list(14, e, directed=True)
    assert O.vertex_diam_ub(O.Graph(g2.n, g2.row_ptr, g2.col, True)) == 7
