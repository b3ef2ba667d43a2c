"""Pins of the oracle's estimator and of Algorithm 1: the per-node weight
reduction (proof of Proposition 5), Lemma 1 exactly and statistically,
Lemma 3, Proposition 2's Lambda against the sample variance, the sample-size
supremum against an independent optimiser, and the (eps, delta) guarantee
of Proposition 4 over many seeds."""
import math

import numpy as np
import pytest
from scipy import optimize

import brute as B
import oracle as O
import workloads as W


def test_d_v_closed_form():
    """d_v = max kappa/kappa~ = C / S_v = 1 + sum_u |x_v - x_u| / S_v."""
    rng = np.random.default_rng(1)
    for n in [4, 6, 9]:
        k = W.uniform_states(n, rng)
        st = O.States(k)
        S = st.arrays()["S"]
        d = B.likelihood_ratios(k)
        for v in range(n):
            A = sum(abs(int(k[v]) - int(k[u])) for u in range(n))
            assert abs(float(d[v]) - st.C / S[v]) < 1e-12
            assert abs(1 + A / S[v] - st.C / S[v]) < 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_lemma1_exact(seed):
    """d_v * sum_{s,t} kappa~(s,t) sigma_st(v)/sigma_st = p(v) in rationals."""
    g = W.random_small_graph(8, 0.35, 200 + seed, directed=bool(seed % 2))
    rng = np.random.default_rng(seed)
    k = W.uniform_states(g.n, rng)
    e = B.hit_expectation(g, k)
    d = B.likelihood_ratios(k)
    p = B.exact_percolation(g, k)
    for v in range(g.n):
        assert d[v] * e[v] == p[v]


def test_unbiased_hits_statistically():
    """E[hits_v] / l = sum kappa~ sigma_st(v)/sigma_st: binomial 5-sigma band."""
    g = W.random_small_graph(10, 0.3, 7)
    k = W.uniform_states(g.n, np.random.default_rng(7))
    og, st = O.Graph(g.n, g.row_ptr, g.col), O.States(k)
    ell = 200000
    hits, stats = O.sample_range(og, st, 0, ell, 42)
    assert stats["samples"] == ell
    e = B.hit_expectation(g, k)
    for v in range(g.n):
        q = float(e[v])
        sd = math.sqrt(max(q * (1 - q), 1e-12) / ell)
        assert abs(hits[v] / ell - q) < 5 * sd + 1e-9, (v, hits[v] / ell, q)
    r = float(B.rho(g, k))
    assert abs(stats["sum_I"] / ell - r) < 0.02 * max(r, 1)


def test_ranges_are_additive():
    g, k = W.workload_er1000()
    og, st = O.Graph(g.n, g.row_ptr, g.col), O.States(k)
    h0, s0 = O.sample_range(og, st, 0, 300, 5, 0)
    h1, s1 = O.sample_range(og, st, 300, 200, 5, 0)
    h, s = O.sample_range(og, st, 0, 500, 5, 0)
    assert np.array_equal(h0 + h1, h)
    assert s0["sum_I"] + s1["sum_I"] == s["sum_I"]


def test_lemma3_and_literal_estimator():
    g, k = W.workload_er1000()
    og, st = O.Graph(g.n, g.row_ptr, g.col), O.States(k)
    p = O.exact(og, st)
    S = st.arrays()["S"]
    d = st.C / S
    dhat = d.max()
    # rho from many samples (its estimate) brackets sum p within Lemma 3
    hits, stats = O.sample_range(og, st, 0, 20000, 9, 0)
    rho = stats["sum_I"] / stats["samples"]
    assert rho * 0.97 <= p.sum() <= dhat * rho * 1.03
    # the literal estimator of Algorithm 1 equals d_v h_v / l
    rc, pe, info = O.estimate(og, st, 0.05, 0.1, 3)
    assert rc == 0
    h2, _ = O.sample_range(og, st, 0, info["l"], 3, 2)
    assert np.allclose(pe, d * h2 / info["l"], rtol=1e-12, atol=1e-15)


def test_lambda_is_sample_variance():
    g, k = W.workload_er1000()
    og, st = O.Graph(g.n, g.row_ptr, g.col), O.States(k)
    rc, _, info = O.estimate(og, st, 0.05, 0.1, 11)
    _, _, I = O.sample_range(og, st, 0, info["l1"], 11, 1, with_I=True)
    assert abs(info["Lambda"] - np.var(I.astype(np.float64), ddof=1)) < 1e-9
    assert abs(info["rho_tilde"] - I.mean()) < 1e-12
    l1 = info["l1"]
    L8 = math.log(8 / 0.1)
    want = I.mean() + math.sqrt(2 * info["Lambda"] * L8 / l1) + 7 * info["D"] * L8 / (3 * (l1 - 1))
    assert abs(info["rho_hat"] - want) < 1e-9
    assert info["l1"] == 1000


def f_bound(x, d, rho, eps, delta):
    gx = x * (d - x)
    y = eps * d / gx
    h = (1 + y) * math.log1p(y) - y
    return d * d * math.log(4 * d * rho / (x * delta)) / (gx * h)


@pytest.mark.parametrize("d,rho,v,eps,delta", [
    (1.003, 2.4, 0.028, 0.01, 0.1), (1.05, 9.7, 0.3, 0.005, 0.05), (1.5, 3.0, 0.9, 0.05, 0.1),
    (1.0, 5.0, 0.001, 0.001, 0.1), (2.0, 40.0, 5.0, 0.01, 0.01)])
def test_sample_size_supremum(d, rho, v, eps, delta):
    got, x_hat = O.sample_size(d, rho, v, eps, delta)
    assert abs(x_hat - (d / 2 - math.sqrt(d * d / 4 - min(d * d / 4, v)))) < 1e-15
    # independent optimiser over log x in [log(x_hat) - 35, log(x_hat)]
    lo, hi = math.log(x_hat) - 35, math.log(x_hat)
    res = optimize.minimize_scalar(lambda y: -f_bound(math.exp(y), d, rho, eps, delta),
                                   bounds=(lo, hi), method="bounded", options={"xatol": 1e-10})
    best = max(-res.fun, f_bound(x_hat, d, rho, eps, delta))
    # the grid has 13333 points per decade: its max is within 1e-6 of the sup
    assert got >= best * (1 - 1e-6)
    assert got <= best * (1 + 1e-6)
    # near x -> 0 the bound tends to d/eps (from above)
    assert f_bound(x_hat * 1e-12, d, rho, eps, delta) > d / eps
    # the approximate form quoted after Theorem 1, with the constants of Alg. 1
    approx = (2 * v + 2 / 3 * eps * d) / eps ** 2 * (math.log(d * rho / v) + math.log(4 / delta))
    if v < d * d / 8:
        assert 0.5 < got / approx < 2.0


def test_sample_size_monotone():
    base = O.sample_size(1.01, 3.0, 0.05, 0.01, 0.1)[0]
    assert O.sample_size(1.01, 3.0, 0.05, 0.005, 0.1)[0] > base
    assert O.sample_size(1.01, 3.0, 0.05, 0.01, 0.05)[0] > base
    assert O.sample_size(1.01, 6.0, 0.05, 0.01, 0.1)[0] > base
    assert O.sample_size(1.01, 3.0, 0.10, 0.01, 0.1)[0] > base


@pytest.mark.slow
def test_eps_delta_guarantee_over_seeds():
    """Proposition 4: max_v |p~ - p| <= eps fails with probability <= delta.
    100 seeds; with delta = 0.2 the count of failures must stay below what a
    Binomial(100, 0.2) exceeds with probability 1e-4 (35)."""
    rng = np.random.default_rng(4)
    g = W.er_graph(300, 900, 4)
    k = W.uniform_states(g.n, rng)
    og, st = O.Graph(g.n, g.row_ptr, g.col), O.States(k)
    p = O.exact(og, st)
    eps, delta = 0.05, 0.2
    fails = 0
    for seed in range(100):
        rc, pe, info = O.estimate(og, st, eps, delta, 1000 + seed)
        assert rc == 0
        fails += np.abs(pe - p).max() > eps
    assert fails <= 35
    # the bound is conservative: failures are expected to be rare
    assert fails <= 10


def test_eps_guarantee_ic_setting():
    """IC-style states (an isolated path, half at state 1): PercIS still
    meets eps on a graph where uniform sampling would need many samples."""
    g0 = W.er_graph(150, 450, 8)
    g, k = W.with_isolated_component(g0, length=20)
    og, st = O.Graph(g.n, g.row_ptr, g.col), O.States(k)
    p = O.exact(og, st)
    rc, pe, info = O.estimate(og, st, 0.05, 0.1, 77)
    assert rc == 0
    assert np.abs(pe - p).max() <= 0.05


def test_percis_di_bound_and_sampling():
    """PercIS-DI (Section IV, sample size bound experiment): no first phase,
    rho_hat = D and v_hat = d_hat^2/4, so x_hat = d_hat/2; its phase-2 hits
    are the plain sampler's; its bound is at least PercIS's data-dependent
    one (the paper finds it larger in every setting) and grows like
    1/eps^2 (it is O(ln(D/delta)/eps^2))."""
    rng = np.random.default_rng(12)
    g = W.er_graph(120, 360, 12)
    k = W.uniform_states(g.n, rng)
    og, st = O.Graph(g.n, g.row_ptr, g.col), O.States(k)
    rc, p_di, I = O.estimate_di(og, st, 0.1, 0.1, 31)
    assert rc == 0 and I["l1"] == 0
    D = O.vertex_diam_ub(og)
    assert I["D"] == D and I["rho_hat"] == D
    assert abs(I["v_hat"] - I["d_hat"] ** 2 / 4) < 1e-15
    assert abs(I["x_hat"] - I["d_hat"] / 2) < 1e-15
    want_l = math.ceil(O.sample_size(I["d_hat"], D, I["d_hat"] ** 2 / 4, 0.1, 0.1)[0])
    assert I["l"] == want_l
    # the estimate is phase 2 of the plain sampler, scaled by d_v / l
    hits, _ = O.sample_range(og, st, 0, I["l"], 31, 2)
    dv = np.array([float(x) for x in B.likelihood_ratios(k)])
    assert np.allclose(p_di, dv * hits / I["l"], rtol=1e-15, atol=0)
    # data-dependent bound no larger; 1/eps^2 growth
    rc2, _, I2 = O.estimate(og, st, 0.1, 0.1, 31)
    assert rc2 == 0 and I2["l"] <= I["l"]
    l_half = O.sample_size(I["d_hat"], D, I["d_hat"] ** 2 / 4, 0.05, 0.1)[0]
    assert 3.0 < l_half / want_l < 4.6
