"""Pins of the oracle's pair sampler (Algorithm 2): the preprocessing arrays
against the closed forms of the proof of Proposition 1, the two binary
searches by exhaustive enumeration of the integer draws, and the pair
distribution kappa~(s,t) of Section III-A."""
import json
import os
from collections import Counter

import numpy as np
import pytest

import oracle as O
import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def ranks_by_hand(k):
    return sorted(range(len(k)), key=lambda v: (-int(k[v]), v))


@pytest.mark.parametrize("seed", range(6))
def test_alg2_arrays_closed_forms(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 40))
    k = rng.integers(0, 6, size=n).astype(np.uint16) * (1 if seed % 2 else 9000)
    if seed == 5:
        k = W.uniform_states(n, rng)
    st = O.States(k)
    a = st.arrays()
    order = ranks_by_hand(k)
    assert [int(v) for v in a["perm"][1:n + 1]] == order
    x = [int(k[v]) for v in order]
    for i in range(1, n + 1):
        xi = x[i - 1]
        assert int(a["x"][i]) == xi
        assert int(a["w"][i]) == sum(x[i - 1:])
        assert int(a["c"][i]) == sum(max(0, xi - xj) for xj in x[i - 1:])
        assert int(a["r"][i]) == sum(int(a["c"][j]) for j in range(i, n + 1))
    tot = sum(max(0, int(k[u]) - int(k[w])) for u in range(n) for w in range(n) if u != w)
    assert st.C == tot
    for v in range(n):
        S_v = sum(max(0, int(k[u]) - int(k[w])) for u in range(n) for w in range(n) if u != v and w != v)
        assert a["S"][v] == S_v


@pytest.mark.parametrize("seed", range(5))
def test_searches_exhaustive(seed):
    """Every integer U in [0, C) maps to rank s exactly c_s times, and for
    each s every U in [0, c_s) maps to t exactly R(k_s - k_t) times: the pair
    probabilities are exactly kappa~(s,t) = R(x_s - x_t) / sum R."""
    rng = np.random.default_rng(50 + seed)
    n = int(rng.integers(2, 9))
    k = rng.integers(0, 5, size=n).astype(np.uint16)
    if len(set(k.tolist())) == 1:
        k[0] = k[0] + 1
    st = O.States(k)
    a = st.arrays()
    order = ranks_by_hand(k)
    cs = Counter(O.search_s(st, U) for U in range(st.C))
    for i in range(1, n + 1):
        assert cs.get(i, 0) == int(a["c"][i])
    for s in range(1, n + 1):
        cst = int(a["c"][s])
        if cst == 0:
            continue
        ct = Counter(O.search_t(st, s, U) for U in range(cst))
        for t in range(1, n + 1):
            want = max(0, int(k[order[s - 1]]) - int(k[order[t - 1]])) if t > s else 0
            assert ct.get(t, 0) == want


def test_search_boundaries_large():
    """U = P_{i-1} and U = P_i - 1 select rank i, for every rank with c_i > 0
    (P_i = C - r_{i+1}); same for t inside the row of a few s."""
    rng = np.random.default_rng(7)
    k = W.uniform_states(3000, rng)
    st = O.States(k)
    a = st.arrays()
    n = st.n
    P = [st.C - int(a["r"][i + 1]) for i in range(n + 1)]
    for i in range(1, n + 1):
        if P[i] > P[i - 1]:
            assert O.search_s(st, P[i - 1]) == i
            assert O.search_s(st, P[i] - 1) == i
    x, w = a["x"], a["w"]
    for s in [1, 2, 17, 1500, n - 1]:
        def F(d):
            return (d - s + 1) * int(x[s]) - (int(w[s]) - int(w[d + 1]))
        for t in range(s + 1, n + 1):
            if F(t) > F(t - 1):
                assert O.search_t(st, s, F(t - 1)) == t
                assert O.search_t(st, s, F(t) - 1) == t


def test_pair_distribution_chi2():
    """Sampled pairs follow kappa~ (chi-square over 60000 draws)."""
    k = np.array([65535, 40000, 40000, 1000, 0, 0], np.uint16)
    st = O.States(k)
    n = len(k)
    tot = sum(max(0, int(k[u]) - int(k[w])) for u in range(n) for w in range(n) if u != w)
    draws = 60000
    cnt = Counter()
    for idx in range(draws):
        s, t, _, _ = O.draw_pair(st, 3, 0, idx)
        cnt[(s, t)] += 1
    chi2 = 0.0
    dof = 0
    for s in range(n):
        for t in range(n):
            p = max(0, int(k[s]) - int(k[t])) / tot
            if p == 0:
                assert cnt.get((s, t), 0) == 0
                continue
            e = p * draws
            chi2 += (cnt.get((s, t), 0) - e) ** 2 / e
            dof += 1
    # 99.9% quantile of chi-square with 13 dof is about 34.5
    assert chi2 < 34.5 + 2 * max(0, dof - 13), (chi2, dof)


def test_prop6_S_b_closed_form():
    g = GOLD["prop6_S_b"]
    K = 65535
    for n in g["n_values"]:
        kc = int(W.quantise([0.5])[0])
        k = np.zeros(n, np.uint16)
        k[0], k[1], k[2] = K, 0, kc
        S = O.States(k).arrays()["S"]
        assert S[1] == (K - kc) + (n - 3) * (K + kc)
        # the printed real-valued form, 3/2 (n-3) + 1/2, up to the quantisation of 1/2
        assert abs(S[1] / K - (1.5 * (n - 3) + 0.5)) <= (n - 2) / K


def test_states_tied_and_degenerate():
    st = O.States(np.full(10, 1234, np.uint16))
    assert st.C == 0
    st = O.States(np.array([5], np.uint16))
    assert st.C == 0
