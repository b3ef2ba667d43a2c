"""Brute-force references for tiny graphs, in exact rationals.

Independent of both the oracle and the HIP library: distances come from
Floyd-Warshall, shortest paths from enumerating simple paths, centralities
from Definition 1 (Eq. 1) summed term by term with ``fractions.Fraction``.
"""
from fractions import Fraction
from itertools import product

INF = float("inf")


def adjacency(g):
    adj = [set() for _ in range(g.n)]
    for u in range(g.n):
        for v in g.col[g.row_ptr[u]:g.row_ptr[u + 1]]:
            adj[u].add(int(v))
    return adj


def floyd_warshall(g):
    n = g.n
    adj = adjacency(g)
    d = [[0 if i == j else (1 if j in adj[i] else INF) for j in range(n)] for i in range(n)]
    for k, i, j in product(range(n), repeat=3):
        if d[i][k] + d[k][j] < d[i][j]:
            d[i][j] = d[i][k] + d[k][j]
    return d


def shortest_paths(g, s, t, dist=None):
    """All shortest s-t paths, by enumerating simple paths of length
    d(s,t) (d from Floyd-Warshall)."""
    if dist is None:
        dist = floyd_warshall(g)
    L = dist[s][t]
    if L == INF:
        return []
    adj = adjacency(g)
    out = []

    def rec(path):
        u = path[-1]
        if len(path) - 1 == L:
            if u == t:
                out.append(list(path))
            return
        for v in adj[u]:
            if v not in path:
                path.append(v)
                rec(path)
                path.pop()

    rec([s])
    return out


def canonical_order(paths):
    """Paths sorted by (v_{L-1}, v_{L-2}, ..., v_1): the order of the
    backward walk that picks predecessors in ascending id."""
    return sorted(paths, key=lambda p: tuple(reversed(p[1:-1])))


def ramp(x):
    return x if x > 0 else 0


def exact_percolation(g, k):
    """Definition 1, term by term, with x = k/65535 (the scale cancels)."""
    n = g.n
    dist = floyd_warshall(g)
    sig = {}
    through = {}
    for s in range(n):
        for t in range(n):
            if s == t:
                continue
            ps = shortest_paths(g, s, t, dist)
            sig[(s, t)] = len(ps)
            for p in ps:
                for v in p[1:-1]:
                    through[(s, t, v)] = through.get((s, t, v), 0) + 1
    p_out = []
    for v in range(n):
        S_v = sum(ramp(int(k[u]) - int(k[w])) for u in range(n) for w in range(n) if u != v and w != v)
        if S_v == 0:
            p_out.append(Fraction(0))
            continue
        tot = Fraction(0)
        for s in range(n):
            for t in range(n):
                if s == t or s == v or t == v or sig[(s, t)] == 0:
                    continue
                c = through.get((s, t, v), 0)
                if c:
                    tot += Fraction(c, sig[(s, t)]) * Fraction(ramp(int(k[s]) - int(k[t])), S_v)
        p_out.append(tot)
    return p_out


def pair_weights(k):
    """kappa~(s,t) numerators R(k_s - k_t) and their total."""
    n = len(k)
    Wt = {(s, t): ramp(int(k[s]) - int(k[t])) for s in range(n) for t in range(n) if s != t}
    return Wt, sum(Wt.values())


def likelihood_ratios(k):
    """d_v = max over pairs with kappa~ > 0 of kappa(s,t,v)/kappa~(s,t)."""
    n = len(k)
    Wt, tot = pair_weights(k)
    d = []
    for v in range(n):
        S_v = sum(ramp(int(k[u]) - int(k[w])) for u in range(n) for w in range(n) if u != v and w != v)
        best = Fraction(0)
        for (s, t), r in Wt.items():
            if r > 0 and s != v and t != v and S_v > 0:
                best = max(best, Fraction(r, S_v) / Fraction(r, tot))
        d.append(best)
    return d


def rho(g, k):
    """rho = sum_{s,t} |I(tau_st)| kappa~(s,t) (Section III-C)."""
    dist = floyd_warshall(g)
    Wt, tot = pair_weights(k)
    acc = Fraction(0)
    for (s, t), r in Wt.items():
        if r and dist[s][t] != INF:
            acc += Fraction((dist[s][t] - 1) * r, tot)
    return acc


def hit_expectation(g, k):
    """E[hits_v]/l = sum_{s,t} kappa~(s,t) sigma_st(v)/sigma_st (exact)."""
    n = g.n
    dist = floyd_warshall(g)
    Wt, tot = pair_weights(k)
    e = [Fraction(0)] * n
    for (s, t), r in Wt.items():
        if not r:
            continue
        ps = shortest_paths(g, s, t, dist)
        if not ps:
            continue
        for p in ps:
            for v in p[1:-1]:
                e[v] += Fraction(r, tot) / len(ps)
    return e
