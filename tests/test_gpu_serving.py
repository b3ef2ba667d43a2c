"""GPU tests of the continuous-batching server: each query's estimate is
bit-identical alone, in a mix, and to percis_graph_estimate with the same
arguments; admission never exceeds the memory budget."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def serving_context():
    from paper_2509_11454_amd import percis as P
    rng = np.random.default_rng(3)
    c = P.Context(0)
    g0, k0 = W.workload_er1000()
    c.load_csr(g0.n, g0.row_ptr, g0.col)
    c.set_states(k0)
    ids = [0]
    for n in (2000, 5000):
        g = W.ba_graph(n, 4, n)
        ids.append(c.add_graph(g.n, g.row_ptr, g.col, W.uniform_states(g.n, rng)))
    g = W.with_isolated_component(W.er_graph(300, 800, 6), 20)
    ids.append(c.add_graph(g[0].n, g[0].row_ptr, g[0].col, g[1]))
    return c, ids


QUERIES = [(0, 0.05, 0.1, 1), (1, 0.03, 0.1, 2), (2, 0.05, 0.05, 3), (3, 0.04, 0.1, 4), (0, 0.02, 0.1, 5),
           (2, 0.05, 0.1, 6), (1, 0.05, 0.2, 7)]


def run_server(c, queries, budget, chunk=2048, step=16384):
    from paper_2509_11454_amd import percis as P
    srv = P.Server(c, budget, chunk, step)
    qids = [srv.submit(*q) for q in queries]
    out = {}
    steps = 0
    peak_active = 0
    while len(out) < len(qids):
        srv.step()
        steps += 1
        st = srv.status()
        peak_active = max(peak_active, st["active"])
        assert st["bytes_in_use"] <= budget
        for q in qids:
            if q not in out:
                r = srv.result(q)
                if r is not None:
                    out[q] = r
        assert steps < 100000
    st = srv.status()
    srv.close()
    return [out[q] for q in qids], peak_active, st


def test_server_matches_estimate_and_alone():
    c, ids = serving_context()
    queries = [(ids[g], e, d, s) for g, e, d, s in QUERIES]
    mixed, peak_active, st = run_server(c, queries, budget=1 << 30)
    assert peak_active >= 3  # queries really overlapped
    for q, (rc, p, info) in zip(queries, mixed):
        assert rc == 0
        p_ref, info_ref = c.graph_estimate(q[0], q[1], q[2], q[3])
        assert info["l1"] == info_ref["l1"] and info["l"] == info_ref["l"]
        assert np.array_equal(p, p_ref)
        alone, _, _ = run_server(c, [q], budget=1 << 30)
        assert np.array_equal(alone[0][1], p)


def test_server_memory_admission():
    """A budget that holds one hit buffer of the largest graph: at most one
    query is admitted at a time, results are unchanged."""
    c, ids = serving_context()
    queries = [(ids[g], e, d, s) for g, e, d, s in QUERIES[:4]]
    budget = 5000 * 4 + 256
    res, peak_active, st = run_server(c, queries, budget=budget)
    assert st["peak_bytes"] <= budget
    for q, (rc, p, info) in zip(queries, res):
        assert rc == 0
        p_ref, _ = c.graph_estimate(q[0], q[1], q[2], q[3])
        assert np.array_equal(p, p_ref)
