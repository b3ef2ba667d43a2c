"""GPU parity on the full-size workloads, in the launch configurations the
benchmark times, against the oracle's bidirectional search mode (proved equal
to its truncated BFS by the CPU tests):

- R-MAT scale 18, skewed states: two windows of 10^4 samples of the
  10^6-sample step, and the step itself by additivity;
- directed R-MAT scale 24, Beta(1/2, 1/2) states: the first 10^5 samples of
  the 10^7-sample step, a window that holds hundreds of samples handed on by
  the compact slots and of samples whose visited set spilled to device
  memory, and the step itself by additivity;
- 64 Barabasi-Albert graphs: every graph's 10^5 samples from inside the one
  captured launch, with the knobs the autotuner chose over all 64 graphs;
- serving: one query per resident graph (66), each the same in the mix,
  alone in the server, through percis_graph_estimate and from the oracle's
  phase-1 statistics and phase-2 hits.
Integer results (hits, sample statistics) must be bit-identical; floating
results are held to the tolerances stated beside each check."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_common import gpu_context, gpu_hits, oracle_hits, oracle_objects, release_oracle_work, same_stats

pytestmark = pytest.mark.gpu


def check_window(c, og, st, first, count, seed):
    hg, sg = gpu_hits(c, first, count, seed)
    ho, so = oracle_hits(og, st, first, count, seed, bidir=True)
    assert np.array_equal(ho, hg), (first, count)
    same_stats(so, sg)
    return hg, sg


@pytest.mark.timeout(600)
def test_rmat18_windows_and_full_step():
    g, k = W.workload_rmat18()
    og, st = oracle_objects(g, k)
    c = gpu_context(g, k)
    N, w = 1_000_000, 10_000
    h_head, s_head = check_window(c, og, st, 0, w, 1)
    check_window(c, og, st, N - w, w, 1)
    assert s_head["reachable"] > 3000
    release_oracle_work()
    h_full, s_full = gpu_hits(c, 0, N, 1)
    assert s_full["samples"] == N and s_full["overflow"] == 0
    assert int(h_full.astype(np.uint64).sum()) == s_full["sum_I"]
    h_rest, s_rest = gpu_hits(c, w, N - w, 1)
    assert np.array_equal(h_full, h_head + h_rest)
    for key in ("samples", "reachable", "sum_I", "sum_I2"):
        assert s_full[key] == s_head[key] + s_rest[key], key
    c.close()


@pytest.mark.timeout(900)
def test_rmat24_directed_window_and_full_step():
    """The window [0, 10^5) is one launch in the benchmark's shape (compact
    slots, then per-node slots for the samples handed on); it must carry at
    least 200 handed-on samples and 50 samples that spilled a visited set,
    so that both passes and the spill path are checked."""
    g, k = W.workload_rmat24_directed()
    c = gpu_context(g, k)
    N, w = 10_000_000, 100_000
    h_win, s_win = gpu_hits(c, 0, w, 1)
    print("rmat24d window: deferred %d spilled %d reachable %d" % (s_win["deferred"], s_win["spilled"],
                                                                   s_win["reachable"]), flush=True)
    assert s_win["deferred"] >= 200 and s_win["spilled"] >= 50
    h_full, s_full = gpu_hits(c, 0, N, 1)
    h_rest, s_rest = gpu_hits(c, w, N - w, 1)
    assert s_full["samples"] == N and s_full["overflow"] == 0
    assert int(h_full.astype(np.uint64).sum()) == s_full["sum_I"]
    assert np.array_equal(h_full, h_win + h_rest)
    for key in ("samples", "reachable", "sum_I", "sum_I2"):
        assert s_full[key] == s_win[key] + s_rest[key], key
    c.close()
    del c
    og, st = oracle_objects(g, k)
    del g
    ho, so = oracle_hits(og, st, 0, w, 1, bidir=True)
    release_oracle_work()
    assert np.array_equal(ho, h_win)
    same_stats(so, s_win)


@pytest.mark.timeout(900)
def test_ba64_captured_launch_full_parity():
    """The benchmark's batch: 64 BA graphs, the knobs autotuned over all
    of them, 10^5 samples per graph (seed 1 + graph index) in one captured
    launch; each graph's hits and statistics from the replay equal the
    oracle's over the same 10^5 samples."""
    import torch
    from paper_2509_11454_amd import percis as P
    graphs = W.workload_ba_batch(64, 4, 1)
    c = P.Context(0)
    g0, k0 = graphs[0]
    c.load_csr(g0.n, g0.row_ptr, g0.col)
    c.set_states(k0)
    ids = [0] + [c.add_graph(g.n, g.row_ptr, g.col, kk) for g, kk in graphs[1:]]
    tune = c.autotune(-1, 200_000)
    print("autotune:", tune, flush=True)
    per = 100_000
    hits = [torch.zeros(g.n, dtype=torch.int32, device="cuda") for g, _ in graphs]
    tasks = [dict(graph=ids[i], first=0, count=per, seed=1 + i, phase=0, hits=hits[i]) for i in range(64)]
    b = c.capture_batch(tasks)
    per_task, launch = b.replay()
    torch.cuda.synchronize()
    got = [h.cpu().numpy().view(np.uint32).copy() for h in hits]
    b.close()
    c.close()
    assert launch["samples"] == 64 * per
    nmax = max(g.n for g, _ in graphs)
    from gpu_common import oracle_work
    oracle_work(16, nmax)
    for i, (g, kk) in enumerate(graphs):
        og, st = oracle_objects(g, kk)
        ho, so = oracle_hits(og, st, 0, per, 1 + i, bidir=True)
        assert np.array_equal(ho, got[i]), i
        same_stats(so, per_task[i])
        if i % 8 == 7:
            print("ba64: graphs 0..%d equal the oracle" % i, flush=True)
    release_oracle_work()


def serving_graphs():
    g0, k0 = W.workload_er1000()
    g1, k1 = W.workload_rmat18()
    return [(g0, k0), (g1, k1)] + W.workload_ba_batch(64, 4, 1)


@pytest.mark.timeout(1200)
def test_serving_66_graphs_mixed_alone_and_oracle():
    """One query per resident graph (ER 1000, R-MAT 18, 64 BA), eps drawn
    from {0.01, 0.005, 0.001}, delta 0.1, seed = the query's index, all
    submitted at once to a server with the benchmark's budget and chunking.
    Each result equals the same query alone in a server and
    percis_graph_estimate bit for bit. Against the oracle: the phase-1
    sample statistics give rho_tilde and Lambda (1e-12 relative), l is the
    oracle's supremum for the query's d_hat, rho_hat and v_hat (to the
    resolution of the two searches), and the estimate is d_v h_v / l with
    the oracle's phase-2 hits h (the same double formula, 1e-12 relative)."""
    from paper_2509_11454_amd import percis as P
    graphs = serving_graphs()
    c = P.Context(0)
    c.load_csr(graphs[0][0].n, graphs[0][0].row_ptr, graphs[0][0].col)
    c.set_states(graphs[0][1])
    ids = [0] + [c.add_graph(g.n, g.row_ptr, g.col, kk) for g, kk in graphs[1:]]
    rng = np.random.default_rng(5)
    queries = [(ids[i], float(rng.choice([0.01, 0.005, 0.001])), 0.1, i) for i in range(len(ids))]
    budget, chunk, step = 256 << 20, 65536, 524288

    def serve(qs):
        srv = P.Server(c, budget, chunk, step)
        qids = [srv.submit(*q) for q in qs]
        out, peak = {}, 0
        while len(out) < len(qids):
            srv.step()
            peak = max(peak, srv.status()["active"])
            for q in qids:
                if q not in out:
                    r = srv.result(q)
                    if r is not None:
                        out[q] = r
        srv.close()
        return [out[q] for q in qids], peak

    mixed, peak = serve(queries)
    assert peak >= 8
    print("serving: %d queries in the mix, peak %d active" % (len(queries), peak), flush=True)
    for i, (q, (rc, p, info)) in enumerate(zip(queries, mixed)):
        if i % 11 == 0:
            print("serving: alone and graph_estimate from query %d" % i, flush=True)
        assert rc == 0
        (rc1, p1, info1), = serve([q])[0]
        assert rc1 == 0 and np.array_equal(p1, p) and info1["l"] == info["l"]
        p2, info2 = c.graph_estimate(*q)
        assert np.array_equal(p2, p) and info2["l"] == info["l"]
    c.close()
    nmax = max(g.n for g, _ in graphs)
    from gpu_common import oracle_work
    oracle_work(16, nmax)
    for i, (q, (rc, p, info), (g, kk)) in enumerate(zip(queries, mixed, graphs)):
        if i % 11 == 0:
            print("serving: oracle from query %d (l = %d)" % (i, info["l"]), flush=True)
        og, st = oracle_objects(g, kk)
        _, eps, delta, seed = q
        l1 = info["l1"]
        assert l1 == math.ceil(max(1000, math.log(1 / delta) / eps))
        _, s1 = oracle_hits(og, st, 0, l1, seed, phase=1, bidir=True)
        rho = s1["sum_I"] / l1
        lam = (s1["sum_I2"] - s1["sum_I"] ** 2 / l1) / (l1 - 1)
        assert abs(info["rho_tilde"] - rho) <= 1e-12 * max(1.0, rho)
        assert abs(info["Lambda"] - lam) <= 1e-12 * max(1.0, lam)
        l_orc = O.sample_size(info["d_hat"], info["rho_hat"], info["v_hat"], eps, delta)[0]
        assert abs(info["l"] - math.ceil(l_orc)) <= 1 + 1e-6 * l_orc
        h2, _ = oracle_hits(og, st, 0, info["l"], seed, phase=2, bidir=True)
        S = st.arrays()["S"]
        dv = np.where(S > 0, st.C / np.where(S > 0, S, 1.0), 0.0)
        assert np.allclose(p, dv * h2 / info["l"], rtol=1e-12, atol=0), q
    release_oracle_work()
