"""GPU tests of the captured batch launch (percis_batch_*): a task set on
several graphs captured once as a HIP graph and replayed, with eager library
work and synchronisations between the replays. Every replay must give the
eager launch's hits and statistics bit for bit."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def build(P, compact, chunk=0):
    import torch
    rng = np.random.default_rng(21)
    g0, k0 = W.workload_er1000()
    g1 = W.ba_graph(3000, 4, 5)
    g2 = W.random_small_graph(120, 0.04, 7, directed=True)
    g3 = W.grid_graph(35, 35)                 # corner pair: counts past 2^64 (the 128-bit path)
    k3 = np.full(g3.n, 32768, np.uint16)
    k3[0], k3[g3.n - 1] = 65535, 0
    g4, k4 = W.with_isolated_component(W.er_graph(400, 900, 3), 40)
    c = P.Context(0)
    c.set_option(P.OPT_COMPACT, compact)
    c.set_option(P.OPT_PAIR_CHUNK, chunk)
    c.load_csr(g0.n, g0.row_ptr, g0.col)
    c.set_states(k0)
    ids = [0,
           c.add_graph(g1.n, g1.row_ptr, g1.col, W.skewed_states(g1.n, rng)),
           c.add_graph(g2.n, g2.row_ptr, g2.col, W.uniform_states(g2.n, rng), directed=True),
           c.add_graph(g3.n, g3.row_ptr, g3.col, k3),
           c.add_graph(g4.n, g4.row_ptr, g4.col, k4)]
    ns = [g0.n, g1.n, g2.n, g3.n, g4.n]
    hits = [torch.zeros(n, dtype=torch.int32, device="cuda") for n in ns]
    tasks = [dict(graph=ids[0], first=0, count=5000, seed=3, phase=0, hits=hits[0]),
             dict(graph=ids[1], first=100, count=7000, seed=4, phase=1, hits=hits[1]),
             dict(graph=ids[2], first=0, count=3000, seed=5, phase=2, hits=hits[2]),
             dict(graph=ids[3], first=0, count=6000, seed=2, phase=0, hits=hits[3]),
             dict(graph=ids[4], first=50, count=4000, seed=6, phase=0, hits=hits[4], accumulate=True)]
    return c, tasks, hits


@pytest.mark.parametrize("compact,chunk", [(1, 0), (2, 0), (1, 4096), (2, 4096)])
def test_captured_batch_replays_match_eager(compact, chunk):
    """chunk 4096: the captured launch holds seven pair-kernel chunks, and
    tasks start and end inside them."""
    import torch
    from paper_2509_11454_amd import percis as P
    c, tasks, hits = build(P, compact, chunk)
    eager_stats, eager_launch = c.sample_tasks(tasks)
    torch.cuda.synchronize()
    eager = [h.cpu().numpy().copy() for h in hits]
    acc_once = eager[4].copy()                 # the accumulating task's hits after one launch
    b = c.capture_batch(tasks)
    side = torch.zeros(1000, dtype=torch.int32, device="cuda")
    for rep in range(3):
        for i in range(4):
            hits[i].fill_(7)                   # cleared by the launch itself
        per, launch = b.replay()
        torch.cuda.synchronize()
        for i in range(4):
            assert np.array_equal(hits[i].cpu().numpy(), eager[i]), (rep, i)
        assert np.array_equal(hits[4].cpu().numpy(), acc_once * (rep + 2)), rep
        for i in range(5):
            for key in ("samples", "reachable", "sum_I", "sum_I2", "overflow"):
                assert per[i][key] == eager_stats[i][key], (rep, i, key)
        # work counters (edges, sigma_adds) may differ between runs: which
        # arcs of a last level are skipped, and (compact slots) which samples
        # near a table's limit are handed on and redone, depend on timing
        assert launch["samples"] == eager_launch["samples"], rep
        # eager work on the same context between replays
        c.sample_range(0, 1500, 11 + rep, 0, hits=side)
        torch.cuda.synchronize()
    b.close()


def test_capture_is_invalidated_by_new_states():
    import torch
    from paper_2509_11454_amd import percis as P
    c, tasks, hits = build(P, 0)
    b = c.capture_batch(tasks[:2])
    b.replay()
    c.set_states(W.uniform_states(1000, np.random.default_rng(3)))
    with pytest.raises(P.PercisError) as e:
        b.replay()
    assert e.value.status == P.E_STATE
    b.close()
    b2 = c.capture_batch(tasks[:2])           # a new capture sees the new states
    per, _ = b2.replay()
    eager, _ = c.sample_tasks(tasks[:2])
    torch.cuda.synchronize()
    assert [p["sum_I"] for p in per] == [p["sum_I"] for p in eager]
    b2.close()


def test_capture_is_invalidated_by_degenerate_states():
    """All-equal states are rejected (the pair distribution is undefined),
    but their build has already rewritten the arrays the capture reads: the
    replay must refuse to run, and sampling the graph must too, until new
    states are set."""
    from paper_2509_11454_amd import percis as P
    c, tasks, hits = build(P, 0)
    b = c.capture_batch(tasks[:2])
    b.replay()
    with pytest.raises(P.PercisError) as e:
        c.set_states(np.full(1000, 1234, np.uint16))
    assert e.value.status == P.E_DEGENERATE
    with pytest.raises(P.PercisError) as e:
        b.replay()
    assert e.value.status == P.E_STATE
    with pytest.raises(P.PercisError) as e:
        c.sample_tasks(tasks[:1])
    assert e.value.status == P.E_STATE
    b.close()
    c.set_states(W.uniform_states(1000, np.random.default_rng(4)))
    b2 = c.capture_batch(tasks[:2])
    per, _ = b2.replay()
    eager, _ = c.sample_tasks(tasks[:2])
    assert [p["sum_I"] for p in per] == [p["sum_I"] for p in eager]
    b2.close()
