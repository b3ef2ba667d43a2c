"""GPU parity of the compact slots (PERCIS_OPT_COMPACT = 2): node records
indexed by LDS-table position, with the samples whose ball outgrows a table
handed to the per-node slots. Hits and statistics must equal the oracle's
bit for bit, whether a sample stayed compact, was handed on, or took the
128-bit path."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_common import gpu_hits, oracle_hits, oracle_objects, same_stats

pytestmark = pytest.mark.gpu


def compact_context(g, k, slots=0, block=0):
    from paper_2509_11454_amd import percis as P
    c = P.Context(0)
    c.set_option(P.OPT_COMPACT, 2)
    if slots:
        c.set_option(P.OPT_SLOTS, slots)
    if block:
        c.set_option(P.OPT_BLOCK, block)
    c.load_csr(g.n, g.row_ptr, g.col, directed=g.directed)
    c.set_states(k)
    return c


def cases():
    rng = np.random.default_rng(8)
    out = []
    g, k = W.workload_er1000()
    out.append(("er1000", g, k, 5000, 0, 0, False))
    g = W.ba_graph(2000, 4, 11)
    out.append(("ba2000 skewed", g, W.skewed_states(g.n, rng), 4000, 3, 0, False))
    g = W.random_small_graph(60, 0.06, 301, directed=True)
    out.append(("directed 60", g, W.uniform_states(g.n, rng), 4000, 0, 256, False))
    g, k = W.with_isolated_component(W.er_graph(300, 700, 9), 50)
    out.append(("isolated", g, k, 4000, 0, 64, False))
    g = W.grid_graph(40, 40)        # balls past 768 nodes: samples handed on
    out.append(("grid 40x40", g, W.uniform_states(g.n, rng), 3000, 0, 0, True))
    # the end layers at the extreme states: about one sample in n joins
    # them, and that search takes the 4000-node middle layer into a ball
    g = W.layered_graph([1, 3, 4000, 2, 1])
    out.append(("layered 4000", g, ends_states(g.n, 1), 40000, 5, 0, True))
    g = W.layered_graph([2, 40, 4000, 40, 2], directed=True)
    out.append(("layered 4000 directed", g, ends_states(g.n, 2), 40000, 0, 0, True))
    return out


def ends_states(n, width):
    k = np.full(n, 32768, np.uint16)
    k[:width] = 65535
    k[n - width:] = 0
    return k


@pytest.mark.parametrize("ci", range(7))
def test_compact_slots_match_oracle(ci):
    from paper_2509_11454_amd import percis as P
    name, g, k, n, slots, block, hands_on = cases()[ci]
    og, st = oracle_objects(g, k)
    ho, so = oracle_hits(og, st, 0, n, 40 + ci)
    c = compact_context(g, k, slots, block)
    assert c.get_option(P.OPT_COMPACT) == 2
    hg, sg = gpu_hits(c, 0, n, 40 + ci)
    assert np.array_equal(ho, hg), name
    same_stats(so, sg)
    if hands_on:
        assert sg["deferred"] > 0, name
    c.close()


def test_compact_wide_counts():
    """35 x 35 grid with a likely corner pair: samples with sigma_st >= 2^64
    go from the compact slots (or, handed on, from the per-node slots) to the
    128-bit path; hits equal the oracle's."""
    g = W.grid_graph(35, 35)
    k = np.full(g.n, 32768, np.uint16)
    k[0], k[g.n - 1] = 65535, 0
    og, st = oracle_objects(g, k)
    ho, so = oracle_hits(og, st, 0, 6000, 2)
    assert so["overflow"] == 0
    c = compact_context(g, k)
    hg, sg = gpu_hits(c, 0, 6000, 2)
    assert np.array_equal(ho, hg)
    same_stats(so, sg)
    c.close()


def test_compact_agrees_with_per_node_slots_on_rmat18():
    """A window of the R-MAT 18 benchmark: compact and per-node slots give
    identical hits and statistics."""
    from paper_2509_11454_amd import percis as P
    g, k = W.workload_rmat18()
    res = []
    for mode in (1, 2):
        c = P.Context(0)
        c.set_option(P.OPT_COMPACT, mode)
        c.load_csr(g.n, g.row_ptr, g.col)
        c.set_states(k)
        assert c.get_option(P.OPT_COMPACT) == mode
        res.append(gpu_hits(c, 1000, 60000, 9))
        c.close()
    assert np.array_equal(res[0][0], res[1][0])
    same_stats(res[0][1], res[1][1])


def double_broom(leaves):
    """Hubs 0 and 1 joined by the path 0 - 2 - 3 - 1, each with `leaves`
    leaves: a search between leaves of different hubs takes a whole broom
    (leaves + 1 nodes) into one ball."""
    e = [(0, 2), (2, 3), (3, 1)]
    n = 4
    for hub in (0, 1):
        for _ in range(leaves):
            e.append((hub, n))
            n += 1
    return W.from_edge_list(n, e, directed=False, name="double broom %d" % leaves)


def test_compact_hands_large_balls_to_per_node_slots():
    """Balls of 30001 nodes outgrow any compact slot, so these samples end on
    the per-node slots; hits and statistics equal the oracle's."""
    g = double_broom(30000)
    rng = np.random.default_rng(12)
    k = W.uniform_states(g.n, rng)
    og, st = oracle_objects(g, k)
    ho, so = oracle_hits(og, st, 0, 2000, 13)
    c = compact_context(g, k)
    hg, sg = gpu_hits(c, 0, 2000, 13)
    assert np.array_equal(ho, hg)
    same_stats(so, sg)
    assert sg["deferred"] > 0
    c.close()


def test_compact_estimates_equal_per_node_estimates():
    """Algorithm 1 and PercIS-DI end to end (bounds, both phases, the
    estimate) give bit-identical results on compact and per-node slots."""
    from paper_2509_11454_amd import percis as P
    g, k = W.workload_er1000()
    h = W.ba_graph(3000, 4, 5)
    kh = W.skewed_states(h.n, np.random.default_rng(4))
    res = []
    for mode in (1, 2):
        c = P.Context(0)
        c.set_option(P.OPT_COMPACT, mode)
        c.load_csr(g.n, g.row_ptr, g.col)
        c.set_states(k)
        gid = c.add_graph(h.n, h.row_ptr, h.col, kh)
        assert c.get_option(P.OPT_COMPACT) == mode
        res.append([c.estimate(0.02, 0.1, 3), c.graph_estimate(gid, 0.03, 0.1, 4),
                    c.graph_estimate_di(0, 0.05, 0.1, 5)])
        c.close()
    for (p1, i1), (p2, i2) in zip(res[0], res[1]):
        assert np.array_equal(p1, p2)
        for key in ("l1", "l", "D", "d_hat", "rho_hat", "v_hat", "x_hat", "overflow"):
            assert i1[key] == i2[key], key


def test_compact_serving_matches_per_node_estimates():
    """The continuous-batching server on compact slots returns, per query,
    the estimate that per-node slots give."""
    from paper_2509_11454_amd import percis as P
    import test_gpu_serving as S
    c, ids = S.serving_context()
    ref = [c.graph_estimate(ids[gi], e, d, s) for gi, e, d, s in S.QUERIES[:5]]
    c.close()
    c, ids = S.serving_context()
    c.set_option(P.OPT_COMPACT, 2)
    queries = [(ids[gi], e, d, s) for gi, e, d, s in S.QUERIES[:5]]
    out, _, _ = S.run_server(c, queries, budget=1 << 30)
    assert c.get_option(P.OPT_COMPACT) == 2
    for (rc, p, info), (p_ref, info_ref) in zip(out, ref):
        assert rc == 0 and info["l"] == info_ref["l"]
        assert np.array_equal(p, p_ref)
