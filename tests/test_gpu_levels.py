"""GPU parity of BFS levels whose frontier rows span more than one batch.

Such a level first scans its entries for arcs into the other ball and lists
them in LDS. The processing pass then takes one of three routes:
- the list, when the level meets;
- every entry again, when it does not meet;
- a rescan that keeps the arcs into the other ball, when they outnumber the
  list's 128 entries.

Two hubs with `shared` common neighbours and `private` leaves each reach all
three routes. From one hub's side, the first level scans shared + private
entries and does not meet. From the other side, the level meets through the
`shared` arcs. Paths, counts and hits must equal the oracle's bit for bit,
at every block size and on per-node and compact slots."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_common import gpu_hits, oracle_hits, oracle_objects, same_stats

pytestmark = pytest.mark.gpu


def two_hubs(shared, private, directed=False):
    """Hubs 0 and 1; nodes 2 .. 2+shared-1 adjacent to both; then `private`
    leaves of hub 0 and `private` leaves of hub 1. Directed: 0 -> shared -> 1,
    0 -> its leaves, hub 1's leaves -> 1, and 1 -> 0 so that both hubs reach
    everything."""
    e = []
    n = 2
    for _ in range(shared):
        e += [(0, n), (n, 1)]
        n += 1
    for hub in (0, 1):
        for _ in range(private):
            e.append((0, n) if hub == 0 else (n, 1))
            n += 1
    if directed:
        e.append((1, 0))
    return W.from_edge_list(n, e, directed=directed,
                            name="two hubs %d shared %d private%s" % (shared, private, " directed" if directed else ""))


# (shared, private, directed). A batch is 6 entries per thread: 384 entries
# at 64 threads, 3072 at 512. The hub rows of 3600 to 4300 entries span
# several batches at every block size below, those of about 1100 entries at
# 64 and 128 threads. The compact slots hold balls of up to 1536 nodes, which
# the 1100-node cases stay within.
GRAPHS = [(100, 1000, False), (100, 4000, False), (300, 4000, False), (1000, 60, False), (3500, 100, False),
          (100, 4000, True), (300, 4000, True)]


@pytest.mark.parametrize("gi", range(len(GRAPHS)))
@pytest.mark.parametrize("block", [0, 64, 256, 512])
def test_hub_pair_paths(gi, block):
    """The hub-to-hub search meets through `shared` arcs in a level of
    shared + private entries; L, sigma and the chosen paths equal the
    oracle's."""
    from paper_2509_11454_amd import percis as P
    g = two_hubs(*GRAPHS[gi])
    og = O.Graph(g.n, g.row_ptr, g.col, g.directed)
    c = P.Context(0)
    if block:
        c.set_option(P.OPT_BLOCK, block)
    c.load_csr(g.n, g.row_ptr, g.col, directed=g.directed)
    pairs = [(0, 1), (2 + GRAPHS[gi][0], g.n - 1), (g.n - 1, 2 + GRAPHS[gi][0])]
    if not g.directed:
        pairs.append((1, 0))
    for s, t in pairs:
        L0, sig0, _ = O.path(og, s, t, 0)
        rs = sorted({0, sig0 // 2, sig0 - 1}) if L0 > 0 else [0]
        for r in rs:
            L, sig, ovf, p = c.debug_path(s, t, r)
            assert (L, ovf) == (L0, 0), (g.name, s, t)
            if L0 > 0:
                assert sig == sig0
                assert p == O.path(og, s, t, r)[2], (g.name, s, t, r)
        if L0 > 0:
            # a path index past sigma_st: L and sigma_st, no path, no error
            assert c.debug_path(s, t, sig0) == (L0, sig0, 0, None), (g.name, s, t)
    c.close()


@pytest.mark.parametrize("gi", range(len(GRAPHS)))
@pytest.mark.parametrize("compact,block", [(1, 0), (1, 512), (2, 0), (2, 256)])
def test_hub_graph_sampling(gi, compact, block):
    """Sampling with uniform states: leaf-to-leaf searches across the hubs
    take all three routes. Hits and statistics equal the oracle's."""
    from paper_2509_11454_amd import percis as P
    g = two_hubs(*GRAPHS[gi])
    k = W.uniform_states(g.n, np.random.default_rng(30 + gi))
    og, st = oracle_objects(g, k)
    ho, so = oracle_hits(og, st, 0, 4000, 60 + gi)
    c = P.Context(0)
    c.set_option(P.OPT_COMPACT, compact)
    if block:
        c.set_option(P.OPT_BLOCK, block)
    c.load_csr(g.n, g.row_ptr, g.col, directed=g.directed)
    c.set_states(k)
    hg, sg = gpu_hits(c, 0, 4000, 60 + gi)
    assert np.array_equal(ho, hg), g.name
    same_stats(so, sg)
    c.close()
