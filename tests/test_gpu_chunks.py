"""GPU parity of launches split into many pair-kernel chunks
(PERCIS_OPT_PAIR_CHUNK): each chunk draws and lists its own pairs, and the
sampler, the handed-on pass and the 128-bit path run per chunk. Hits and
statistics must not depend on the chunk size, and must equal the oracle's."""
import numpy as np
import pytest

import workloads as W
from gpu_common import gpu_hits, oracle_hits, oracle_objects, same_stats

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("compact", [1, 2])
def test_small_chunks_match_oracle(compact):
    """ER(1000, 5000), 30,000 samples in chunks of 4096 (eight chunks, the
    last one ragged); a 35 x 35 grid whose corner pair takes the 128-bit path;
    a BA graph on compact slots. The result equals the oracle's and the
    one-chunk launch's."""
    from paper_2509_11454_amd import percis as P
    rng = np.random.default_rng(5)
    grid = W.grid_graph(35, 35)
    kg = np.full(grid.n, 32768, np.uint16)
    kg[0], kg[grid.n - 1] = 65535, 0
    ba = W.ba_graph(3000, 4, 9)
    cases = [W.workload_er1000() + (30000,), (grid, kg, 9000), (ba, W.uniform_states(ba.n, rng), 20000)]
    for g, k, n in cases:
        og, st = oracle_objects(g, k)
        ho, so = oracle_hits(og, st, 0, n, 17)
        out = []
        for chunk in (0, 4096, 1000):
            c = P.Context(0)
            c.set_option(P.OPT_COMPACT, compact)
            c.set_option(P.OPT_PAIR_CHUNK, chunk)
            c.load_csr(g.n, g.row_ptr, g.col, directed=g.directed)
            c.set_states(k)
            out.append(gpu_hits(c, 0, n, 17))
            c.close()
        for hg, sg in out:
            assert np.array_equal(ho, hg), g.name
            same_stats(so, sg)


def test_tasks_across_chunks():
    """Three tasks on two graphs in one launch of chunks of 2500 samples, so
    that tasks start and end inside chunks: each task's hits and statistics
    equal its own oracle run."""
    import torch
    from paper_2509_11454_amd import percis as P
    rng = np.random.default_rng(11)
    g0, k0 = W.workload_er1000()
    g1 = W.ba_graph(2000, 4, 3)
    k1 = W.skewed_states(g1.n, rng)
    c = P.Context(0)
    c.set_option(P.OPT_PAIR_CHUNK, 2500)
    c.load_csr(g0.n, g0.row_ptr, g0.col)
    c.set_states(k0)
    gid = c.add_graph(g1.n, g1.row_ptr, g1.col, k1)
    hits = [torch.zeros(g0.n, dtype=torch.int32, device="cuda"),
            torch.zeros(g1.n, dtype=torch.int32, device="cuda"),
            torch.zeros(g1.n, dtype=torch.int32, device="cuda")]
    tasks = [dict(graph=0, first=100, count=6100, seed=3, phase=0, hits=hits[0]),
             dict(graph=gid, first=0, count=4300, seed=4, phase=1, hits=hits[1]),
             dict(graph=gid, first=50, count=2600, seed=5, phase=2, hits=hits[2])]
    per, _ = c.sample_tasks(tasks)
    torch.cuda.synchronize()
    objs = [oracle_objects(g0, k0), oracle_objects(g1, k1), oracle_objects(g1, k1)]
    for i, t in enumerate(tasks):
        og, st = objs[i]
        ho, so = oracle_hits(og, st, t["first"], t["count"], t["seed"], t["phase"])
        assert np.array_equal(ho, hits[i].cpu().numpy().astype(np.uint32)), i
        same_stats(so, per[i])
    c.close()
