"""The no-allocation sampling call, percis_sample_range_noalloc, against
percis_sample_range through the C ABI. Calls in a row on one GPU share the
library's static scratch, laid out anew for each graph: each must give the
existing entry point's hits and statistics bit for bit, whatever the call
before it left there."""
import ctypes as C

import numpy as np
import pytest

import workloads as W
from gpu_common import gpu_context, same_stats

pytestmark = pytest.mark.gpu


def noalloc(c, first, count, seed, phase, hits, accumulate=False, flags=None):
    """The entry point called through the raw C ABI; returns (status, stats)."""
    from paper_2509_11454_amd import percis as P
    st = P.Stats()
    if flags is None:
        flags = P.DEVICE_PTRS | (P.ACCUMULATE if accumulate else 0)
    rc = P.raw_library().percis_sample_range_noalloc(c._h, first, count, seed, phase, C.c_void_p(hits.data_ptr()),
                                                     flags, C.byref(st))
    return rc, st.to_dict()


def reference(c, first, count, seed, phase, n):
    import torch
    h = torch.zeros(n, dtype=torch.int32, device="cuda")
    _, st = c.sample_range(first, count, seed, phase, hits=h)
    torch.cuda.synchronize()
    return h.cpu().numpy(), st


def check(c, n, first, count, seed, phase=0):
    import torch
    from paper_2509_11454_amd import percis as P
    ref_h, ref_st = reference(c, first, count, seed, phase, n)
    h = torch.full((n,), 7, dtype=torch.int32, device="cuda")    # overwritten by the call
    rc, st = noalloc(c, first, count, seed, phase, h)
    torch.cuda.synchronize()
    assert rc == P.OK, P.raw_library().percis_last_error(c._h)
    assert np.array_equal(h.cpu().numpy(), ref_h)
    same_stats(ref_st, st)
    assert st["samples"] == count
    return st


def test_noalloc_calls_in_a_row_match_sample_range():
    import torch
    from paper_2509_11454_amd import percis as P
    # 1: R-MAT scale 16 (65,536 nodes), 150,000 samples: three chunks, the
    # last one ragged, compact slots and a per-node slot for the samples
    # handed on
    g1 = W.rmat_graph(16, 16, seed=3)
    k1 = W.skewed_states(g1.n, np.random.default_rng(3))
    c1 = gpu_context(g1, k1)
    st = check(c1, g1.n, 1000, 150_000, 5)
    assert st["reachable"] > 0
    # 2: a smaller input: ER(1000, 5000), 3,000 samples, another context
    g2, k2 = W.workload_er1000()
    c2 = gpu_context(g2, k2)
    check(c2, g2.n, 0, 3000, 1)
    # 3: a 35 x 35 grid whose corner pairs have more than 2^64 shortest paths
    # (the 128-bit path's slot in the scratch)
    g3 = W.grid_graph(35, 35)
    k3 = np.full(g3.n, 32768, np.uint16)
    k3[0], k3[g3.n - 1] = 65535, 0
    c3 = gpu_context(g3, k3)
    check(c3, g3.n, 0, 4000, 2)
    # 4: back to the first graph, accumulating onto earlier hits
    ref_a, _ = reference(c1, 0, 20_000, 9, 1, g1.n)
    ref_b, ref_st = reference(c1, 20_000, 30_000, 9, 1, g1.n)
    h = torch.from_numpy(ref_a.copy()).cuda()
    rc, st = noalloc(c1, 20_000, 30_000, 9, 1, h, accumulate=True)
    assert rc == P.OK
    assert np.array_equal(h.cpu().numpy(), ref_a + ref_b)
    same_stats(ref_st, st)


def test_noalloc_rejections():
    import torch
    from paper_2509_11454_amd import percis as P
    g, k = W.workload_er1000()
    c = gpu_context(g, k)
    h = torch.zeros(g.n, dtype=torch.int32, device="cuda")
    assert noalloc(c, 0, 10, 1, 0, h, flags=0)[0] == P.E_INVAL            # host hits need staging
    assert noalloc(c, 0, 1 << 32, 1, 0, h)[0] == P.E_TOO_LARGE
    empty = P.Context(0)
    assert noalloc(empty, 0, 10, 1, 0, h)[0] == P.E_STATE                  # no graph yet
    # a path of 4,000,000 nodes: one per-node slot does not fit the scratch
    n = 4_000_000
    src = np.arange(n - 1, dtype=np.int32)
    big = W.csr_from_edges(n, src, src + 1, False, "path4M")
    kb = np.zeros(n, np.uint16)
    kb[0] = 65535
    cb = gpu_context(big, kb)
    hb = torch.zeros(n, dtype=torch.int32, device="cuda")
    rc, _ = noalloc(cb, 0, 10, 1, 0, hb)
    assert rc == P.E_TOO_LARGE
    assert b"about" in P.raw_library().percis_last_error(cb._h)
