"""CPU-only checks of the C ABI: the library loads and exports every symbol
that include/percis.h declares, and the host-side logic (validation, call
order, degenerate states, size limits) behaves as the header documents,
through a host-only context that makes no HIP call."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "percis.h")
LIB = os.path.join(ROOT, "paper_2509_11454_amd", "lib", "libpercis.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libpercis.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(percis_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    lib = C.CDLL(LIB)
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    out = os.popen("nm -D --defined-only %s" % LIB).read()
    for name in names:
        assert re.search(r"\bT %s\b" % name, out), name


@pytest.fixture(scope="module")
def P():
    from paper_2509_11454_amd import percis
    return percis


def ctx(P):
    return P.Context(P.HOST_ONLY)


def test_binding_names_match_header(P):
    assert set(P.EXPORTED) == set(declared_functions())


def test_host_only_valid_graph_and_states(P):
    c = ctx(P)
    g, k = W.workload_er1000()
    c.load_csr(g.n, g.row_ptr, g.col)
    c.set_states(k)
    with pytest.raises(P.PercisError) as e:
        c.sample(10, 1, hits=np.zeros(g.n, np.uint32))
    assert e.value.status == P.E_STATE


@pytest.mark.parametrize("case", ["nonmonotone", "range", "selfloop", "dup", "asym", "rp0", "rpn"])
def test_csr_validation(P, case):
    c = ctx(P)
    n = 4
    rp = np.array([0, 1, 2, 3, 4], np.int32)
    col = np.array([1, 0, 3, 2], np.int32)
    c.load_csr(n, rp, col)  # valid: two edges
    if case == "nonmonotone":
        rp = np.array([0, 2, 1, 3, 4], np.int32)
    elif case == "range":
        col = np.array([1, 0, 3, 7], np.int32)
    elif case == "selfloop":
        col = np.array([0, 0, 3, 2], np.int32)
    elif case == "dup":
        rp = np.array([0, 2, 3, 4, 5], np.int32)
        col = np.array([1, 1, 0, 3, 2], np.int32)
    elif case == "asym":
        col = np.array([1, 0, 3, 1], np.int32)
    elif case == "rp0":
        rp = np.array([1, 1, 2, 3, 4], np.int32)
    elif case == "rpn":
        rp = np.array([0, 1, 2, 3, 3], np.int32)
    with pytest.raises(P.PercisError) as e:
        c.load_csr(n, rp, col)
    assert e.value.status == P.E_INVAL


def test_directed_asymmetric_ok_and_unsorted_rows(P):
    c = ctx(P)
    rp = np.array([0, 2, 2, 3], np.int32)
    col = np.array([2, 1, 0], np.int32)   # row 0 unsorted
    c.load_csr(3, rp, col, directed=True)
    with pytest.raises(P.PercisError):
        c.load_csr(3, rp, col, directed=False)


def test_call_order_and_degenerate(P):
    c = ctx(P)
    with pytest.raises(P.PercisError) as e:
        c.set_states(np.zeros(3, np.uint16))
    assert e.value.status == P.E_STATE
    g = W.path_graph(5)
    c.load_csr(g.n, g.row_ptr, g.col)
    with pytest.raises(P.PercisError) as e:
        c.set_states(np.full(5, 777, np.uint16))
    assert e.value.status == P.E_DEGENERATE
    c.set_states(np.array([1, 0, 0, 0, 0], np.uint16))


def test_too_large(P):
    c = ctx(P)
    rp = np.zeros(2, np.int32)
    lib = P.raw_library()
    rc = lib.percis_load_csr(c._h, (1 << 25) + 1, 0, rp.ctypes.data_as(C.c_void_p), None, 0)
    assert rc == P.E_TOO_LARGE


def test_status_strings(P):
    lib = P.raw_library()
    for code in range(0, -8, -1):
        assert lib.percis_status_str(code)
    assert lib.percis_status_str(-99) == b"unknown status"


def test_option_validation(P):
    c = ctx(P)
    for b in (0, 64, 128, 256, 512, 1024):
        c.set_option(P.OPT_BLOCK, b)
        assert c.get_option(P.OPT_BLOCK) == b
    for b in (32, 100, 2048):
        with pytest.raises(P.PercisError) as e:
            c.set_option(P.OPT_BLOCK, b)
        assert e.value.status == P.E_INVAL
    with pytest.raises(P.PercisError):
        c.set_option(P.OPT_BITMAPS, 3)
    with pytest.raises(P.PercisError):
        c.set_option(P.OPT_SLOTS, -1)
    for v in (0, 1, 2):
        c.set_option(P.OPT_COMPACT, v)
        assert c.get_option(P.OPT_COMPACT) == v
    with pytest.raises(P.PercisError) as e:
        c.set_option(P.OPT_COMPACT, 3)
    assert e.value.status == P.E_INVAL
    for b in (0, 64, 128, 256, 512, 1024):
        c.set_option(P.OPT_DEFER_BLOCK, b)
        assert c.get_option(P.OPT_DEFER_BLOCK) == b
    with pytest.raises(P.PercisError):
        c.set_option(P.OPT_DEFER_BLOCK, 96)
    assert c.get_option(P.OPT_PAIR_CHUNK) == 1 << 24   # the default chunk
    for v in (1, 4096, 1 << 30):
        c.set_option(P.OPT_PAIR_CHUNK, v)
        assert c.get_option(P.OPT_PAIR_CHUNK) == v
    with pytest.raises(P.PercisError) as e:
        c.set_option(P.OPT_PAIR_CHUNK, (1 << 30) + 1)
    assert e.value.status == P.E_INVAL
    c.set_option(P.OPT_PAIR_CHUNK, 0)
    assert c.get_option(P.OPT_PAIR_CHUNK) == 1 << 24
    assert c.get_option(P.OPT_BALANCE) == 100   # the balanced rule
    for v in (25, 50, 200, 400):
        c.set_option(P.OPT_BALANCE, v)
        assert c.get_option(P.OPT_BALANCE) == v
    for v in (1, 24, 401):
        with pytest.raises(P.PercisError):
            c.set_option(P.OPT_BALANCE, v)
    c.set_option(P.OPT_BALANCE, 0)
    assert c.get_option(P.OPT_BALANCE) == 100
    with pytest.raises(P.PercisError) as e:   # nothing to time on a host-only context
        c.autotune(-1, 1000)
    assert e.value.status == P.E_STATE


def test_batch_capture_needs_a_device(P):
    c = ctx(P)
    g, k = W.workload_er1000()
    c.load_csr(g.n, g.row_ptr, g.col)
    c.set_states(k)
    lib = P.raw_library()
    h = C.c_void_p()
    rc = lib.percis_batch_capture(c._h, 0, None, C.byref(h))
    assert rc == P.E_INVAL and not h.value
    arr = (P.Task * 1)()
    arr[0] = P.Task(0, 0, 0, 10, 1, C.c_void_p(0x1000), 0, None)   # never dereferenced: no device
    rc = lib.percis_batch_capture(c._h, 1, arr, C.byref(h))
    assert rc == P.E_STATE and not h.value
    lib.percis_batch_destroy(None)   # a null batch is accepted


def test_task_hits_checked_before_any_launch(P):
    """A task's hits tensor must hold its graph's node count: the library
    gets a bare pointer and would write past a shorter buffer. The binding
    rejects it (and a host tensor) before calling into the library."""
    import torch
    c = ctx(P)
    g, k = W.workload_er1000()
    c.load_csr(g.n, g.row_ptr, g.col)
    c.set_states(k)
    small = torch.zeros(g.n - 1, dtype=torch.int32)
    task = dict(graph=0, first=0, count=10, seed=1, hits=small)
    for call in (c.sample_tasks, c.capture_batch):
        with pytest.raises(ValueError, match="holds %d entries" % (g.n - 1)):
            call([task])
        with pytest.raises(ValueError, match="device tensor"):
            call([dict(task, hits=torch.zeros(g.n, dtype=torch.int32))])
        with pytest.raises(TypeError):
            call([dict(task, hits=torch.zeros(g.n, dtype=torch.int64))])
    with pytest.raises(ValueError):
        c.sample_range(0, 10, 1, hits=np.zeros(g.n - 1, np.uint32))


def test_threaded_graph_checks_report_the_first_failure(P):
    """A graph of 2^20 nodes and ~12 M arcs is checked and renumbered on
    several host threads; each planted fault must be caught and, with two
    faults of one kind, the one a serial pass meets first is reported."""
    g = W.rmat_graph(20, 12, seed=7, directed=True)
    assert g.m > 8 << 20
    c = ctx(P)
    c.load_csr(g.n, g.row_ptr, g.col, directed=True)
    rp = g.row_ptr.astype(np.int64)
    deg = np.diff(rp)
    early = int(np.nonzero(deg >= 2)[0][10])
    late = int(np.nonzero(deg >= 2)[0][-10])
    # a duplicate early and a self-loop late: the duplicate's row comes first
    col = g.col.copy()
    col[rp[early] + 1] = col[rp[early]]
    col[rp[late]] = late
    with pytest.raises(P.PercisError, match="duplicate arc %d -> " % early) as e:
        c.load_csr(g.n, g.row_ptr, col, directed=True)
    assert e.value.status == P.E_INVAL
    # two out-of-range entries: the first index is named
    col = g.col.copy()
    col[g.m - 3] = g.n
    col[rp[early]] = -1
    with pytest.raises(P.PercisError, match=r"col\[%d\] = -1 out of range" % rp[early]):
        c.load_csr(g.n, g.row_ptr, col, directed=True)
    # an undirected graph with one reverse arc missing
    u = W.rmat_graph(19, 12, seed=8, directed=False)
    assert u.m > 8 << 20
    c.load_csr(u.n, u.row_ptr, u.col)
    ucol = u.col.copy()
    urp = u.row_ptr.astype(np.int64)
    v0 = int(np.nonzero(np.diff(urp) >= 3)[0][-5])
    x = int(ucol[urp[v0]])
    ucol[urp[v0]] = (x + 1) % u.n if (x + 1) % u.n != v0 else (x + 2) % u.n
    with pytest.raises(P.PercisError, match="lacks arc") as e:
        c.load_csr(u.n, u.row_ptr, ucol)
    assert e.value.status == P.E_INVAL
    c.close()
