"""Helpers shared by the GPU tests: building library contexts and running the
oracle (threaded over disjoint sample ranges, whose hit counts add up)."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle as O


def gpu_context(g, k, slots=0):
    from paper_2509_11454_amd import percis as P
    c = P.Context(0)
    if slots:
        c.set_option(P.OPT_SLOTS, slots)
    c.load_csr(g.n, g.row_ptr, g.col, directed=g.directed)
    c.set_states(k)
    return c


def oracle_objects(g, k):
    return O.Graph(g.n, g.row_ptr, g.col, g.directed), O.States(k)


_WORK = []  # scratch of the oracle's bidirectional mode, one per thread


def oracle_work(parts, n):
    """`parts` bidirectional-search workspaces of at least n nodes, kept
    across calls (allocating and touching them costs more than thousands of
    samples on the largest graphs)."""
    global _WORK
    if len(_WORK) < parts or _WORK[0].n < n:
        _WORK = []
        _WORK = [O.BidirWork(n) for _ in range(parts)]
    return _WORK[:parts]


def release_oracle_work():
    global _WORK
    _WORK = []


def oracle_hits(og, st, first, count, seed, phase=0, threads=None, bidir=False):
    """Oracle hits and merged stats over [first, first+count); bidir runs the
    oracle's bidirectional search mode (the CPU tests prove it equal to the
    truncated BFS)."""
    threads = threads or min(16, os.cpu_count() or 1)
    parts = max(1, min(threads, count))
    bounds = [first + count * i // parts for i in range(parts + 1)]
    work = oracle_work(parts, og.n) if bidir else [None] * parts

    def job(i):
        return O.sample_range(og, st, bounds[i], bounds[i + 1] - bounds[i], seed, phase, bidir=bidir,
                              work=work[i])

    with ThreadPoolExecutor(parts) as ex:
        res = list(ex.map(job, range(parts)))
    hits = np.zeros(og.n, np.uint64)
    stats = {"samples": 0, "reachable": 0, "sum_I": 0, "sum_I2": 0, "overflow": 0,
             "first_overflow": 2 ** 64 - 1}
    for h, s in res:
        hits += h
        for key in ("samples", "reachable", "sum_I", "sum_I2", "overflow"):
            stats[key] += s[key]
        stats["first_overflow"] = min(stats["first_overflow"], s["first_overflow"])
    return hits.astype(np.uint32), stats


def gpu_hits(c, first, count, seed, phase=0, allow_overflow=False):
    h = np.zeros(c.n, np.uint32)
    _, st = c.sample_range(first, count, seed, phase, hits=h, allow_overflow=allow_overflow)
    return h, st


def same_stats(a, b):
    for key in ("samples", "reachable", "sum_I", "sum_I2", "overflow"):
        assert a[key] == b[key], (key, a[key], b[key])
    if a["overflow"]:
        assert a["first_overflow"] == b["first_overflow"]
