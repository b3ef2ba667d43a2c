"""CPU oracle of the PercIS hot path -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. It wraps ``percis_oracle.c`` (plain,
single-threaded C) through ctypes and shares no code with the HIP library.
"""
from .oracle import (  # noqa: F401
    Graph, States, build, philox4x64_10, word, bounded, sample_range, path,
    exact, bounded128, SIGMA_SATURATED, vertex_diam_ub, estimate, estimate_di, sample_size, search_s, search_t, draw_pair,
    BidirWork,
)
