"""ctypes wrapper of the C oracle (test infrastructure only).

Every function here only marshals arguments; the arithmetic lives in
``percis_oracle.c``, whose header names the passage of the paper each
function follows.
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "percis_oracle.c")
# PERCIS_ORACLE_LIB names a prebuilt copy to load instead (the sanitizer run)
_LIB = os.environ.get("PERCIS_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force=True, sanitize=False, out=None):
    """Compile the oracle with gcc into oracle/liboracle.so; sanitize=True
    builds a copy at `out` with clang's AddressSanitizer and
    UndefinedBehaviorSanitizer (one runtime with the library's host code)."""
    lib = out or _LIB
    if not sanitize and not force and os.path.exists(lib) and os.path.getmtime(lib) >= os.path.getmtime(_SRC):
        return lib
    tmp = lib + ".tmp%d" % os.getpid()
    cc = ["/opt/rocm/llvm/bin/clang", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
          "-fno-sanitize-recover=undefined"] if sanitize else ["gcc"]
    subprocess.check_call(cc + ["-O2", "-std=c11", "-shared", "-fPIC", "-Wall", "-Wextra",
                                "-Wno-unused-parameter", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, lib)
    return lib


class _Stats(C.Structure):
    _fields_ = [("samples", C.c_uint64), ("reachable", C.c_uint64), ("sum_I", C.c_uint64),
                ("sum_I2", C.c_uint64), ("overflow", C.c_uint64), ("first_overflow", C.c_uint64),
                ("edges", C.c_uint64)]

    def to_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class _EstInfo(C.Structure):
    _fields_ = [("l1", C.c_uint64), ("l", C.c_uint64), ("D", C.c_int64), ("d_hat", C.c_double),
                ("rho_tilde", C.c_double), ("Lambda", C.c_double), ("rho_hat", C.c_double),
                ("v_hat", C.c_double), ("x_hat", C.c_double), ("overflow", C.c_uint64)]

    def to_dict(self):
        return {k: (float(getattr(self, k)) if t is C.c_double else int(getattr(self, k)))
                for k, t in self._fields_}


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = C.CDLL(_LIB)
    P = C.c_void_p
    u64, i64, i32 = C.c_uint64, C.c_int64, C.c_int32
    sig = {
        "orc_philox4x64_10": (None, [P, P, P]),
        "orc_word": (u64, [u64, u64, u64, u64, u64]),
        "orc_bounded": (u64, [u64, u64, u64, u64, u64, P]),
        "orc_graph_new": (P, [i32, i64, P, P, C.c_int]),
        "orc_graph_free": (None, [P]),
        "orc_states_new": (P, [i32, P]),
        "orc_states_free": (None, [P]),
        "orc_states_total": (u64, [P]),
        "orc_states_arrays": (None, [P, P, P, P, P, P, P]),
        "orc_search_s": (None, [P, u64, P]),
        "orc_search_t": (None, [P, i32, u64, P]),
        "orc_draw_pair": (None, [P, u64, u64, u64, P, P, P, P]),
        "orc_path": (i32, [P, i32, i32, u64, P, i32, P, P]),
        "orc_path128": (i32, [P, i32, i32, u64, u64, P, i32, P, P]),
        "orc_bounded128_parts": (None, [u64, u64, u64, u64, u64, u64, P, P, P]),
        "orc_sample_range": (None, [P, P, u64, u64, u64, u64, P, P, P]),
        "orc_sample_range_bidir": (None, [P, P, u64, u64, u64, u64, P, P, P, P]),
        "orc_bidir_work_new": (P, [i32]),
        "orc_bidir_work_free": (None, [P]),
        "orc_path_bidir128": (i32, [P, i32, i32, u64, u64, P, i32, P, P]),
        "orc_exact": (None, [P, P, P]),
        "orc_vertex_diam_ub": (i64, [P]),
        "orc_sample_size": (C.c_double, [C.c_double] * 5 + [P]),
        "orc_estimate": (C.c_int, [P, P, C.c_double, C.c_double, u64, i64, P, P]),
        "orc_estimate_di": (C.c_int, [P, P, C.c_double, C.c_double, u64, i64, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def philox4x64_10(ctr, key):
    lib = _load()
    c = np.asarray(ctr, dtype=np.uint64).copy()
    k = np.asarray(key, dtype=np.uint64).copy()
    out = np.zeros(4, dtype=np.uint64)
    lib.orc_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def word(seed, phase, idx, variate, attempt):
    return int(_load().orc_word(seed, phase, idx, variate, attempt))


def bounded(seed, phase, idx, variate, N):
    used = C.c_uint64(0)
    v = int(_load().orc_bounded(seed, phase, idx, variate, N, C.byref(used)))
    return v, int(used.value)


class Graph:
    """Oracle graph: copies a CSR (row_ptr[n+1] int, col[m] int32)."""

    def __init__(self, n, row_ptr, col, directed=False):
        lib = _load()
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        self.n = int(n)
        self.m = int(cl.size)
        self.directed = bool(directed)
        self._h = lib.orc_graph_new(self.n, self.m, _ptr(rp), _ptr(cl), int(directed))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_graph_free(self._h)
            self._h = None


class States:
    """Oracle states (k_v in 0..65535) and the preprocessing of Algorithm 2."""

    def __init__(self, k):
        lib = _load()
        self.k = np.ascontiguousarray(k, dtype=np.uint16)
        self.n = int(self.k.size)
        self._h = lib.orc_states_new(self.n, _ptr(self.k))
        self.C = int(lib.orc_states_total(self._h))

    def arrays(self):
        n = self.n
        perm = np.zeros(n + 2, np.int32)
        x, w, c, r = (np.zeros(n + 2, np.uint64) for _ in range(4))
        S = np.zeros(n, np.float64)
        _lib.orc_states_arrays(self._h, _ptr(perm), _ptr(x), _ptr(w), _ptr(c), _ptr(r), _ptr(S))
        return dict(perm=perm, x=x, w=w, c=c, r=r, S=S, C=self.C)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_states_free(self._h)
            self._h = None


def search_s(st, U):
    out = C.c_int32(0)
    _load().orc_search_s(st._h, U, C.byref(out))
    return int(out.value)


def search_t(st, s_rank, U):
    out = C.c_int32(0)
    _load().orc_search_t(st._h, s_rank, U, C.byref(out))
    return int(out.value)


def draw_pair(st, seed, phase, idx):
    s, t, sr, tr = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    _load().orc_draw_pair(st._h, seed, phase, idx, C.byref(s), C.byref(t), C.byref(sr), C.byref(tr))
    return int(s.value), int(t.value), int(sr.value), int(tr.value)


SIGMA_SATURATED = (1 << 128) - 1


def path(g, s, t, r=0, bidir=False):
    """Returns (L, sigma, path) with path = [s, ..., t] or None; r and sigma
    are Python ints (sigma saturates at 2^128 - 1, which means overflow).
    bidir: through the balanced bidirectional search instead of the
    truncated BFS (the same result)."""
    buf = np.zeros(g.n + 1, np.int32)
    lo, hi = C.c_uint64(0), C.c_uint64(0)
    fn = _load().orc_path_bidir128 if bidir else _load().orc_path128
    L = int(fn(g._h, s, t, r & ((1 << 64) - 1), r >> 64, _ptr(buf), g.n + 1, C.byref(lo), C.byref(hi)))
    sigma = (int(hi.value) << 64) | int(lo.value)
    p = None
    if L >= 0 and sigma < SIGMA_SATURATED and r < sigma:
        p = [int(v) for v in buf[:L + 1]]
    return L, sigma, p


def bounded128(seed, phase, idx, variate, N):
    """Uniform integer in [0, N) for 2^64 <= N < 2^128 (Lemire at 128 bits);
    returns (value, attempts)."""
    lo, hi, used = C.c_uint64(0), C.c_uint64(0), C.c_uint64(0)
    _load().orc_bounded128_parts(seed, phase, idx, variate, N & ((1 << 64) - 1), N >> 64,
                                 C.byref(lo), C.byref(hi), C.byref(used))
    return (int(hi.value) << 64) | int(lo.value), int(used.value)


class BidirWork:
    """Scratch of the bidirectional search for graphs of up to n nodes; one
    thread uses it at a time. Reusing it across sample ranges saves
    allocating and touching about 70 bytes per node for every range."""

    def __init__(self, n):
        self.n = int(n)
        self._h = _load().orc_bidir_work_new(self.n)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_bidir_work_free(self._h)
            self._h = None


def sample_range(g, st, first, count, seed, phase=0, with_I=False, bidir=False, work=None):
    """Returns (hits uint32[n], stats dict[, I int32[count]]). bidir: each
    sample's path through the balanced bidirectional search instead of the
    truncated BFS (the same results, much faster on large graphs); work: a
    BidirWork of at least g.n nodes to run it in."""
    lib = _load()
    hits = np.zeros(g.n, np.uint32)
    S = _Stats()
    I = np.zeros(max(count, 1), np.int32) if with_I else None
    if bidir:
        assert work is None or work.n >= g.n
        lib.orc_sample_range_bidir(g._h, st._h, first, count, seed, phase, _ptr(hits), C.byref(S),
                                   _ptr(I) if with_I else None, work._h if work is not None else None)
    else:
        lib.orc_sample_range(g._h, st._h, first, count, seed, phase, _ptr(hits), C.byref(S),
                             _ptr(I) if with_I else None)
    if with_I:
        return hits, S.to_dict(), I[:count]
    return hits, S.to_dict()


def exact(g, st):
    p = np.zeros(g.n, np.float64)
    _load().orc_exact(g._h, st._h, _ptr(p))
    return p


def vertex_diam_ub(g):
    return int(_load().orc_vertex_diam_ub(g._h))


def sample_size(d_hat, rho_hat, v_hat, eps, delta):
    xh = C.c_double(0)
    v = float(_load().orc_sample_size(d_hat, rho_hat, v_hat, eps, delta, C.byref(xh)))
    return v, float(xh.value)


def estimate(g, st, eps, delta, seed, D=-1):
    """Algorithm 1. Returns (status, p[n], info dict)."""
    p = np.zeros(g.n, np.float64)
    info = _EstInfo()
    rc = int(_load().orc_estimate(g._h, st._h, eps, delta, seed, D, _ptr(p), C.byref(info)))
    return rc, p, info.to_dict()


def estimate_di(g, st, eps, delta, seed, D=-1):
    """PercIS-DI (no first phase, rho_hat = D, v_hat = d_hat^2/4). Returns
    (status, p[n], info dict)."""
    p = np.zeros(g.n, np.float64)
    info = _EstInfo()
    rc = int(_load().orc_estimate_di(g._h, st._h, eps, delta, seed, D, _ptr(p), C.byref(info)))
    return rc, p, info.to_dict()
