"""Python binding of libpercis (the C ABI in include/percis.h).

Argument marshalling only: every step of the sampler runs in the HIP
library. torch provides device memory (tensors whose data pointers are
passed with PERCIS_DEVICE_PTRS) and the stream (torch's current stream).
Importing this module fails loudly if the library has not been built.
"""
import ctypes as C
import os

import numpy as np
import torch  # loaded first: libpercis then binds to the same HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
# PERCIS_LIB_PATH names another build to load (the sanitizer run)
LIB_PATH = os.environ.get("PERCIS_LIB_PATH") or os.path.join(_HERE, "lib", "libpercis.so")

HOST_ONLY = -1
OK, E_INVAL, E_STATE, E_NOMEM, E_DEVICE, E_DEGENERATE, E_TOO_LARGE, E_SIGMA_OVERFLOW = 0, -1, -2, -3, -4, -5, -6, -7
DIRECTED, DEVICE_PTRS, ACCUMULATE = 0x1, 0x2, 0x4
OPT_SLOTS, OPT_SCRATCH_MB, OPT_BLOCK, OPT_BITMAPS, OPT_COMPACT, OPT_DEFER_BLOCK, OPT_PAIR_CHUNK = 1, 2, 3, 4, 5, 6, 7
OPT_BALANCE = 8

if not os.path.exists(LIB_PATH):
    raise ImportError("libpercis.so is not built (%s); run __graft_entry__.build() or "
                      "python -m paper_2509_11454_amd.build" % LIB_PATH)

_lib = C.CDLL(LIB_PATH)


class Stats(C.Structure):
    _fields_ = [("samples", C.c_uint64), ("reachable", C.c_uint64), ("sum_I", C.c_uint64),
                ("sum_I2", C.c_uint64), ("overflow", C.c_uint64), ("first_overflow", C.c_uint64),
                ("edges", C.c_uint64), ("sigma_adds", C.c_uint64), ("vertices_expanded", C.c_uint64),
                ("vertices_discovered", C.c_uint64), ("kernel_ms", C.c_double), ("phase_ms", C.c_double * 5),
                ("pair_ms", C.c_double), ("spilled", C.c_uint64), ("deferred", C.c_uint64),
                ("pass_ms", C.c_double * 2)]

    PHASES = ("start", "bfs", "dag", "walk", "clear")

    def to_dict(self):
        d = {}
        for k, t in self._fields_:
            if k == "phase_ms":
                d[k] = dict(zip(self.PHASES, [float(x) for x in self.phase_ms]))
            elif k == "pass_ms":
                d[k] = [float(x) for x in self.pass_ms]
            else:
                d[k] = float(getattr(self, k)) if t is C.c_double else int(getattr(self, k))
        return d


class EstimateInfo(C.Structure):
    _fields_ = [("l1", C.c_uint64), ("l", C.c_uint64), ("D", C.c_int64), ("d_hat", C.c_double),
                ("rho_tilde", C.c_double), ("Lambda", C.c_double), ("rho_hat", C.c_double),
                ("v_hat", C.c_double), ("x_hat", C.c_double), ("phase1_ms", C.c_double),
                ("bounds_ms", C.c_double), ("phase2_ms", C.c_double), ("total_ms", C.c_double),
                ("overflow", C.c_uint64)]

    def to_dict(self):
        return {k: (float(getattr(self, k)) if t is C.c_double else int(getattr(self, k)))
                for k, t in self._fields_}


class Task(C.Structure):
    _fields_ = [("graph", C.c_int32), ("phase", C.c_uint32), ("first", C.c_uint64), ("count", C.c_uint64),
                ("seed", C.c_uint64), ("hits", C.c_void_p), ("flags", C.c_uint32), ("stats", C.POINTER(Stats))]


class Tuning(C.Structure):
    _fields_ = [("block", C.c_int32), ("bitmaps", C.c_int32), ("slots", C.c_int32), ("candidates", C.c_int32),
                ("samples_per_s", C.c_double), ("compact", C.c_int32), ("balance", C.c_int32),
                ("defer_block", C.c_int32), ("auto_samples_per_s", C.c_double)]

    def to_dict(self):
        return {k: (float(getattr(self, k)) if t is C.c_double else int(getattr(self, k))) for k, t in self._fields_}


_P = C.c_void_p
_SIGS = {
    "percis_create": (C.c_int, [C.c_int, _P, C.POINTER(_P)]),
    "percis_destroy": (None, [_P]),
    "percis_set_stream": (C.c_int, [_P, _P]),
    "percis_load_csr": (C.c_int, [_P, C.c_int32, C.c_int64, _P, _P, C.c_uint32]),
    "percis_set_states": (C.c_int, [_P, _P, C.c_uint32]),
    "percis_sample_range": (C.c_int, [_P, C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint32, _P, C.c_uint32,
                                      C.POINTER(Stats)]),
    "percis_sample": (C.c_int, [_P, C.c_uint64, C.c_uint64, _P, C.c_uint32, C.POINTER(Stats)]),
    "percis_sample_range_noalloc": (C.c_int, [_P, C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint32, _P, C.c_uint32,
                                              C.POINTER(Stats)]),
    "percis_estimate": (C.c_int, [_P, C.c_double, C.c_double, C.c_uint64, _P, C.POINTER(EstimateInfo)]),
    "percis_set_vertex_diameter": (C.c_int, [_P, C.c_int64]),
    "percis_debug_path": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_uint64, _P, C.c_int32,
                                    C.POINTER(C.c_int32), C.POINTER(C.c_uint64), C.POINTER(C.c_int32)]),
    "percis_graph_vertex_diameter": (C.c_int, [_P, C.c_int32, _P]),
    "percis_debug_states": (C.c_int, [_P, C.c_int32, _P, _P, _P, _P, _P, _P, _P, _P]),
    "percis_debug_path_wide": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_uint64, C.c_uint64, _P, C.c_int32,
                                         C.POINTER(C.c_int32), C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                         C.POINTER(C.c_int32)]),
    "percis_add_graph": (C.c_int, [_P, C.c_int32, C.c_int64, _P, _P, _P, C.c_uint32, C.POINTER(C.c_int32)]),
    "percis_graph_info": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                    C.POINTER(C.c_int32)]),
    "percis_sample_tasks": (C.c_int, [_P, C.c_int32, C.POINTER(Task), C.POINTER(Stats)]),
    "percis_batch_capture": (C.c_int, [_P, C.c_int32, C.POINTER(Task), C.POINTER(_P)]),
    "percis_batch_replay": (C.c_int, [_P, C.POINTER(Stats)]),
    "percis_batch_destroy": (None, [_P]),
    "percis_graph_estimate": (C.c_int, [_P, C.c_int32, C.c_double, C.c_double, C.c_uint64, _P,
                                        C.POINTER(EstimateInfo)]),
    "percis_graph_estimate_di": (C.c_int, [_P, C.c_int32, C.c_double, C.c_double, C.c_uint64, _P,
                                           C.POINTER(EstimateInfo)]),
    "percis_graph_set_vertex_diameter": (C.c_int, [_P, C.c_int32, C.c_int64]),
    "percis_autotune": (C.c_int, [_P, C.c_int32, C.c_uint64, C.c_uint64, C.POINTER(Tuning)]),
    "percis_server_create": (C.c_int, [_P, C.c_int64, C.c_uint64, C.c_uint64, C.POINTER(_P)]),
    "percis_server_destroy": (None, [_P]),
    "percis_server_submit": (C.c_int, [_P, C.c_int32, C.c_double, C.c_double, C.c_uint64, C.POINTER(C.c_int64)]),
    "percis_server_step": (C.c_int, [_P, C.POINTER(C.c_int32)]),
    "percis_server_result": (C.c_int, [_P, C.c_int64, C.POINTER(C.c_int32), _P, C.c_int32,
                                       C.POINTER(EstimateInfo)]),
    "percis_server_status": (C.c_int, [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                       C.POINTER(C.c_int64), C.POINTER(C.c_uint64)]),
    "percis_exact": (C.c_int, [_P, C.c_int32, _P, C.POINTER(C.c_double)]),
    "percis_set_option": (C.c_int, [_P, C.c_int, C.c_int64]),
    "percis_get_option": (C.c_int, [_P, C.c_int, C.POINTER(C.c_int64)]),
    "percis_status_str": (C.c_char_p, [C.c_int]),
    "percis_last_error": (C.c_char_p, [_P]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_SIGS)


class PercisError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s (%d): %s" % (_lib.percis_status_str(status).decode(), status, message))
        self.status = status


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


class Context:
    """One library context on one device; owns the device copies of a graph,
    its states and the sampler scratch."""

    def __init__(self, device=0, stream=None):
        """device = HOST_ONLY gives a context that validates inputs and builds
        host-side structures but never touches a GPU."""
        self.device = int(device)
        h = C.c_void_p()
        if self.device == HOST_ONLY:
            self._stream = None
            rc = _lib.percis_create(HOST_ONLY, None, C.byref(h))
        else:
            if not torch.cuda.is_available():
                raise RuntimeError("no HIP device visible: the PercIS sampler runs on the GPU only")
            torch.cuda.set_device(self.device)
            if stream is None:
                stream = torch.cuda.current_stream(self.device)
            self._stream = stream
            rc = _lib.percis_create(self.device, C.c_void_p(stream.cuda_stream), C.byref(h))
        if rc != OK:
            raise PercisError(rc, "percis_create failed")
        self._h = h
        self.n = 0
        self.directed = False

    def close(self):
        if getattr(self, "_h", None):
            _lib.percis_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow=()):
        if rc != OK and rc not in allow:
            raise PercisError(rc, _lib.percis_last_error(self._h).decode())
        return rc

    def set_stream(self, stream):
        self._stream = stream
        return self._check(_lib.percis_set_stream(self._h, C.c_void_p(stream.cuda_stream)))

    def load_csr(self, n, row_ptr, col, directed=False):
        """row_ptr/col: numpy arrays (host) or int32 torch tensors on this device."""
        flags = DIRECTED if directed else 0
        if isinstance(row_ptr, torch.Tensor):
            assert row_ptr.is_cuda and col.is_cuda and row_ptr.dtype == torch.int32 and col.dtype == torch.int32
            rc = _lib.percis_load_csr(self._h, int(n), int(col.numel()), C.c_void_p(row_ptr.data_ptr()),
                                      C.c_void_p(col.data_ptr()), flags | DEVICE_PTRS)
        else:
            rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
            cl = np.ascontiguousarray(col, dtype=np.int32)
            rc = _lib.percis_load_csr(self._h, int(n), int(cl.size), _np_ptr(rp), _np_ptr(cl), flags)
        self._check(rc)
        self.n = int(n)
        self.directed = bool(directed)

    def set_states(self, k):
        if isinstance(k, torch.Tensor):
            assert k.is_cuda and k.dtype in (torch.int16, torch.uint16)
            return self._check(_lib.percis_set_states(self._h, C.c_void_p(k.data_ptr()), DEVICE_PTRS))
        kk = np.ascontiguousarray(k, dtype=np.uint16)
        return self._check(_lib.percis_set_states(self._h, _np_ptr(kk), 0))

    def sample_range(self, first, count, seed, phase=0, hits=None, accumulate=False, allow_overflow=False):
        """Returns (hits, stats dict). hits: None (a new int32 device tensor is
        returned, holding the uint32 counts), a torch int32 device tensor, or a
        numpy uint32 array (host)."""
        st = Stats()
        flags = ACCUMULATE if accumulate else 0
        if hits is None:
            hits = torch.zeros(self.n, dtype=torch.int32, device="cuda:%d" % self.device)
        if isinstance(hits, torch.Tensor):
            if hits.dtype != torch.int32 or hits.numel() < self.n:
                raise ValueError("hits must be an int32 tensor of at least %d entries" % self.n)
            if not hits.is_cuda or not hits.is_contiguous():
                raise ValueError("hits must be a contiguous device tensor")
            rc = _lib.percis_sample_range(self._h, int(first), int(count), int(seed), int(phase),
                                          C.c_void_p(hits.data_ptr()), flags | DEVICE_PTRS, C.byref(st))
        else:
            if hits.dtype != np.uint32 or hits.size < self.n or not hits.flags.c_contiguous:
                raise ValueError("hits must be a contiguous uint32 array of at least %d entries" % self.n)
            rc = _lib.percis_sample_range(self._h, int(first), int(count), int(seed), int(phase),
                                          _np_ptr(hits), flags, C.byref(st))
        self._check(rc, allow=(E_SIGMA_OVERFLOW,) if allow_overflow else ())
        return hits, st.to_dict()

    def sample_range_noalloc(self, first, count, seed, phase, hits, accumulate=False, allow_overflow=False):
        """percis_sample_range_noalloc: hits is an int32 device tensor of at
        least n entries; returns the stats dict."""
        if not isinstance(hits, torch.Tensor) or hits.dtype != torch.int32 or hits.numel() < self.n:
            raise ValueError("hits must be an int32 tensor of at least %d entries" % self.n)
        if not hits.is_cuda or not hits.is_contiguous():
            raise ValueError("hits must be a contiguous device tensor")
        st = Stats()
        flags = DEVICE_PTRS | (ACCUMULATE if accumulate else 0)
        rc = _lib.percis_sample_range_noalloc(self._h, int(first), int(count), int(seed), int(phase),
                                              C.c_void_p(hits.data_ptr()), flags, C.byref(st))
        self._check(rc, allow=(E_SIGMA_OVERFLOW,) if allow_overflow else ())
        return st.to_dict()

    def sample(self, n_samples, seed, hits=None):
        return self.sample_range(0, n_samples, seed, 0, hits)

    def estimate(self, eps, delta, seed):
        p = np.zeros(self.n, np.float64)
        info = EstimateInfo()
        self._check(_lib.percis_estimate(self._h, float(eps), float(delta), int(seed), _np_ptr(p), C.byref(info)))
        return p, info.to_dict()

    def set_vertex_diameter(self, D):
        return self._check(_lib.percis_set_vertex_diameter(self._h, int(D)))

    def debug_path(self, s, t, r, cap=None):
        cap = self.n + 1 if cap is None else cap
        buf = np.zeros(max(cap, 1), np.int32)
        L, sig, ovf = C.c_int32(), C.c_uint64(), C.c_int32()
        self._check(_lib.percis_debug_path(self._h, int(s), int(t), int(r), _np_ptr(buf), int(cap),
                                           C.byref(L), C.byref(sig), C.byref(ovf)))
        L, sig, ovf = int(L.value), int(sig.value), int(ovf.value)
        path = [int(v) for v in buf[:L + 1]] if (L >= 0 and not ovf and r < sig and L + 1 <= cap) else None
        return L, sig, ovf, path

    def debug_path_wide(self, s, t, r, cap=None):
        """The 128-bit path for (s, t, r): returns (L, sigma, overflow, path)
        with r and sigma Python ints."""
        cap = self.n + 1 if cap is None else cap
        buf = np.zeros(max(cap, 1), np.int32)
        L, lo, hi, ovf = C.c_int32(), C.c_uint64(), C.c_uint64(), C.c_int32()
        self._check(_lib.percis_debug_path_wide(self._h, int(s), int(t), int(r) & ((1 << 64) - 1), int(r) >> 64,
                                                _np_ptr(buf), int(cap), C.byref(L), C.byref(lo), C.byref(hi),
                                                C.byref(ovf)))
        L, sig, ovf = int(L.value), (int(hi.value) << 64) | int(lo.value), int(ovf.value)
        path = [int(v) for v in buf[:L + 1]] if (L >= 0 and not ovf and r < sig and L + 1 <= cap) else None
        return L, sig, ovf, path

    def vertex_diameter(self, graph=0):
        """VertexDiamUB of graph `graph` (the override if set, else the
        device-computed bound)."""
        D = C.c_int64()
        self._check(_lib.percis_graph_vertex_diameter(self._h, int(graph), C.byref(D)))
        return int(D.value)

    def debug_states(self, graph=0):
        """The device-built pair distribution of graph `graph` as numpy arrays:
        perm (caller ids), kr, W, P, d_v, S_v, and the scalars C, d_hat."""
        n = self.graph_info(graph)[0]
        perm = np.zeros(n + 1, np.int32)
        kr = np.zeros(n + 2, np.uint32)
        W = np.zeros(n + 2, np.uint64)
        P = np.zeros(n + 1, np.uint64)
        dv = np.zeros(n, np.float64)
        Sv = np.zeros(n, np.float64)
        Cv, dh = C.c_uint64(), C.c_double()
        self._check(_lib.percis_debug_states(self._h, int(graph), _np_ptr(perm), _np_ptr(kr), _np_ptr(W), _np_ptr(P),
                                             _np_ptr(dv), _np_ptr(Sv), C.byref(Cv), C.byref(dh)))
        return dict(perm=perm, kr=kr, W=W, P=P, d_v=dv, S_v=Sv, C=int(Cv.value), d_hat=float(dh.value))

    def add_graph(self, n, row_ptr, col, k, directed=False):
        """Adds a graph with its states; returns its id."""
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        kk = np.ascontiguousarray(k, dtype=np.uint16)
        gid = C.c_int32()
        self._check(_lib.percis_add_graph(self._h, int(n), int(cl.size), _np_ptr(rp), _np_ptr(cl), _np_ptr(kk),
                                          DIRECTED if directed else 0, C.byref(gid)))
        return int(gid.value)

    def graph_info(self, graph):
        n, m, na = C.c_int32(), C.c_int64(), C.c_int32()
        self._check(_lib.percis_graph_info(self._h, int(graph), C.byref(n), C.byref(m), C.byref(na)))
        return int(n.value), int(m.value), int(na.value)

    def _task_table(self, tasks):
        """The C task table of `tasks` and their stats records. Each task's
        hits must be an int32 device tensor of at least its graph's node
        count: the library receives a bare pointer and writes that many
        entries (checked before any launch)."""
        arr = (Task * len(tasks))()
        sts = [Stats() for _ in tasks]
        for i, t in enumerate(tasks):
            h = t["hits"]
            if not isinstance(h, torch.Tensor) or h.dtype != torch.int32:
                raise TypeError("task %d: hits must be an int32 torch tensor" % i)
            n = self.graph_info(int(t["graph"]))[0]
            if h.numel() < n:
                raise ValueError("task %d: hits holds %d entries, graph %d has %d nodes" % (i, h.numel(), t["graph"], n))
            if not h.is_cuda or not h.is_contiguous():
                raise ValueError("task %d: hits must be a contiguous device tensor" % i)
            arr[i] = Task(int(t["graph"]), int(t.get("phase", 0)), int(t.get("first", 0)), int(t["count"]),
                          int(t["seed"]), C.c_void_p(h.data_ptr()), ACCUMULATE if t.get("accumulate") else 0,
                          C.pointer(sts[i]))
        return arr, sts

    def sample_tasks(self, tasks, allow_overflow=False):
        """tasks: list of dicts with graph, first, count, seed, phase, hits
        (int32 device tensor), accumulate. Returns (per-task stats, launch stats)."""
        arr, sts = self._task_table(tasks)
        ls = Stats()
        rc = _lib.percis_sample_tasks(self._h, len(tasks), arr, C.byref(ls))
        self._check(rc, allow=(E_SIGMA_OVERFLOW,) if allow_overflow else ())
        return [s.to_dict() for s in sts], ls.to_dict()

    def capture_batch(self, tasks):
        """The launch of sample_tasks(tasks) captured as a HIP graph; returns a
        Batch whose replay() re-runs it."""
        arr, sts = self._task_table(tasks)
        b = _P()
        self._check(_lib.percis_batch_capture(self._h, len(tasks), arr, C.byref(b)))
        return Batch(self, b, sts, [t["hits"] for t in tasks])

    def graph_estimate(self, graph, eps, delta, seed):
        n = self.graph_info(graph)[0]
        p = np.zeros(n, np.float64)
        info = EstimateInfo()
        self._check(_lib.percis_graph_estimate(self._h, int(graph), float(eps), float(delta), int(seed), _np_ptr(p),
                                               C.byref(info)))
        return p, info.to_dict()

    def graph_estimate_di(self, graph, eps, delta, seed):
        """PercIS-DI on graph `graph` (no first phase; data-independent bound)."""
        n = self.graph_info(graph)[0]
        p = np.zeros(n, np.float64)
        info = EstimateInfo()
        self._check(_lib.percis_graph_estimate_di(self._h, int(graph), float(eps), float(delta), int(seed),
                                                  _np_ptr(p), C.byref(info)))
        return p, info.to_dict()

    def graph_set_vertex_diameter(self, graph, D):
        return self._check(_lib.percis_graph_set_vertex_diameter(self._h, int(graph), int(D)))

    def exact(self, graph=0):
        """Exact percolation centrality on the device; returns (p, kernel ms)."""
        n = self.graph_info(graph)[0]
        p = np.zeros(n, np.float64)
        ms = C.c_double()
        self._check(_lib.percis_exact(self._h, int(graph), _np_ptr(p), C.byref(ms)))
        return p, float(ms.value)

    def autotune(self, graph=0, probe_samples=20000, seed=12345):
        t = Tuning()
        self._check(_lib.percis_autotune(self._h, int(graph), int(probe_samples), int(seed), C.byref(t)))
        return t.to_dict()

    def set_option(self, opt, value):
        return self._check(_lib.percis_set_option(self._h, int(opt), int(value)))

    def get_option(self, opt):
        v = C.c_int64()
        self._check(_lib.percis_get_option(self._h, int(opt), C.byref(v)))
        return int(v.value)


class Batch:
    """A captured task launch (percis_batch_*)."""

    def __init__(self, ctx, handle, stats, hits):
        self._ctx, self._h, self._stats, self._hits = ctx, handle, stats, hits

    def replay(self, allow_overflow=False):
        """Returns (per-task stats, launch stats), as Context.sample_tasks."""
        ls = Stats()
        rc = _lib.percis_batch_replay(self._h, C.byref(ls))
        self._ctx._check(rc, allow=(E_SIGMA_OVERFLOW,) if allow_overflow else ())
        return [s.to_dict() for s in self._stats], ls.to_dict()

    def close(self):
        if self._h:
            _lib.percis_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            self.close()


class Server:
    """Continuous-batching query server over the graphs of a Context."""

    def __init__(self, ctx, memory_budget_bytes, chunk_samples=8192, step_samples=262144):
        self.ctx = ctx
        h = C.c_void_p()
        ctx._check(_lib.percis_server_create(ctx._h, int(memory_budget_bytes), int(chunk_samples),
                                             int(step_samples), C.byref(h)))
        self._h = h
        self._n = {}

    def close(self):
        if getattr(self, "_h", None):
            _lib.percis_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, graph, eps, delta, seed):
        qid = C.c_int64()
        self.ctx._check(_lib.percis_server_submit(self._h, int(graph), float(eps), float(delta), int(seed),
                                                  C.byref(qid)))
        self._n[int(qid.value)] = self.ctx.graph_info(graph)[0]
        return int(qid.value)

    def step(self):
        done = C.c_int32()
        self.ctx._check(_lib.percis_server_step(self._h, C.byref(done)))
        return int(done.value)

    def result(self, qid):
        """None while running; else (status, p or None, info dict)."""
        n = self._n[qid]
        p = np.zeros(n, np.float64)
        done = C.c_int32()
        info = EstimateInfo()
        rc = _lib.percis_server_result(self._h, int(qid), C.byref(done), _np_ptr(p), n, C.byref(info))
        if not done.value:
            if rc != OK:
                self.ctx._check(rc)
            return None
        del self._n[qid]
        return rc, (p if rc == OK else None), info.to_dict()

    def status(self):
        q, a, b, pk, sd = C.c_int32(), C.c_int32(), C.c_int64(), C.c_int64(), C.c_uint64()
        self.ctx._check(_lib.percis_server_status(self._h, C.byref(q), C.byref(a), C.byref(b), C.byref(pk),
                                                  C.byref(sd)))
        return dict(queued=int(q.value), active=int(a.value), bytes_in_use=int(b.value), peak_bytes=int(pk.value),
                    samples_done=int(sd.value))


def raw_library():
    return _lib
