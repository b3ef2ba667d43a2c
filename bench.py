#!/usr/bin/env python3
"""PercIS hot-path benchmark on one MI355X.

One step = one call of the sampler over the workload's full batch of samples
(pair draw, bidirectional shortest-path-counting BFS, canonical path, hits)
with the graph, the pair distribution and the hit buffer resident in HBM.
The default workload is the largest one that fits one GPU: directed R-MAT
scale 24 (16.8M nodes, 263M arcs) with Beta(1/2, 1/2) states, 10^7 samples
per step.
Prints one JSON line: sampled s-t paths per second (value), GTEPS, the
roofline of the sampler kernel (algorithmic bytes / kernel time against the
8 TB/s HBM peak), the CPU oracle timed on the host, and the time to an
(eps = 0.01, delta = 0.1) estimate.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sampled s-t paths/sec + GTEPS and HBM GB/s vs peak; time-to-ε=0.01 estimate"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (builder, samples per step, description)
    "rmat18": ("workload_rmat18", 1_000_000,
               "R-MAT scale 18 undirected (a=0.57, b=c=0.19), edge factor 16; 95% of states 0, rest uniform"),
    "er1000": ("workload_er1000", 10_000, "Erdos-Renyi G(1000, 5000) undirected; uniform states"),
    "rmat24d": ("workload_rmat24_directed", 10_000_000,
                "R-MAT scale 24 directed (a=0.57, b=c=0.19), edge factor 16; states Beta(1/2, 1/2)"),
}


def kernel_source_hash():
    """Hash of the sampler's source (percis_kernels.hip, percis_internal.h)
    with comments and whitespace removed: a comment edit keeps the committed
    counters valid, a code edit does not."""
    h = hashlib.sha256()
    for f in ("percis_kernels.hip", "percis_internal.h"):
        with open(os.path.join(ROOT, "paper_2509_11454_amd", "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def algorithmic_bytes(st):
    """Bytes the method must move for the counted work: per adjacency entry
    its column id and the neighbour's level word (4 + 4), per shortest-path
    accumulation a 64-bit read-modify-write (16), per expanded vertex its row
    bounds, its count and its queue slot (24), per discovered vertex its level
    write and queue append (8), per hit a 32-bit read-modify-write (8)."""
    return (8 * st["edges"] + 16 * st["sigma_adds"] + 24 * st["vertices_expanded"]
            + 8 * st["vertices_discovered"] + 8 * st["sum_I"])


def measured_traffic(workload, samples):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "sampler_%s_traffic.json" % workload)
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except ValueError:
        return None
    if d.get("kernel_source_hash") != kernel_source_hash() or d.get("samples_per_launch") != samples:
        return None
    return d.get("bytes_per_launch")


def oracle_threads():
    """Threads for the oracle: the CPUs this process may run on, at most 16
    (a GPU server's host share for one GPU); and the CPUs the host has."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return max(1, min(16, avail)), os.cpu_count() or avail


def cpu_baseline(og, st, seed, budget_s, threads, bidir=True, cap=5_000_000):
    """The oracle as it is, on host cores: disjoint windows of the same sample
    stream in parallel threads (ctypes releases the GIL), grown until about
    budget_s of work. bidir: the oracle's bidirectional search mode (each
    thread keeps one workspace, first touched by an untimed window of 8
    samples), else its truncated BFS."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle as O
    work = [O.BidirWork(og.n) for _ in range(threads)] if bidir else [None] * threads
    if bidir:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(lambda i: O.sample_range(og, st, 10 ** 12 + 8 * i, 8, seed, 0, bidir=True, work=work[i]),
                        range(threads)))
    per = 8
    total = 0
    elapsed = 0.0
    while True:
        t0 = time.perf_counter()
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(lambda i: O.sample_range(og, st, total + i * per, per, seed, 0, bidir=bidir, work=work[i]),
                        range(threads)))
        dt = time.perf_counter() - t0
        total += per * threads
        elapsed += dt
        if elapsed >= budget_s or total >= cap:
            break
        per = max(per, int(per * min(8.0, max(1.5, (budget_s - elapsed) / max(dt, 1e-3)))))
    del work
    mode = "bidirectional search" if bidir else "truncated BFS"
    return {"value": total / elapsed, "unit": "samples/s", "cores": threads, "kind": "oracle",
            "sample": "first %d sample indices of the same stream (seed %d), %d threads over disjoint windows, "
                      "oracle's %s, %.1f s" % (total, seed, threads, mode, elapsed)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=6)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat24d", choices=sorted(WORKLOADS))
    ap.add_argument("--samples", type=int, default=0, help="samples per step (default: the workload's)")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--slots", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--bitmaps", type=int, default=0,
                    help="visited sets: 0 auto, 1 device bitmaps, 2 LDS hash tables")
    ap.add_argument("--compact", type=int, default=0,
                    help="compact slots: 0 auto, 1 off, 2 on (samples outgrowing them go to per-node slots)")
    ap.add_argument("--scratch-mb", type=int, default=0, help="cap on the sampler scratch (0 = the library's default)")
    ap.add_argument("--defer-block", type=int, default=0,
                    help="threads per sample of the per-node slots while compact slots are on (0 auto)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-estimate", action="store_true")
    ap.add_argument("--one-per-launch", type=int, default=2000, metavar="N",
                    help="also time N samples drawn one per launch (0 = skip)")
    ap.add_argument("--mode", default="single", choices=["single", "batch", "serve", "setup"],
                    help="single: one graph (default); batch: 64 BA graphs in one launch; serve: query stream; "
                         "setup: state-only updates and VertexDiamUB on the device")
    ap.add_argument("--queries", type=int, default=120, help="serve: queries per load level")
    ap.add_argument("--serve-chunk", type=int, default=65536, help="serve: samples per query per launch")
    ap.add_argument("--serve-step", type=int, default=524288, help="serve: samples per launch")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (reference for HBM counters)")
    args = ap.parse_args()

    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.mode == "batch":
        run_batch(args)
        return
    if args.mode == "serve":
        run_serve(args)
        return
    if args.mode == "setup":
        run_setup(args)
        return

    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (samples would be sharded by index "
              "range with one integer all-reduce of the hit counts); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as W
    from paper_2509_11454_amd import percis as P

    builder, default_samples, desc = WORKLOADS[args.workload]
    samples = args.samples or default_samples
    t0 = time.perf_counter()
    g, k = getattr(W, builder)(args.seed)
    gen_s = time.perf_counter() - t0
    print("[bench] workload %s: n=%d m=%d (%s), generated in %.1f s" % (args.workload, g.n, g.m, desc, gen_s),
          file=sys.stderr, flush=True)

    c = P.Context(0)
    c.set_option(P.OPT_SLOTS, args.slots)
    c.set_option(P.OPT_BLOCK, args.block)
    c.set_option(P.OPT_BITMAPS, args.bitmaps)
    c.set_option(P.OPT_COMPACT, args.compact)
    if args.scratch_mb:
        c.set_option(P.OPT_SCRATCH_MB, args.scratch_mb)
    c.set_option(P.OPT_DEFER_BLOCK, args.defer_block)
    c.load_csr(g.n, g.row_ptr, g.col, directed=g.directed)
    c.set_states(k)
    hits = torch.zeros(g.n, dtype=torch.int32, device="cuda")
    for i in range(args.warmup):
        _, st = c.sample_range(0, samples, args.seed, 0, hits=hits)
        print("[bench] warmup %d: %.1f ms" % (i, st["kernel_ms"]), file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    totals = dict(edges=0, sigma_adds=0, vertices_expanded=0, vertices_discovered=0, sum_I=0, reachable=0, spilled=0,
                  deferred=0)
    phases = {}
    kernel_ms = []
    pair_ms = []
    pass_ms = [0.0, 0.0]
    t_start = time.perf_counter()
    for i in range(args.steps):
        _, st = c.sample_range(0, samples, args.seed, 0, hits=hits)
        for key in totals:
            totals[key] += st[key]
        for key, v in st["phase_ms"].items():
            phases[key] = phases.get(key, 0.0) + v
        kernel_ms.append(st["kernel_ms"])
        pair_ms.append(st["pair_ms"])
        pass_ms = [a + b for a, b in zip(pass_ms, st["pass_ms"])]
        print("[bench] step %d: sampler %.1f ms (passes %.1f + %.1f), pairs %.2f ms"
              % (i, st["kernel_ms"], st["pass_ms"][0], st["pass_ms"][1], st["pair_ms"]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start

    value = samples * args.steps / elapsed
    avg_kernel_s = sum(kernel_ms) / len(kernel_ms) / 1e3
    per_launch = {key: v // args.steps for key, v in totals.items()}
    b_alg = algorithmic_bytes(per_launch)
    achieved = b_alg / avg_kernel_s / 1e9
    traffic = measured_traffic(args.workload, samples)
    slots = c.get_option(P.OPT_SLOTS)
    block = c.get_option(P.OPT_BLOCK)
    bitmaps = "lds tables" if c.get_option(P.OPT_BITMAPS) == 2 else "device bitmaps"

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "%s: %s" % (args.workload, desc), "n": g.n, "m_arcs": g.m,
                   "samples_per_step": samples, "seed": args.seed, "slots": slots,
                   "threads_per_sample": block, "visited_sets": bitmaps,
                   "compact_slots": c.get_option(P.OPT_COMPACT) == 2},
        "gteps": totals["edges"] / elapsed / 1e9,
        "edges_per_sample": totals["edges"] / (samples * args.steps),
        "per_sample": {key: totals[key] / (samples * args.steps)
                       for key in ("sigma_adds", "vertices_expanded", "vertices_discovered", "sum_I")},
        "reachable_fraction": totals["reachable"] / (samples * args.steps),
        "spilled_fraction": totals["spilled"] / (samples * args.steps),
        "deferred_fraction": totals["deferred"] / (samples * args.steps),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "sampler_kernel", "kernel_ms": avg_kernel_s * 1e3,
                     "pass_ms": [v / args.steps for v in pass_ms],
                     "passes": ("compact slots, then per-node slots for the samples handed on"
                                if c.get_option(P.OPT_COMPACT) == 2 else "per-node slots"),
                     "pair_kernel_ms": sum(pair_ms) / len(pair_ms),
                     "algorithmic_bytes_per_launch": b_alg},
        "hbm_gbs_measured": (traffic / avg_kernel_s / 1e9) if traffic else None,
    }
    if traffic:
        out["hbm_frac_measured"] = out["hbm_gbs_measured"] / HBM_PEAK_GBS

    ptot = sum(phases.values())
    if ptot > 0:
        out["phase_split"] = {key: v / ptot for key, v in phases.items()}

    if args.one_per_launch:
        h1 = torch.zeros(g.n, dtype=torch.int32, device="cuda")
        c.sample_range(0, 1, args.seed, 0, hits=h1)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for i in range(args.one_per_launch):
            c.sample_range(i, 1, args.seed, 0, hits=h1, accumulate=i > 0)
        torch.cuda.synchronize()
        dt1 = time.perf_counter() - t1
        out["one_sample_per_launch"] = {"value": args.one_per_launch / dt1, "unit": "samples/s",
                                        "samples": args.one_per_launch,
                                        "form": "one percis_sample_range call (one kernel launch) per sample"}
        out["speedup_vs_one_per_launch"] = value / out["one_sample_per_launch"]["value"]
        print("[bench] one sample per launch: %.1f samples/s" % out["one_sample_per_launch"]["value"],
              file=sys.stderr, flush=True)

    if not args.no_estimate:
        p, info = c.estimate(0.01, 0.1, args.seed)
        # again with another seed: VertexDiamUB is cached from the first call
        _, again = c.estimate(0.01, 0.1, args.seed + 1)
        out["time_to_eps"] = {"eps": 0.01, "delta": 0.1, "wall_ms": info["total_ms"], "l1": info["l1"],
                              "l": info["l"], "D": info["D"], "d_hat": info["d_hat"], "rho_hat": info["rho_hat"],
                              "v_hat": info["v_hat"],
                              "phase1_ms": info["phase1_ms"], "bounds_ms": info["bounds_ms"],
                              "phase2_ms": info["phase2_ms"],
                              "second_call_ms": again["total_ms"],
                              "predicted_ms": (info["l1"] + info["l"]) / value * 1e3}
        print("[bench] estimate: l1=%d l=%d in %.1f ms" % (info["l1"], info["l"], info["total_ms"]),
              file=sys.stderr, flush=True)

    if not args.no_cpu_baseline:
        import oracle as O
        threads, host_cpus = oracle_threads()
        og, ost = O.Graph(g.n, g.row_ptr, g.col, g.directed), O.States(k)
        out["cpu_baseline"] = cpu_baseline(og, ost, args.seed, args.cpu_seconds, threads)
        out["cpu_baseline"]["host"] = host_cpu_model()
        out["cpu_baseline"]["host_cpus"] = host_cpus
        one = cpu_baseline(og, ost, args.seed, min(4.0, args.cpu_seconds / 4), 1)
        out["cpu_baseline"]["one_thread"] = {"value": one["value"], "sample": one["sample"]}
        trunc = cpu_baseline(og, ost, args.seed, min(5.0, args.cpu_seconds / 3), threads, bidir=False)
        out["cpu_baseline"]["truncated_bfs"] = {"value": trunc["value"], "sample": trunc["sample"]}
        print("[bench] cpu baseline: %.1f samples/s (%d threads; truncated BFS %.1f)"
              % (out["cpu_baseline"]["value"], threads, trunc["value"]), file=sys.stderr, flush=True)

    print(json.dumps(out), flush=True)


def run_batch(args):
    """64 Barabasi-Albert graphs (m = 4, n log-uniform in [1e4, 1e6], own
    uniform states) with 1e5 samples each: one autotuned launch over all
    graphs, captured as a HIP graph and replayed (the headline value), beside
    the same launch issued eagerly, 64 per-graph launches and one sample per
    launch. The autotuner's probe is a launch of 2e5 samples spread over all
    64 graphs (untimed set-up)."""
    import torch
    import workloads as W
    from paper_2509_11454_amd import percis as P

    per_graph = args.samples or 100_000
    t0 = time.perf_counter()
    graphs = W.workload_ba_batch(64, 4, args.seed)
    print("[bench] 64 BA graphs: %d nodes, %d arcs in %.1f s" % (sum(g.n for g, _ in graphs),
                                                                    sum(g.m for g, _ in graphs),
                                                                    time.perf_counter() - t0),
          file=sys.stderr, flush=True)
    c = P.Context(0)
    g0, k0 = graphs[0]
    c.load_csr(g0.n, g0.row_ptr, g0.col)
    c.set_states(k0)
    ids = [0] + [c.add_graph(g.n, g.row_ptr, g.col, k) for g, k in graphs[1:]]
    tune = c.autotune(-1, 200_000)
    print("[bench] autotune: %s" % tune, file=sys.stderr, flush=True)
    hits = [torch.zeros(g.n, dtype=torch.int32, device="cuda") for g, _ in graphs]
    tasks = [dict(graph=ids[i], first=0, count=per_graph, seed=args.seed + i, phase=0, hits=hits[i])
             for i in range(64)]
    for _ in range(args.warmup):
        c.sample_tasks(tasks)
    torch.cuda.synchronize()
    kern = []
    launch = None
    t1 = time.perf_counter()
    for _ in range(args.steps):
        _, launch = c.sample_tasks(tasks)
        kern.append(launch["kernel_ms"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t1
    total = per_graph * 64
    eager_rate = total * args.steps / elapsed
    # the same launch captured once as a HIP graph, then replayed
    batch = c.capture_batch(tasks)
    for _ in range(args.warmup):
        batch.replay()
    torch.cuda.synchronize()
    kern = []
    t1 = time.perf_counter()
    for _ in range(args.steps):
        _, launch = batch.replay()
        kern.append(launch["kernel_ms"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t1
    batch.close()
    value = total * args.steps / elapsed
    # the same work as 64 separate launches, one graph each
    t2 = time.perf_counter()
    for i in range(64):
        c.sample_tasks([tasks[i]])
    torch.cuda.synchronize()
    seq_rate = total / (time.perf_counter() - t2)
    # one sample per launch, on the median-size graph
    mid = sorted(range(64), key=lambda i: graphs[i][0].n)[32]
    one = dict(graph=ids[mid], first=0, count=1, seed=args.seed, phase=0, hits=hits[mid])
    t3 = time.perf_counter()
    nops = 500
    for j in range(nops):
        one["first"] = j
        c.sample_tasks([one])
    torch.cuda.synchronize()
    opl_rate = nops / (time.perf_counter() - t3)
    avg_kernel_s = sum(kern) / len(kern) / 1e3
    b_alg = algorithmic_bytes(launch)
    achieved = b_alg / avg_kernel_s / 1e9
    traffic = measured_traffic("ba64", total)
    out = {
        "metric": METRIC, "value": value, "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "64 Barabasi-Albert graphs (m=4, n log-uniform in [1e4, 1e6], uniform states), "
                               "%d samples per graph in one launch, captured as a HIP graph and replayed" % per_graph,
                   "nodes": sum(g.n for g, _ in graphs), "arcs": sum(g.m for g, _ in graphs), "tuning": tune},
        "gteps": launch["edges"] * args.steps / elapsed / 1e9,
        "per_sample": {k: launch[k] / total for k in ("edges", "sigma_adds", "vertices_expanded",
                                                       "vertices_discovered", "sum_I", "spilled")},
        "eager_launch": {"value": eager_rate, "unit": "samples/s", "form": "the same launch, issued kernel by kernel"},
        "per_graph_launches": {"value": seq_rate, "unit": "samples/s", "form": "64 launches, one graph each"},
        "one_sample_per_launch": {"value": opl_rate, "unit": "samples/s", "samples": nops},
        "speedup_vs_per_graph": value / seq_rate,
        "speedup_vs_one_per_launch": value / opl_rate,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": "sampler_kernel",
                     "kernel_ms": avg_kernel_s * 1e3, "algorithmic_bytes_per_launch": b_alg,
                     "hbm_gbs_measured": (traffic / avg_kernel_s / 1e9) if traffic else None},
    }
    print(json.dumps(out), flush=True)


def run_setup(args):
    """Device-side setup on one workload: the first percis_set_states (graph
    upload included), state-only updates from a host array and from a device
    tensor (the pair distribution rebuilt on the device each time), and
    VertexDiamUB on the device; the oracle's serial preprocessing and
    VertexDiamUB on the host beside them."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2509_11454_amd import percis as P

    builder, _, desc = WORKLOADS[args.workload]
    g, k = getattr(W, builder)(args.seed)
    rng = np.random.default_rng(args.seed + 1)
    c = P.Context(0)
    t0 = time.perf_counter()
    c.load_csr(g.n, g.row_ptr, g.col, directed=g.directed)
    load_ms = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    c.set_states(k)
    first_ms = (time.perf_counter() - t0) * 1e3
    new_k = [W.beta_states(g.n, rng) for _ in range(args.steps + args.warmup)]
    host_ms, dev_ms = [], []
    for i, kk in enumerate(new_k):
        t0 = time.perf_counter()
        c.set_states(kk)
        if i >= args.warmup:
            host_ms.append((time.perf_counter() - t0) * 1e3)
    dev_k = [torch.from_numpy(kk.view(np.int16)).cuda() for kk in new_k]
    torch.cuda.synchronize()
    for i, kk in enumerate(dev_k):
        t0 = time.perf_counter()
        c.set_states(kk)
        if i >= args.warmup:
            dev_ms.append((time.perf_counter() - t0) * 1e3)
    t0 = time.perf_counter()
    D = c.vertex_diameter()
    diam_ms = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    D2 = c.vertex_diameter()
    cached_ms = (time.perf_counter() - t0) * 1e3
    assert D2 == D
    out = {"metric": "state_update_ms", "value": float(np.median(dev_ms)), "unit": "ms", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "higher_is_better": False, "data": "synthetic",
           "config": {"workload": args.workload + ": " + desc, "n": g.n, "m_arcs": g.m},
           "load_csr_ms": load_ms, "first_set_states_ms": first_ms,
           "state_update_host_k_ms": float(np.median(host_ms)), "state_update_device_k_ms": float(np.median(dev_ms)),
           "vertex_diam_ub": {"D": D, "first_ms": diam_ms, "cached_ms": cached_ms}}
    if not args.no_cpu_baseline:
        import oracle as O
        t0 = time.perf_counter()
        st = O.States(new_k[-1])
        o_states = (time.perf_counter() - t0) * 1e3
        og = O.Graph(g.n, g.row_ptr, g.col, g.directed)
        t0 = time.perf_counter()
        Do = O.vertex_diam_ub(og)
        o_diam = (time.perf_counter() - t0) * 1e3
        assert Do == D, (Do, D)
        del st
        out["cpu_baseline"] = {"kind": "oracle", "cores": 1, "states_ms": o_states, "vertex_diam_ub_ms": o_diam}
    print(json.dumps(out), flush=True)


def run_serve(args):
    """Poisson stream of centrality queries over 66 resident graphs (ER 1000,
    R-MAT scale 18, 64 BA graphs): graph uniform, eps uniform in {0.01,
    0.005, 0.001}, delta = 0.1, seed = query id. Capacity of both forms is
    measured on one saturating burst: the server with every query submitted
    at once, and one query at a time (percis_graph_estimate per query, in
    order). Then Poisson streams at 50/80/95% of the one-at-a-time capacity
    run through both, each in real time on the same arrival times: p50/p99
    latency (arrival to result) and aggregate samples/s."""
    import numpy as np
    import workloads as W
    from paper_2509_11454_amd import percis as P

    rng = np.random.default_rng(args.seed)
    t0 = time.perf_counter()
    g0, k0 = W.workload_er1000(args.seed)
    c = P.Context(0)
    c.load_csr(g0.n, g0.row_ptr, g0.col)
    c.set_states(k0)
    g1, k1 = W.workload_rmat18(args.seed)
    ids = [0, c.add_graph(g1.n, g1.row_ptr, g1.col, k1)]
    for g, k in W.workload_ba_batch(64, 4, args.seed):
        ids.append(c.add_graph(g.n, g.row_ptr, g.col, k))
    print("[bench] 66 graphs resident in %.1f s" % (time.perf_counter() - t0), file=sys.stderr, flush=True)
    budget = 256 << 20
    chunk, step = args.serve_chunk, args.serve_step

    def make_queries(nq, base):
        return [(ids[int(rng.integers(0, len(ids)))], float(rng.choice([0.01, 0.005, 0.001])), 0.1, base + i)
                for i in range(nq)]

    def drive(queries, arrivals):
        srv = P.Server(c, budget, chunk, step)
        t_start = time.perf_counter()
        pending = list(range(len(queries)))
        qid = {}
        lat = [None] * len(queries)
        samples = 0
        while any(x is None for x in lat):
            now = time.perf_counter() - t_start
            while pending and arrivals[pending[0]] <= now:
                i = pending.pop(0)
                qid[i] = srv.submit(*queries[i])
            if not qid or all(lat[i] is not None for i in qid):
                if pending:
                    time.sleep(max(0.0, min(0.01, arrivals[pending[0]] - now)))
                continue
            srv.step()
            t_now = time.perf_counter() - t_start
            for i, q in qid.items():
                if lat[i] is None:
                    r = srv.result(q)
                    if r is not None:
                        rc, p, info = r
                        assert rc == 0, rc
                        lat[i] = t_now - arrivals[i]
                        samples += info["l1"] + info["l"]
        wall = time.perf_counter() - t_start
        st = srv.status()
        srv.close()
        return lat, wall, samples, st

    def one_at_a_time(queries, arrivals):
        """FIFO, one percis_graph_estimate at a time, each started when it has
        arrived and the one before it has finished."""
        t_start = time.perf_counter()
        lat, samples = [], 0
        for q, a in zip(queries, arrivals):
            now = time.perf_counter() - t_start
            if a > now:
                time.sleep(a - now)
            _, info = c.graph_estimate(*q)
            lat.append(time.perf_counter() - t_start - a)
            samples += info["l1"] + info["l"]
        return lat, time.perf_counter() - t_start, samples

    # capacity of both forms on one saturating burst (the first pass warms up
    # VertexDiamUB and the slots of every graph)
    burst = make_queries(args.queries, 10_000)
    drive(burst[:16], [0.0] * 16)
    lat, wall, samples, _ = drive(burst, [0.0] * len(burst))
    cap_qps, cap_sps = len(burst) / wall, samples / wall
    _, seq_wall, seq_samples = one_at_a_time(burst, [0.0] * len(burst))
    seq_qps = len(burst) / seq_wall
    print("[bench] capacity: server %.2f queries/s (%.3g samples/s), one at a time %.2f queries/s"
          % (cap_qps, cap_sps, seq_qps), file=sys.stderr, flush=True)
    levels = {}
    for load in (0.5, 0.8, 0.95):
        lam = load * seq_qps
        queries = make_queries(args.queries, int(load * 1e6))
        gaps = rng.exponential(1.0 / lam, size=len(queries))
        arrivals = list(np.cumsum(gaps) - gaps[0])
        lat, wall, samples, st = drive(queries, arrivals)
        s_lat, s_wall, s_samples = one_at_a_time(queries, arrivals)
        levels["%d%%" % int(load * 100)] = {
            "arrival_qps": lam, "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "samples_per_s": samples / wall,
            "peak_admitted_bytes": st["peak_bytes"],
            "one_at_a_time_p50_ms": float(np.percentile(s_lat, 50) * 1e3),
            "one_at_a_time_p99_ms": float(np.percentile(s_lat, 99) * 1e3),
            "one_at_a_time_samples_per_s": s_samples / s_wall}
        print("[bench] load %.0f%%: %s" % (load * 100, levels["%d%%" % int(load * 100)]), file=sys.stderr, flush=True)
    out = {"metric": METRIC, "value": cap_sps, "unit": "samples/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": "u64", "data": "synthetic", "vs_baseline": None,
           "config": {"workload": "Poisson query stream over 66 resident graphs (ER 1000, R-MAT 18, 64 BA); "
                                  "eps in {0.01, 0.005, 0.001}, delta 0.1; %d queries per load" % args.queries,
                      "memory_budget_bytes": budget, "chunk": chunk, "step_samples": step},
           "capacity_qps": cap_qps, "one_at_a_time_qps": seq_qps, "capacity_ratio": cap_qps / seq_qps,
           "loads_relative_to": "the one-at-a-time capacity", "levels": levels}
    print(json.dumps(out), flush=True)


def copy_calibration(mib):
    """A plain copy kernel of known size: reads and writes mib MiB once. Its
    FETCH_SIZE / WRITE_SIZE readings calibrate the counters of the sampler."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dst.copy_(src)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(json.dumps({"copy_mib": mib, "read_bytes": n * 4, "write_bytes": n * 4, "seconds": dt,
                      "gbs": 2 * n * 4 / dt / 1e9}), flush=True)


def host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
