#!/usr/bin/env python3
"""PercIS hot-path benchmark on one MI355X.

One step = one call of the sampler over the workload's full batch of samples
(pair draw, bidirectional shortest-path-counting BFS, canonical path, hits)
with the graph, the pair distribution and the hit buffer resident in HBM.
Prints one JSON line: sampled s-t paths per second (value), GTEPS, the
roofline of the sampler kernel (algorithmic bytes / kernel time against the
8 TB/s HBM peak), the CPU oracle timed on the host, and the time to an
(eps = 0.01, delta = 0.1) estimate.
"""
import argparse
import hashlib
import json
import os
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
    h = hashlib.sha256()
    for f in ("percis_kernels.hip", "percis_internal.h"):
        with open(os.path.join(ROOT, "paper_2509_11454_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
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


def cpu_baseline(g, k, seed, budget_s, threads):
    """The oracle as it is, on host cores: disjoint sample windows in parallel
    threads (ctypes releases the GIL), grown until about budget_s of work."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle as O
    og, st = O.Graph(g.n, g.row_ptr, g.col, g.directed), O.States(k)
    per = 8
    total = 0
    elapsed = 0.0
    while True:
        t0 = time.perf_counter()
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(lambda i: O.sample_range(og, st, total + i * per, per, seed, 0), range(threads)))
        dt = time.perf_counter() - t0
        total += per * threads
        elapsed += dt
        if elapsed >= budget_s or total >= 200000:
            break
        per = max(per, int(per * min(8.0, max(1.5, (budget_s - elapsed) / max(dt, 1e-3)))))
    return {"value": total / elapsed, "unit": "samples/s", "cores": threads, "kind": "oracle",
            "sample": "first %d sample indices of the same stream (seed %d), %d threads over disjoint windows, "
                      "%.1f s" % (total, seed, threads, elapsed)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat18", choices=sorted(WORKLOADS))
    ap.add_argument("--samples", type=int, default=0, help="samples per step (default: the workload's)")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--slots", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--bitmaps", type=int, default=0, help="0 auto, 1 device memory, 2 LDS")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-estimate", action="store_true")
    ap.add_argument("--one-per-launch", type=int, default=2000, metavar="N",
                    help="also time N samples drawn one per launch (0 = skip)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (reference for HBM counters)")
    args = ap.parse_args()

    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return

    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (samples would be sharded by index "
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
    c.load_csr(g.n, g.row_ptr, g.col, directed=g.directed)
    c.set_states(k)
    hits = torch.zeros(g.n, dtype=torch.int32, device="cuda")
    for i in range(args.warmup):
        _, st = c.sample_range(0, samples, args.seed, 0, hits=hits)
        print("[bench] warmup %d: %.1f ms" % (i, st["kernel_ms"]), file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    totals = dict(edges=0, sigma_adds=0, vertices_expanded=0, vertices_discovered=0, sum_I=0, reachable=0)
    phases = {}
    kernel_ms = []
    t_start = time.perf_counter()
    for i in range(args.steps):
        _, st = c.sample_range(0, samples, args.seed, 0, hits=hits)
        for key in totals:
            totals[key] += st[key]
        for key, v in st["phase_ms"].items():
            phases[key] = phases.get(key, 0.0) + v
        kernel_ms.append(st["kernel_ms"])
        print("[bench] step %d: kernel %.1f ms" % (i, st["kernel_ms"]), file=sys.stderr, flush=True)
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
    bitmaps = "lds" if c.get_option(P.OPT_BITMAPS) == 2 else "device"

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
                   "threads_per_sample": block, "bitmaps": bitmaps},
        "gteps": totals["edges"] / elapsed / 1e9,
        "edges_per_sample": totals["edges"] / (samples * args.steps),
        "reachable_fraction": totals["reachable"] / (samples * args.steps),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "sampler_kernel", "kernel_ms": avg_kernel_s * 1e3,
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
        out["time_to_eps"] = {"eps": 0.01, "delta": 0.1, "wall_ms": info["total_ms"], "l1": info["l1"],
                              "l": info["l"], "D": info["D"], "d_hat": info["d_hat"], "rho_hat": info["rho_hat"],
                              "v_hat": info["v_hat"],
                              "predicted_ms": (info["l1"] + info["l"]) / value * 1e3}
        print("[bench] estimate: l1=%d l=%d in %.1f ms" % (info["l1"], info["l"], info["total_ms"]),
              file=sys.stderr, flush=True)

    if not args.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline(g, k, args.seed, args.cpu_seconds, threads)
        out["cpu_baseline"]["host"] = host_cpu_model()
        print("[bench] cpu baseline: %.1f samples/s" % out["cpu_baseline"]["value"], file=sys.stderr, flush=True)

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
