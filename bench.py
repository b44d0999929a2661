#!/usr/bin/env python3
"""Throughput of exact DBSCAN on one MI355X, in points per second.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one full exact DBSCAN (grid, sort, cell boxes and guard, box tree,
MarkCore, ClusterCore, relabel, ClusterBorder, scatter) of every (cloud, setting)
of the workload, inputs already resident in HBM and outputs left in HBM.  Three
timed legs run the same workload:

  plain    : one dbscan() call per (cloud, setting), float64 decisions;
  filter   : the same calls with the float32 filter and float64 recheck;
  batched  : dbscan_batch() with the float32 filter, replaying one captured HIP
             graph per step (the headline value).

Each leg runs W untimed warm-up steps and then exactly K steps between device
synchronisations; value = points * K / seconds.  A profiled loop of the filter leg
records per-phase HIP events on the library's stream; the dominant phase gives the
roofline entry.  The CPU oracle is timed on the host cores on the same workload.

Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "exact-DBSCAN points/s on 1 MI355X: batched FP32-filter vs plain FP64"
HBM_PEAK_GBS = 8000.0


def workloads():
    from workloads import (blobs_2d, config_workload, gaussian_mixture_hd, multi_cloud_batch,
                           seed_spreader_3d)

    def one(gen, eps, mp):
        return lambda: [(gen(), [(eps, mp)])]

    return {
        "spreader3d_n1e6": (one(lambda: seed_spreader_3d(1_000_000), 200.0, 10),
                            "3D seed-spreader random walk, n=1,000,000 over [0,1e5]^3, eps=200, minPts=10"),
        "blobs2d_n2e4": (one(lambda: blobs_2d(20_000), 100.0, 10),
                         "2D Gaussian blobs, n=20,000, eps=100, minPts=10"),
        "mixture5d_n2e6": (lambda: [(gaussian_mixture_hd(5), [(1.5, 10), (2.0, 10), (3.0, 10)])],
                           "5D Gaussian mixture, n=2,000,000, eps in {1.5,2,3}, minPts=10"),
        "mixture7d_n2e6": (lambda: [(gaussian_mixture_hd(7), [(1.5, 10), (2.0, 10), (3.0, 10)])],
                           "7D Gaussian mixture, n=2,000,000, eps in {1.5,2,3}, minPts=10"),
        "sweep3d_n1e7": (lambda: [(i.X, list(zip(i.eps, i.min_pts))) for i in config_workload(3)],
                         "3D seed-spreader n=10,000,000 over [0,1e6]^3, 16 settings "
                         "eps in {200,400,800,1600} x minPts in {5,10,50,100}"),
        "multicloud_256": (lambda: [(i.X, list(zip(i.eps, i.min_pts))) for i in multi_cloud_batch()],
                           "256 Gaussian-mixture clouds, n log-uniform in [1e3,1e6], d in {2,3,5}, "
                           "eps = half the median sigma, minPts=10"),
    }


# Algorithmic HBM bytes per point of each phase, d dimensions, plain / filter.
# These count what the method must move once (inputs read once, outputs written
# once), not what an implementation re-reads.
def algorithmic_bytes_per_point(phase: str, d: int, f32: bool) -> float:
    coord = 4 * d if f32 else 8 * d
    table = {
        "bbox": 8 * d,
        "keys": 8 * d + 12,
        "radix_sort": 24,
        "cells": 12 + 8 * d + 8 * d + 8,
        "cell_boxes": 8 * d + 4,
        "tree": 0,
        "markcore": coord + 4,
        "cluster_core": coord + 1,
        "relabel": 0,
        "border": coord + 1,
        "scatter": 1 + 4 + 4 + 1 + 4,
    }
    return float(table.get(phase, 0.0))


# Kernel behind each phase's roofline entry, as rocprofv3 names it.
PHASE_KERNEL = {
    "cluster_core": "void db::k_bcp<{d}, {f}>(db::Work, int)",
    "markcore": "void db::k_markcore<{d}, {f}>(db::Work)",
    "radix_sort": "db::k_sort_pass(db::Work, int, int)",
    "border": "void db::k_border<{d}, {f}>(db::Work)",
    "cells": "void db::k_cells<{d}>(db::Work, int)",
    "keys": "void db::k_keys<{d}>(db::Work)",
    "cell_boxes": "void db::k_cell_box<{d}>(db::Work, int)",
    "scatter": "db::k_scatter(db::Work)",
}


def kernel_source_digest() -> str:
    """sha256 over the HIP sources (names and bytes), to tell whether stored
    counter figures still describe the kernels that run."""
    import hashlib

    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_1912_06255_amd", "csrc")
    for name in sorted(os.listdir(src)):
        if name.endswith((".hip", ".hpp", ".h")):
            h.update(name.encode())
            with open(os.path.join(src, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def stored_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by its copy-kernel factor), or None when
    there is none or the kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"pmc_traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        line = next((ln for ln in f if ln.startswith("traffic-json: ")), None)
    if line is None:
        return None
    rec = json.loads(line[len("traffic-json: "):])
    if rec.get("source_sha256") != kernel_source_digest():
        return None
    k = rec["kernels"].get(kernel)
    if k is None:
        return None
    sc = rec["scale"]
    b = (k["fetch_kib"] * sc["FETCH_SIZE"] + k["write_kib"] * sc["WRITE_SIZE"]) * 1024.0
    return b, (f"profiles/pmc_traffic_{workload}.md: (FETCH_SIZE x {sc['FETCH_SIZE']} + "
               f"WRITE_SIZE x {sc['WRITE_SIZE']}) KiB per dispatch")


def cpu_baseline(items, budget_s: float = 25.0):
    """Time the C oracle on the host cores on (a bounded prefix of) the workload."""
    from oracle.o1 import build_o1, dbscan_o1, o1_threads

    build_o1(force=False)
    cores = o1_threads()
    X, st = items[0]
    eps, mp = st[0]
    n = len(X)
    m = min(n, 50_000)
    t0 = time.perf_counter()
    dbscan_o1(X[:m], eps, mp)
    t_small = time.perf_counter() - t0
    sample = n if t_small * (n / m) <= budget_s else max(m, min(n, int(m * budget_s / max(t_small, 1e-6))))
    t0 = time.perf_counter()
    dbscan_o1(X[:sample], eps, mp)
    t = time.perf_counter() - t0
    return {
        "value": sample / t,
        "unit": "points/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"C oracle (OpenMP, -O3, no FMA) on the first {sample} of {n} points of the "
                   f"first cloud, eps={eps}, minPts={mp}; {t:.2f} s wall"),
    }


def timed(fn, steps, warmup):
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="spreader3d_n1e6", choices=sorted(workloads()))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the options on the first cloud and setting (both modes) "
                         "before the timed legs; the tuning time is reported, not timed")
    ap.add_argument("--profile-pass", action="store_true",
                    help="only run the workload a few times in each mode plus a reference "
                         "elementwise kernel of known size (256 MiB read, 256 MiB written), "
                         "for rocprofv3 counter runs; prints no JSON")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the design notes describe how it would shard); run with --gpus 1", file=sys.stderr)
        return 2

    import torch

    from paper_1912_06255_amd import binding

    gen, desc = workloads()[args.workload]
    items = gen()
    dev = torch.device("cuda:0")
    clouds = [torch.from_numpy(X).to(dev) for X, _ in items]
    settings = [st for _, st in items]
    points = sum(X.shape[0] * len(st) for X, st in zip(clouds, settings))
    binding.reserve(max(X.shape[0] for X in clouds), max(X.shape[1] for X in clouds))
    outs = [[(torch.empty(X.shape[0], dtype=torch.uint8, device=dev),
              torch.empty(X.shape[0], dtype=torch.int32, device=dev)) for _ in st]
            for X, st in zip(clouds, settings)]

    autotune = None
    if args.tune:
        t0 = time.perf_counter()
        X0, (e0, m0) = clouds[0], settings[0][0]
        autotune = {m: binding.tune(X0, e0, m0, mode=m) for m in ("fp64", "fp32_filter")}
        autotune["seconds"] = time.perf_counter() - t0

    def unbatched(mode):
        def step():
            for X, st, o in zip(clouds, settings, outs):
                for (eps, mp), out in zip(st, o):
                    binding.dbscan(X, eps, mp, mode=mode, out=out, check=False)
        return step

    if args.profile_pass:
        for mode in ("fp64", "fp32_filter"):
            for _ in range(3):
                unbatched(mode)()
        binding.stats(raise_on_error=True)
        a = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 2.0, out=b)  # reads 256 MiB, writes 256 MiB
        torch.cuda.synchronize()
        print("profile pass done", flush=True)
        return 0

    rates = {}
    for leg, mode in (("plain", "fp64"), ("filter", "fp32_filter")):
        wall = timed(unbatched(mode), args.steps, args.warmup)
        binding.stats(raise_on_error=True)
        rates[leg] = (points * args.steps / wall, wall * 1e3 / args.steps)

    batch = binding.Batch(clouds, settings, mode="fp32_filter")
    batch.run()  # capture + instantiate (reported separately, not timed)
    t0 = time.perf_counter()
    batch.run()
    first_replay_ms = (time.perf_counter() - t0) * 1e3
    wall = timed(lambda: batch.run(check=False), args.steps, args.warmup)
    st = binding.stats(raise_on_error=True)
    rates["batched"] = (points * args.steps / wall, wall * 1e3 / args.steps)

    # profiled loop: the filter leg of the first cloud and setting with phase events
    X0, (eps0, mp0), out0 = clouds[0], settings[0][0], outs[0][0]
    n0, d0 = X0.shape
    binding.set_profiling(True)
    acc = {}
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        binding.dbscan(X0, eps0, mp0, mode="fp32_filter", out=out0, check=False)
        for k, v in binding.phase_times().items():
            acc[k] = acc.get(k, 0.0) + v
    prof_wall = time.perf_counter() - t1
    binding.set_profiling(False)
    st0 = binding.stats(raise_on_error=True)
    phase_ms = {k: v / args.steps for k, v in acc.items()}
    dom = max(phase_ms, key=phase_ms.get)
    launches = {"radix_sort": max(1, (st0["key_bits"] + 7) // 8)}.get(dom, 1)
    per_launch_ms = phase_ms[dom] / launches
    alg_bytes = algorithmic_bytes_per_point(dom, d0, True) * n0
    achieved = alg_bytes / (per_launch_ms * 1e-3) / 1e9 if per_launch_ms > 0 else 0.0
    kname = PHASE_KERNEL.get(dom, dom).format(d=d0, f="true")
    traffic, traffic_src = stored_traffic(args.workload, kname) or (None, None)
    roofline = {
        "bound": "hbm",
        "kernel": kname,
        "phase": dom,
        "launches_per_step": launches,
        "achieved": round(achieved, 2),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 5),
        "traffic": None if traffic is None else int(traffic),
        "traffic_source": traffic_src,
        "avg_launch_ms": round(per_launch_ms, 5),
        "alg_bytes_per_launch": int(alg_bytes),
    }

    value, ms = rates["batched"]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "points_per_step": points,
                   "clouds": len(clouds), "settings": sum(len(s) for s in settings)},
        "plain_fp64": {"value": rates["plain"][0], "ms_per_step": rates["plain"][1]},
        "filter_unbatched": {"value": rates["filter"][0], "ms_per_step": rates["filter"][1]},
        "speedup_batched_filter_vs_plain": value / rates["plain"][0],
        "graph_first_replay_ms": first_replay_ms,
        "autotune": autotune,
        "roofline": roofline,
        "phase_ms": {k: round(v, 4) for k, v in phase_ms.items()},
        "profiled_ms_per_step": prof_wall * 1e3 / args.steps,
        "stats_batch": {k: st[k] for k in ("bcp_calls", "uf_links", "fp64_rechecks")},
        "stats_first": {k: st0[k] for k in ("n_cells", "n_unsafe", "n_core", "bcp_calls",
                                            "uf_links", "fp64_rechecks", "key_bits", "key_shift")},
    }
    out["cpu_baseline"] = None if args.no_cpu_baseline else cpu_baseline(items)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
