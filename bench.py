#!/usr/bin/env python3
"""Throughput of exact DBSCAN on one MI355X, in points per second.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--mode fp64|fp32_filter]
                    [--workload NAME]

One step is one full exact DBSCAN of one point cloud already resident in HBM
(grid, sort, cell boxes and guard, box tree, MarkCore, ClusterCore, relabel,
ClusterBorder, scatter), outputs left in HBM.  After W untimed warm-up steps
exactly K steps are timed between device synchronisations; value = points * K /
seconds.  A second timed loop with per-phase HIP events (recorded by the library on
its own stream) gives the duration of the dominant kernel for the roofline entry.
The CPU oracle is timed on the host cores on the same workload for reference.

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
    from workloads import blobs_2d, gaussian_mixture_hd, seed_spreader_3d

    return {
        # name: (generator, eps, minPts, description)
        "spreader3d_n1e6": (lambda: seed_spreader_3d(1_000_000), 200.0, 10,
                            "3D seed-spreader random walk, n=1,000,000 over [0,1e5]^3, eps=200, minPts=10"),
        "blobs2d_n2e4": (lambda: blobs_2d(20_000), 100.0, 10,
                         "2D Gaussian blobs, n=20,000, eps=100, minPts=10"),
        "mixture5d_n2e6_eps2": (lambda: gaussian_mixture_hd(5), 2.0, 10,
                                "5D Gaussian mixture, n=2,000,000, eps=2, minPts=10"),
        "mixture7d_n2e6_eps3": (lambda: gaussian_mixture_hd(7), 3.0, 10,
                                "7D Gaussian mixture, n=2,000,000, eps=3, minPts=10"),
    }


# Algorithmic HBM bytes per point of each phase, plain float64 path, d dimensions.
# These count what the method must move once (inputs read once, outputs written
# once), not what an implementation re-reads.
def algorithmic_bytes_per_point(phase: str, d: int) -> float:
    table = {
        "bbox": 8 * d,                    # read the points
        "keys": 8 * d + 12,               # read points, write key + index
        "radix_sort": 24,                 # one (key, index) scatter: 12 B in, 12 B out
        "cells": 12 + 8 * d + 8 * d + 8,  # read key+index, gather point, write SoA + cell id + perm
        "cell_boxes": 8 * d + 4,          # read SoA + cell id
        "markcore": 8 * d + 1,            # read SoA once, write core flag
        "cluster_core": 8 * d + 1,        # read SoA and core flags once
        "border": 8 * d + 1,
        "scatter": 1 + 4 + 4 + 1 + 4,     # core flag, perm, cell id in; flag + id out
    }
    return float(table.get(phase, 0.0))


def cpu_baseline(X, eps, mp, budget_s: float = 25.0):
    """Time the C oracle on the host cores (bounded: a prefix sample if needed)."""
    from oracle.o1 import build_o1, dbscan_o1, o1_threads

    build_o1(force=False)
    cores = o1_threads()
    n = len(X)
    # calibrate on a small prefix, then size the sample to the budget
    m = min(n, 50_000)
    t0 = time.perf_counter()
    dbscan_o1(X[:m], eps, mp)
    t_small = time.perf_counter() - t0
    sample = n
    if t_small * (n / m) ** 1.0 > budget_s:
        sample = max(m, int(m * budget_s / max(t_small, 1e-6)))
        sample = min(sample, n)
    t0 = time.perf_counter()
    dbscan_o1(X[:sample], eps, mp)
    t = time.perf_counter() - t0
    return {
        "value": sample / t,
        "unit": "points/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"C oracle (OpenMP, -O3, no FMA) on the first {sample} of {n} points "
                   f"of the same cloud, same eps/minPts; {t:.2f} s wall"),
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", default="fp64", choices=["fp64", "fp32_filter"])
    ap.add_argument("--workload", default="spreader3d_n1e6", choices=sorted(workloads()))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(see DESIGN.md for how it would shard); run with --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1912_06255_amd import binding

    gen, eps, mp, desc = workloads()[args.workload]
    X = gen()
    n, d = X.shape
    dev = torch.device("cuda:0")
    T = torch.from_numpy(X).to(dev)
    core = torch.empty(n, dtype=torch.uint8, device=dev)
    lab = torch.empty(n, dtype=torch.int32, device=dev)
    binding.reserve(n, d)

    def step():
        binding.dbscan(T, eps, mp, mode=args.mode, out=(core, lab), check=False)

    for _ in range(args.warmup):
        step()
    st = binding.stats(raise_on_error=True)
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    value = n * args.steps / wall

    # second timed loop with per-phase events on the library's stream
    binding.set_profiling(True)
    acc = {}
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        step()
        for k, v in binding.phase_times().items():
            acc[k] = acc.get(k, 0.0) + v
    prof_wall = time.perf_counter() - t1
    binding.set_profiling(False)
    phase_ms = {k: v / args.steps for k, v in acc.items()}
    st = binding.stats(raise_on_error=True)

    # dominant phase -> roofline entry (HBM bound: sort/scan/gather work)
    dom = max(phase_ms, key=phase_ms.get)
    launches = {"radix_sort": max(1, (st["key_bits"] + 7) // 8)}.get(dom, 1)
    per_launch_ms = phase_ms[dom] / launches
    alg_bytes = algorithmic_bytes_per_point(dom, d) * n
    achieved = alg_bytes / (per_launch_ms * 1e-3) / 1e9 if per_launch_ms > 0 else 0.0
    roofline = {
        "bound": "hbm",
        "kernel": dom,
        "launches_per_step": launches,
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": None,
        "avg_launch_ms": round(per_launch_ms, 5),
        "alg_bytes_per_launch": int(alg_bytes),
    }

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.mode == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "n": n, "d": d, "eps": eps,
                   "min_pts": mp, "mode": args.mode, "batched": False},
        "roofline": roofline,
        "phase_ms": {k: round(v, 4) for k, v in phase_ms.items()},
        "profiled_ms_per_step": prof_wall * 1e3 / args.steps,
        "stats": {k: st[k] for k in ("n_cells", "n_unsafe", "n_core", "bcp_calls", "uf_links",
                                     "fp64_rechecks", "key_bits", "key_shift")},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(X, eps, mp)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
