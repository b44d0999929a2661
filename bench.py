#!/usr/bin/env python3
"""Throughput of exact DBSCAN on one MI355X, in points per second.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one full exact DBSCAN (grid, sort, cell boxes and guard, box tree,
MarkCore, ClusterCore, relabel, ClusterBorder, scatter) of every (cloud, setting)
of the workload, inputs already resident in HBM and outputs left in HBM.  The
default workload is the batched parameter sweep: one 3D seed-spreader cloud of
10,000,000 points with 16 (eps, minPts) settings.  Four timed legs run it:

  plain          : one dbscan() call per (cloud, setting), float64 decisions;
  filter         : the same calls with the float32 filter and float64 recheck;
  batched_fp64   : dbscan_batch() in float64, replaying one captured HIP graph;
  batched        : dbscan_batch() with the float32 filter, replaying one captured
                   HIP graph per step (the headline value).

Each leg runs W untimed warm-up steps and then exactly K steps between device
synchronisations; value = points * K / seconds.  A profiled step of the batched
filter leg (run eagerly, HIP events on the library's stream at every phase
boundary) gives the per-phase times: the dominant phase's kernel is the roofline
entry.  The whole-step algorithmic bytes follow the per-point model of the design
notes (grid bytes once per cloud and eps, the rest once per setting).  The CPU
oracle is timed on the host cores on a spatial crop of the first cloud.  With
--extra (the default) the 1M-point 3D cloud, the 256-cloud batch and the 5D / 7D
mixtures (float32 filter forced on) are timed too, with fewer steps.

Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "exact-DBSCAN points/s on 1 MI355X: batched FP32-filter vs plain FP64"
HBM_PEAK_GBS = 8000.0
# vector FP64 = unpacked vector FP32 on MI355X: 256 CUs x 2.4 GHz x 128 flop/clk
VALU_PEAK_TFLOPS = 78.6
DEFAULT_WORKLOAD = "sweep3d_n1e7"


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
        "core_flags": 4 + 4 + 1,
        "cluster_core": coord + 1,
        "cluster_core_warm": coord + 1,
        "relabel": 0,
        "border": coord + 1,
        "scatter": 1 + 4 + 4 + 1 + 4,
    }
    return float(table.get(phase, 0.0))


# Whole-path model (bytes per point): the grid part (read the input, write the
# cell-sorted copy, one key + index pass) is paid once per cloud and eps, the rest
# (three distance phases reading the sorted coordinates, the two outputs) once per
# setting.  Plain: 16d + 24 and 24d + 5; filter: 12d + 28 and 12d + 5.
def step_bytes_per_point(d: int, f32: bool) -> tuple[float, float]:
    if f32:
        return 12.0 * d + 28.0, 12.0 * d + 5.0
    return 16.0 * d + 24.0, 24.0 * d + 5.0


def step_algorithmic_bytes(items, f32: bool) -> float:
    total = 0.0
    for X, st in items:
        n, d = X.shape
        grid, per_setting = step_bytes_per_point(d, f32)
        total += n * (grid * len({e for e, _ in st}) + per_setting * len(st))
    return total


# Phases paid once per cloud and eps (the grid and the one neighbour count); the
# others once per setting.
PER_EPS_PHASES = ("bbox", "keys", "radix_sort", "cells", "cell_boxes", "tree", "markcore",
                  "core_flags")


def phase_algorithmic_bytes(phase: str, items, f32: bool) -> float:
    """Algorithmic bytes of one phase over a whole batched step (every occurrence).
    Settings of one eps run ClusterCore cold once (the largest minPts) and warm-started
    for the others, which the phase events time apart."""
    total = 0.0
    for X, st in items:
        n, d = X.shape
        n_eps = len({e for e, _ in st})
        if phase in PER_EPS_PHASES or phase == "cluster_core":
            reps = n_eps
        elif phase == "cluster_core_warm":
            reps = len(st) - n_eps
        else:
            reps = len(st)
        total += reps * n * algorithmic_bytes_per_point(phase, d, f32)
    return total


# Kernel behind each phase's roofline entry, as rocprofv3 names it.
PHASE_KERNEL = {
    "cluster_core": "void db::k_bcp<{d}, {f}, false, db::OneWork>(db::OneWork, int)",
    "cluster_core_warm": "void db::k_bcp<{d}, {f}, true, db::OneWork>(db::OneWork, int)",
    "markcore": "void db::k_markcore<{d}, {f}, db::OneWork>(db::OneWork)",
    "radix_sort": "void db::k_sort_pass<db::OneWork>(db::OneWork, int)",
    "border": "void db::k_border<{d}, {f}, db::OneWork>(db::OneWork)",
    "cells": "void db::k_cells<{d}, db::OneWork>(db::OneWork, int)",
    "keys": "void db::k_keys<{d}, db::OneWork>(db::OneWork, int)",
    "cell_boxes": "void db::k_cell_box<{d}, db::OneWork>(db::OneWork, int)",
    "scatter": "void db::k_scatter<db::OneWork>(db::OneWork)",
    "core_flags": "void db::k_core_from_count<db::OneWork>(db::OneWork)",
}
# Settings of one eps computed together use these instead.
PHASE_KERNEL_GROUPED = {
    "scatter": "db::k_output_multi(db::Work, db::MultiOut)",
    "core_flags": "db::k_core_multi(db::Work, db::MultiCore)",
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


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def spatial_crop(X, m: int):
    """The points of X inside the box [min, min + L]^d with L chosen so that about m
    points fall inside: a bounded sample with the cloud's own local density (a
    prefix of a shuffled cloud would thin it out)."""
    import numpy as np

    lo = X.min(axis=0)
    span = float((X.max(axis=0) - lo).max())
    a, b = 0.0, span
    for _ in range(40):
        mid = 0.5 * (a + b)
        if int(np.all(X - lo <= mid, axis=1).sum()) < m:
            a = mid
        else:
            b = mid
    return np.ascontiguousarray(X[np.all(X - lo <= b, axis=1)])


def cpu_baseline(items, budget_s: float = 15.0, budget_1t_s: float = 8.0):
    """Time the C oracle on the host cores (all of them, then one) on spatial crops of
    the first cloud at its first setting."""
    from oracle.o1 import build_o1, dbscan_o1, o1_threads

    build_o1(force=False)
    cores = o1_threads()
    X, st = items[0]
    eps, mp = st[0]
    n = len(X)

    def rate(threads, budget):
        m = min(n, 20_000)
        C = spatial_crop(X, m) if m < n else X
        t0 = time.perf_counter()
        dbscan_o1(C, eps, mp, threads=threads)
        t = time.perf_counter() - t0
        while len(C) < n and t < 0.3 * budget:
            m = min(n, int(len(C) * min(8.0, max(1.5, 0.8 * budget / max(t, 1e-3)))))
            C = spatial_crop(X, m) if m < n else X
            t0 = time.perf_counter()
            dbscan_o1(C, eps, mp, threads=threads)
            t = time.perf_counter() - t0
        return len(C) / t, len(C), t

    v, m, t = rate(cores, budget_s)
    v1, m1, t1 = rate(1, budget_1t_s)
    return {
        "value": v,
        "unit": "points/s",
        "cores": cores,
        "kind": "oracle",
        "cpu_model": cpu_model(),
        "sample": (f"C oracle (OpenMP, -O3, no FMA) on a spatial crop of {m} of the {n} points of "
                   f"the first cloud (a corner box keeping the local density), eps={eps}, "
                   f"minPts={mp}; {t:.2f} s wall on {cores} threads"),
        "one_thread": {"value": v1, "unit": "points/s", "sample_points": m1, "seconds": round(t1, 3)},
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


def prepare(items, dev):
    import torch

    from paper_1912_06255_amd import binding

    clouds = [torch.from_numpy(X).to(dev) for X, _ in items]
    settings = [st for _, st in items]
    binding.reserve(max(X.shape[0] for X in clouds), max(X.shape[1] for X in clouds))
    outs = [[(torch.empty(X.shape[0], dtype=torch.uint8, device=dev),
              torch.empty(X.shape[0], dtype=torch.int32, device=dev)) for _ in st]
            for X, st in zip(clouds, settings)]
    points = sum(X.shape[0] * len(st) for X, st in zip(clouds, settings))
    return clouds, settings, outs, points


def unbatched(clouds, settings, outs, mode):
    from paper_1912_06255_amd import binding

    def step():
        for X, st, o in zip(clouds, settings, outs):
            for (eps, mp), out in zip(st, o):
                binding.dbscan(X, eps, mp, mode=mode, out=out, check=False)
    return step


def batched_rate(clouds, settings, mode, points, steps, warmup):
    from paper_1912_06255_amd import binding

    batch = binding.Batch(clouds, settings, mode=mode)
    batch.run()  # capture + instantiate (reported separately, not timed)
    t0 = time.perf_counter()
    batch.run()
    first_ms = (time.perf_counter() - t0) * 1e3
    wall = timed(lambda: batch.run(check=False), steps, warmup)
    st = binding.stats(raise_on_error=True)
    return batch, points * steps / wall, wall * 1e3 / steps, first_ms, st


def extra_workload(name, dev, steps, warmup, filter_max_d=None):
    """Plain (one call per setting) against the batched float32-filter graph on
    another workload; per-eps recheck counts and filter band widths for the
    mixtures (their filter forced on with filter_max_d)."""
    import torch

    from paper_1912_06255_amd import binding

    gen, desc = workloads()[name]
    items = gen()
    clouds, settings, outs, points = prepare(items, dev)
    if filter_max_d is not None:
        binding.set_option("filter_max_d", filter_max_d)
    try:
        wall = timed(unbatched(clouds, settings, outs, "fp64"), steps, warmup)
        binding.stats(raise_on_error=True)
        plain = (points * steps / wall, wall * 1e3 / steps)
        batch, v, ms, _, st = batched_rate(clouds, settings, "fp32_filter", points, steps, warmup)
        rec = {"description": desc, "points_per_step": points, "clouds": len(clouds),
               "settings": sum(len(s) for s in settings), "steps": steps, "warmup": warmup,
               "plain_fp64": {"value": plain[0], "ms_per_step": plain[1]},
               "batched_filter": {"value": v, "ms_per_step": ms},
               "speedup_batched_filter_vs_plain": v / plain[0],
               "fp64_rechecks_batch": st["fp64_rechecks"]}
        if filter_max_d is not None:
            rec["filter_max_d"] = filter_max_d
            # the default choice for comparison: float64 decisions above 3 dimensions
            binding.set_option("filter_max_d", -1)
            b2, v2, ms2, _, _ = batched_rate(clouds, settings, "fp32_filter", points, steps, warmup)
            del b2
            rec["batched_default"] = {"value": v2, "ms_per_step": ms2, "filter_max_d": -1}
            binding.set_option("filter_max_d", filter_max_d)
            per_eps = []
            X, st0, o0 = clouds[0], settings[0], outs[0]
            for (eps, mp), out in zip(st0, o0):
                binding.dbscan(X, eps, mp, mode="fp32_filter", out=out, check=True)
                s = binding.stats(raise_on_error=True)
                e2 = eps * eps
                per_eps.append({"eps": eps, "min_pts": mp, "fp64_rechecks": s["fp64_rechecks"],
                                "pair_tests": s["pair_tests"],
                                "band_width_rel": (s["filter_tout"] - s["filter_tin"]) / e2})
            rec["filter_per_eps"] = per_eps
        del batch
        return rec
    finally:
        if filter_max_d is not None:
            binding.set_option("filter_max_d", -1)
        del clouds, outs
        torch.cuda.empty_cache()


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(workloads()))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other workloads (1M 3D, 256 clouds, 5D/7D mixtures)")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the options on the first cloud and setting (both modes) "
                         "before the timed legs; the tuning time is reported, not timed")
    ap.add_argument("--profile-pass", action="store_true",
                    help="only run the workload a few times (unbatched in both modes, then the "
                         "batched float32-filter graph) plus a reference elementwise kernel of "
                         "known size (256 MiB read, 256 MiB written), for rocprofv3 counter "
                         "runs; prints no JSON")
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
    clouds, settings, outs, points = prepare(items, dev)

    autotune = None
    if args.tune:
        t0 = time.perf_counter()
        X0, (e0, m0) = clouds[0], settings[0][0]
        autotune = {m: binding.tune(X0, e0, m0, mode=m) for m in ("fp64", "fp32_filter")}
        autotune["seconds"] = time.perf_counter() - t0

    if args.profile_pass:
        for mode in ("fp64", "fp32_filter"):
            for _ in range(2):
                unbatched(clouds, settings, outs, mode)()
        b = binding.Batch(clouds, settings, mode="fp32_filter")
        for _ in range(3):
            b.run(check=False)
        binding.stats(raise_on_error=True)
        a = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        o = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 2.0, out=o)  # reads 256 MiB, writes 256 MiB
        torch.cuda.synchronize()
        print("profile pass done", flush=True)
        return 0

    rates = {}
    for leg, mode in (("plain", "fp64"), ("filter", "fp32_filter")):
        wall = timed(unbatched(clouds, settings, outs, mode), args.steps, args.warmup)
        binding.stats(raise_on_error=True)
        rates[leg] = (points * args.steps / wall, wall * 1e3 / args.steps)
        print(f"[bench] {leg}: {rates[leg][1]:.3f} ms/step", file=sys.stderr, flush=True)

    b64, v, ms, _, _ = batched_rate(clouds, settings, "fp64", points, args.steps, args.warmup)
    rates["batched_fp64"] = (v, ms)
    del b64
    batch, v, ms, first_replay_ms, st = batched_rate(clouds, settings, "fp32_filter", points,
                                                     args.steps, args.warmup)
    rates["batched"] = (v, ms)
    print(f"[bench] batched: {ms:.3f} ms/step", file=sys.stderr, flush=True)

    # profiled steps: the batched float32-filter step run eagerly with phase events
    prof_steps = max(1, min(args.steps, 5))
    binding.set_profiling(True)
    acc, occ = {}, {}
    pair_tests = 0
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(prof_steps):
        batch.run(check=False)
        for k, (v_ms, v_occ) in binding.phase_stats().items():
            acc[k] = acc.get(k, 0.0) + v_ms
            occ[k] = v_occ
        pair_tests += binding.stats(raise_on_error=True)["pair_tests"]
    prof_wall = time.perf_counter() - t1
    binding.set_profiling(False)
    phase_ms = {k: v / prof_steps for k, v in acc.items()}
    dom = max(phase_ms, key=phase_ms.get)
    d0 = clouds[0].shape[1]
    launches = max(1, occ.get(dom, 1))
    per_launch_ms = phase_ms[dom] / launches
    alg_launch = phase_algorithmic_bytes(dom, items, True) / launches
    achieved = alg_launch / (per_launch_ms * 1e-3) / 1e9 if per_launch_ms > 0 else 0.0
    grouped = any(len(st) > len({e for e, _ in st}) for _, st in items)
    table = dict(PHASE_KERNEL, **(PHASE_KERNEL_GROUPED if grouped else {}))
    kname = table.get(dom, dom).format(d=d0, f="true")
    traffic, traffic_src = stored_traffic(args.workload, kname) or (None, None)
    step_bytes = step_algorithmic_bytes(items, True)
    step_gbs = step_bytes / (rates["batched"][1] * 1e-3) / 1e9
    # float64-equivalent flops of ClusterCore's pair tests: (3d - 1) per pair (cold and
    # warm-started runs; the pair count covers both)
    cc_ms = phase_ms.get("cluster_core", 0.0) + phase_ms.get("cluster_core_warm", 0.0)
    cc_launches = max(1, occ.get("cluster_core", 0) + occ.get("cluster_core_warm", 0))
    flops = (3 * d0 - 1) * pair_tests / prof_steps
    valu_tflops = flops / (cc_ms * 1e-3) / 1e12 if cc_ms > 0 else 0.0
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
        "alg_bytes_per_launch": int(alg_launch),
        "whole_step": {"alg_bytes": int(step_bytes), "achieved": round(step_gbs, 2), "unit": "GB/s",
                       "frac": round(step_gbs / HBM_PEAK_GBS, 5),
                       "model": "per point: 12d+28 B per cloud and eps (grid) + 12d+5 B per setting"},
        "valu_cluster_core": {"kernel": "void db::k_bcp<{d}, true, *, db::OneWork>(db::OneWork, int)".format(d=d0),
                              "pair_tests_per_step": int(pair_tests / prof_steps),
                              "flops_per_pair": 3 * d0 - 1,
                              "avg_launch_ms": round(cc_ms / cc_launches, 5),
                              "achieved": round(valu_tflops, 4), "peak": VALU_PEAK_TFLOPS,
                              "unit": "TFLOP/s", "frac": round(valu_tflops / VALU_PEAK_TFLOPS, 7)},
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
        "batched_fp64": {"value": rates["batched_fp64"][0], "ms_per_step": rates["batched_fp64"][1]},
        "speedup_batched_filter_vs_plain": value / rates["plain"][0],
        "speedup_batched_fp64_vs_plain": rates["batched_fp64"][0] / rates["plain"][0],
        "graph_first_replay_ms": first_replay_ms,
        "autotune": autotune,
        "roofline": roofline,
        "phase_ms": {k: round(v, 4) for k, v in phase_ms.items()},
        "phase_occurrences": occ,
        "profiled_ms_per_step": prof_wall * 1e3 / prof_steps,
        "stats_batch": {k: st[k] for k in ("bcp_calls", "uf_links", "fp64_rechecks", "pair_tests")},
    }
    del batch, clouds, outs
    torch.cuda.empty_cache()
    if not args.no_extra:
        extra = {}
        for name, fmd in (("spreader3d_n1e6", None), ("multicloud_256", None),
                          ("mixture5d_n2e6", 8), ("mixture7d_n2e6", 8)):
            if name == args.workload:
                continue
            k = max(1, min(args.steps, 5))
            extra[name] = extra_workload(name, dev, k, 1, filter_max_d=fmd)
            e = extra[name]
            msg = (f"[bench] {name}: plain {e['plain_fp64']['ms_per_step']:.2f}, batched "
                   f"{e['batched_filter']['ms_per_step']:.2f} ms/step")
            if "batched_default" in e:
                msg += f" (float64 decisions: {e['batched_default']['ms_per_step']:.2f})"
            print(msg, file=sys.stderr, flush=True)
        out["other_workloads"] = extra
    out["cpu_baseline"] = None if args.no_cpu_baseline else cpu_baseline(items)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
