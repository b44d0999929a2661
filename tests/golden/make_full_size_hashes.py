"""Write full_size_hashes.json: oracle results of full-size workloads, as hashes.

For each workload the C oracle (O1, itself pinned to the brute-force oracle) is run
on the seeded generator output and the SHA-256 of core flags (uint8) followed by
cluster ids (int32, little endian) is stored with a few summary counts.  GPU tests
regenerate the same inputs, run the HIP path and compare hashes.

Cases (names say workload, size, eps and minPts):

* the 2D blobs and the 1M-point 3D spreader;
* both 2M-point mixtures (5D and 7D) at eps 1.5, 2 and 3;
* the 10M-point 3D sweep cloud at every eps and minPts of the sweep (about 2, 5.5,
  13 and 16 minutes per setting at eps 200, 400, 800 and 1600 on 8 cores);
* every cloud of the 256-cloud batch (one record holding one hash per cloud).

The file is updated case by case, so a long run can be split (``--only PREFIX``)
and resumed (cases already present are skipped unless ``--redo``).

Run:  python tests/golden/make_full_size_hashes.py   (about three hours on 8 cores,
most of it the sweep cloud at eps 800 and 1600)
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import dbscan_o1  # noqa: E402
from workloads import config_workload  # noqa: E402

OUT = os.path.join(HERE, "full_size_hashes.json")


def digest(core: np.ndarray, label: np.ndarray) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(core, dtype=np.uint8).tobytes())
    h.update(np.ascontiguousarray(label, dtype="<i4").tobytes())
    return h.hexdigest()


def summary(core, label) -> dict:
    return {
        "n_core": int(core.sum()),
        "n_noise": int((label < 0).sum()),
        "n_clusters": int(len(np.unique(label[core.astype(bool)]))),
    }


def _eps_name(e: float) -> str:
    return f"{e:g}"


# (name, config index, instance index, scale, eps, minPts)
CASES = [
    ("blobs2d_n20000_eps100_mp10", 0, 0, 1.0, 100.0, 10),
    ("blobs2d_n20000_eps100_mp50", 0, 0, 1.0, 100.0, 50),
    ("spreader3d_n1000000_eps200_mp10", 1, 0, 1.0, 200.0, 10),
    ("spreader3d_n1000000_eps200_mp100", 1, 0, 1.0, 200.0, 100),
]
for _d, _inst in ((5, 0), (7, 1)):
    for _e in (1.5, 2.0, 3.0):
        CASES.append((f"mixture{_d}d_n2000000_eps{_eps_name(_e)}_mp10", 2, _inst, 1.0, _e, 10))
for _e in (200.0, 400.0, 800.0, 1600.0):
    for _m in (5, 10, 50, 100):
        CASES.append((f"sweep3d_n10000000_eps{_eps_name(_e)}_mp{_m}", 3, 0, 1.0, _e, _m))

MULTI = "multicloud_256"


def _load() -> dict:
    if os.path.exists(OUT):
        with open(OUT) as f:
            return json.load(f)
    return {}


def _save(out: dict) -> None:
    tmp = OUT + ".tmp"
    with open(tmp, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    os.replace(tmp, OUT)


def _workload(cache: dict, cfg: int, scale: float):
    key = (cfg, scale)
    if key not in cache:
        cache.clear()  # one workload in memory at a time
        cache[key] = config_workload(cfg, scale)
    return cache[key]


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", action="append", default=[], help="run cases with this name prefix")
    ap.add_argument("--redo", action="store_true", help="recompute cases already in the file")
    args = ap.parse_args()

    def wanted(name: str) -> bool:
        return not args.only or any(name.startswith(p) for p in args.only)

    out = _load()
    cache: dict = {}
    for name, cfg, inst, scale, eps, mp in CASES:
        if not wanted(name) or (name in out and not args.redo):
            continue
        X = _workload(cache, cfg, scale)[inst].X
        t0 = time.time()
        core, label = dbscan_o1(X, eps, mp)
        rec = {"config": cfg, "instance": inst, "scale": scale, "eps": eps, "min_pts": mp,
               "n": int(len(X)), "sha256": digest(core, label), "oracle_s": round(time.time() - t0, 1)}
        rec.update(summary(core, label))
        out[name] = rec
        _save(out)
        print(f"{name}: {rec}", flush=True)

    if wanted(MULTI) and (MULTI not in out or args.redo):
        insts = _workload(cache, 4, 1.0)
        clouds = []
        t0 = time.time()
        for ci, I in enumerate(insts):
            core, label = dbscan_o1(I.X, I.eps[0], I.min_pts[0])
            rec = {"n": I.n, "d": I.d, "eps": I.eps[0], "min_pts": I.min_pts[0],
                   "sha256": digest(core, label)}
            rec.update(summary(core, label))
            clouds.append(rec)
            if ci % 32 == 31:
                print(f"{MULTI}: {ci + 1} clouds, {time.time() - t0:.1f}s", flush=True)
        out[MULTI] = {"config": 4, "scale": 1.0, "clouds": clouds,
                      "oracle_s": round(time.time() - t0, 1)}
        _save(out)
        print(f"{MULTI}: done in {time.time() - t0:.1f}s", flush=True)


if __name__ == "__main__":
    main()
