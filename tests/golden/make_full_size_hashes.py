"""Write full_size_hashes.json: oracle results of full-size workloads, as hashes.

For each workload the C oracle (O1, itself pinned to the brute-force oracle) is run
on the seeded generator output and the SHA-256 of core flags (uint8) followed by
cluster ids (int32, little endian) is stored with a few summary counts.  GPU tests
regenerate the same inputs, run the HIP path and compare hashes.

Run:  python tests/golden/make_full_size_hashes.py   (about eight minutes on 8 cores)
"""

from __future__ import annotations

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


CASES = [
    # (name, config index, instance index, scale, eps, minPts)
    ("blobs2d_n20000_eps100_mp10", 0, 0, 1.0, 100.0, 10),
    ("blobs2d_n20000_eps100_mp50", 0, 0, 1.0, 100.0, 50),
    ("spreader3d_n1000000_eps200_mp10", 1, 0, 1.0, 200.0, 10),
    ("spreader3d_n1000000_eps200_mp100", 1, 0, 1.0, 200.0, 100),
    ("mixture5d_n2000000_eps1.5_mp10", 2, 0, 1.0, 1.5, 10),
    ("mixture5d_n2000000_eps2_mp10", 2, 0, 1.0, 2.0, 10),
    ("mixture5d_n2000000_eps3_mp10", 2, 0, 1.0, 3.0, 10),
]


def main() -> None:
    out = {}
    for name, cfg, inst, scale, eps, mp in CASES:
        X = config_workload(cfg, scale)[inst].X
        t0 = time.time()
        core, label = dbscan_o1(X, eps, mp)
        rec = {"config": cfg, "instance": inst, "scale": scale, "eps": eps, "min_pts": mp,
               "n": int(len(X)), "sha256": digest(core, label)}
        rec.update(summary(core, label))
        out[name] = rec
        print(f"{name}: {time.time() - t0:.1f}s {rec}")
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
