"""Calling the HIP path from tests: numpy in, numpy out, one line logged per call.

The log line goes straight to the process's stderr (flushed, not captured) so that
the case being run is known even if a GPU run ends abruptly.
"""

from __future__ import annotations

import hashlib
import json
import os
import sys

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def log(msg: str) -> None:
    sys.__stderr__.write(f"[gpu] {msg}\n")
    sys.__stderr__.flush()


def gpu_dbscan(X, eps, min_pts, mode="fp64", tag="", want_stats=False):
    import torch

    from paper_1912_06255_amd import binding

    X = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
    if X.ndim == 1:
        X = X[:, None]
    log(f"{tag} dbscan n={X.shape[0]} d={X.shape[1]} eps={eps!r} minPts={min_pts} mode={mode}")
    T = torch.from_numpy(X).to("cuda")
    core, lab = binding.dbscan(T, eps, min_pts, mode=mode, check=True)
    st = binding.stats()
    out = core.cpu().numpy().astype(np.uint8), lab.cpu().numpy().astype(np.int32)
    return (out, st) if want_stats else out


def digest(core, label) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(core, dtype=np.uint8).tobytes())
    h.update(np.ascontiguousarray(label, dtype="<i4").tobytes())
    return h.hexdigest()


def full_size_cases() -> dict:
    with open(os.path.join(GOLDEN, "full_size_hashes.json")) as f:
        return json.load(f)
