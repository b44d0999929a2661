"""Host-side logic of bench.py (no GPU): the stored-counter lookup and its guard."""

import json
import os

import bench


def _tree(tmp_path, src_text):
    csrc = tmp_path / "paper_1912_06255_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "a.hpp").write_text(src_text)
    (tmp_path / "profiles").mkdir()
    return csrc


def test_stored_traffic_needs_matching_sources(tmp_path, monkeypatch):
    csrc = _tree(tmp_path, "kernel v1\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    rec = {"scale": {"FETCH_SIZE": 2.0, "WRITE_SIZE": 1.0}, "source_sha256": bench.kernel_source_digest(),
           "kernels": {"k": {"fetch_kib": 10.0, "write_kib": 4.0, "dispatches": 3}}}
    (tmp_path / "profiles" / "pmc_traffic_w.md").write_text("# t\n\ntraffic-json: " + json.dumps(rec) + "\n")
    b, src = bench.stored_traffic("w", "k")
    assert b == (10.0 * 2.0 + 4.0) * 1024.0 and "pmc_traffic_w.md" in src
    assert bench.stored_traffic("w", "other") is None
    assert bench.stored_traffic("missing", "k") is None
    (csrc / "a.hpp").write_text("kernel v2\n")  # the kernels changed since the counters
    assert bench.stored_traffic("w", "k") is None


def test_algorithmic_bytes_table():
    # float64 whole path per point: 8d (bbox) + 8d+12 (keys) + 24 (one pass) + 16d+20
    # (cells) + 8d+4 (boxes) + 3 (8d + 1..4) (distance kernels) + 14 (scatter)
    d = 3
    total = sum(bench.algorithmic_bytes_per_point(p, d, False)
                for p in ("bbox", "keys", "radix_sort", "cells", "cell_boxes", "markcore",
                          "cluster_core", "border", "scatter"))
    assert total == 8 * d + (8 * d + 12) + 24 + (12 + 16 * d + 8) + (8 * d + 4) + (8 * d + 4) + \
        (8 * d + 1) + (8 * d + 1) + 14
    assert bench.algorithmic_bytes_per_point("cluster_core", d, True) == 4 * d + 1


def test_gpus_other_than_one_exit(monkeypatch, capsys):
    monkeypatch.setattr("sys.argv", ["bench.py", "--gpus", "2"])
    assert bench.main() == 2
    assert "one GPU" in capsys.readouterr().err
    assert os.environ.get("WORLD_SIZE", "1") == "1"


def test_step_bytes_model():
    import numpy as np

    # float32 filter: 12d + 28 per cloud and eps, 12d + 5 per setting; float64: 16d + 24, 24d + 5
    X = np.zeros((1000, 3))
    items = [(X, [(1.0, 5), (1.0, 10), (2.0, 5)])]
    assert bench.step_algorithmic_bytes(items, True) == 1000 * (2 * (12 * 3 + 28) + 3 * (12 * 3 + 5))
    assert bench.step_algorithmic_bytes(items, False) == 1000 * (2 * (16 * 3 + 24) + 3 * (24 * 3 + 5))
    # grid phases once per eps, the others once per setting; ClusterCore runs cold once
    # per eps and warm-started for the other settings of that eps
    assert bench.phase_algorithmic_bytes("keys", items, True) == 2 * 1000 * (8 * 3 + 12)
    assert bench.phase_algorithmic_bytes("cluster_core", items, True) == 2 * 1000 * (4 * 3 + 1)
    assert bench.phase_algorithmic_bytes("cluster_core_warm", items, True) == 1 * 1000 * (4 * 3 + 1)
    assert bench.phase_algorithmic_bytes("border", items, True) == 3 * 1000 * (4 * 3 + 1)
    assert bench.phase_algorithmic_bytes("markcore", items, True) == 2 * 1000 * (4 * 3 + 4)


def test_spatial_crop_keeps_density():
    import numpy as np

    rng = np.random.default_rng(5)
    X = rng.uniform(0.0, 100.0, size=(200_000, 3))
    C = bench.spatial_crop(X, 5_000)
    assert 4_900 <= len(C) <= 5_100
    side = float((C.max(axis=0) - X.min(axis=0)).max())
    # uniform density 200k / 1e6: the crop's box holds the same density
    assert abs(len(C) / side ** 3 - 0.2) < 0.03
    assert np.all(C <= X.min(axis=0) + side + 1e-9)
