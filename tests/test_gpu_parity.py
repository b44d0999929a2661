"""HIP path against the CPU oracle: element-by-element parity, edge cases, errors.

Expected values come only from the oracle (O1, pinned to the brute-force O0) or
from the fixtures under golden/; nothing expected is produced by the HIP path.
"""

import numpy as np
import pytest

from oracle import dbscan_brute, dbscan_o1
from tests.gpu_helpers import digest, full_size_cases, gpu_dbscan, log
from tests.pins import ALL_PINS
from workloads import blobs_2d, config_workload, gaussian_mixture, multi_cloud_batch, seed_spreader_3d

pytestmark = pytest.mark.gpu

MODES = ["fp64", "fp32_filter"]


def _impl(mode):
    def f(X, eps, mp):
        return gpu_dbscan(X, eps, mp, mode=mode, tag="pin")

    return f


def _assert_parity(X, eps, mp, mode, tag, oracle=dbscan_o1):
    want = oracle(X, eps, mp)
    got = gpu_dbscan(X, eps, mp, mode=mode, tag=tag)
    bad_core = np.flatnonzero(got[0] != want[0])
    bad_lab = np.flatnonzero(got[1] != want[1])
    assert bad_core.size == 0, f"{tag}: {bad_core.size} core flags differ, first {bad_core[:5]}"
    assert bad_lab.size == 0, (
        f"{tag}: {bad_lab.size} labels differ, first idx {bad_lab[:5]} "
        f"got {got[1][bad_lab[:5]]} want {want[1][bad_lab[:5]]}"
    )


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("pin", sorted(ALL_PINS))
def test_pins_on_gpu(pin, mode, gpu_lib):
    fails = ALL_PINS[pin](_impl(mode))
    assert not fails, "\n".join(fails)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("mp", [1, 4, 10, 30, 100])
def test_blobs(mp, mode, gpu_lib):
    _assert_parity(blobs_2d(6000, seed=201), 100.0, mp, mode, f"blobs mp={mp}")


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("eps,mp", [(200.0, 10), (400.0, 50), (120.0, 5), (60.0, 100)])
def test_seed_spreader(eps, mp, mode, gpu_lib):
    n = 60_000
    X = seed_spreader_3d(n, domain=1e5 * (n / 1e6) ** (1 / 3), seed=202)
    _assert_parity(X, eps, mp, mode, f"spreader eps={eps} mp={mp}")


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("d", [4, 5, 7, 8])
@pytest.mark.parametrize("eps", [1.5, 3.0])
def test_high_dim(d, eps, mode, gpu_lib):
    rng = np.random.Generator(np.random.PCG64(203 + d))
    X = gaussian_mixture(8000, d, 12, 1.0, 16.0, 0.05, rng)
    _assert_parity(X, eps, 10, mode, f"mixture d={d} eps={eps}")
    if mode == "fp32_filter":
        # the float32 filter path itself, which is off by default above 3 dimensions
        try:
            _set_opts(filter_max_d=8)
            _assert_parity(X, eps, 10, mode, f"mixture d={d} eps={eps} filter forced")
        finally:
            _set_opts(filter_max_d=-1)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("filter_max_d", [-1, 8])
def test_multi_cloud_small(mode, filter_max_d, gpu_lib):
    try:
        _set_opts(filter_max_d=filter_max_d)
        for i, inst in enumerate(multi_cloud_batch(n_clouds=16, size_scale=0.01)):
            _assert_parity(inst.X, inst.eps[0], inst.min_pts[0], mode, f"cloud {i} d={inst.d}")
    finally:
        _set_opts(filter_max_d=-1)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("d", [1, 2, 3, 5])
def test_lattice_exact_boundaries(d, mode, gpu_lib):
    rng = np.random.Generator(np.random.PCG64(204))
    P = rng.integers(0, 12, size=(5000, d)).astype(np.float64)
    for mp in (2, 3, 2 * d + 1, 40):
        _assert_parity(P, 1.0, mp, mode, f"lattice d={d} mp={mp}")


# eps values for which a grid cell of side fl(eps / fl(sqrt(d))) contains two
# corner points whose float64 distance test fails (found by search): the dense-cell
# shortcut would be wrong there without the diameter guard.
UNSAFE_EPS = [(3, 2.464117292042362), (7, 2.379220351910591)]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("d,eps", UNSAFE_EPS)
def test_unsafe_cells_split(d, eps, mode, gpu_lib):
    s = eps / np.sqrt(d)
    hi = np.nextafter(s, 0.0)
    lo_pts = np.zeros((6, d))
    hi_pts = np.full((6, d), hi)
    rng = np.random.Generator(np.random.PCG64(205))
    far = rng.uniform(5 * eps, 9 * eps, size=(300, d))
    X = np.concatenate([lo_pts, hi_pts, far])
    (got, st) = gpu_dbscan(X, eps, 10, mode=mode, tag=f"unsafe d={d}", want_stats=True)
    want = dbscan_o1(X, eps, 10)
    assert st["n_unsafe"] >= 1, st
    assert not want[0][:12].any(), "test data must make the corner points non-core"
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


def test_filter_band_ignores_split_cells(gpu_lib):
    """Coarsened keys make every cell unsafe: all are split into single points, whose
    anchors are the points themselves, so the float32 filter keeps its narrow band
    (the extent of a split cell must not widen it) and rechecks stay rare."""
    rng = np.random.Generator(np.random.PCG64(215))
    blob = rng.normal(0.0, 1.5, size=(5_000, 2))
    X = np.concatenate([blob, [[1e30, 1e30], [-1e30, 2e30]]])
    (got, st) = gpu_dbscan(X, 1.0, 5, mode="fp32_filter", tag="split cells band", want_stats=True)
    want = dbscan_brute(X, 1.0, 5)  # (the bucket oracle does not take extents of 1e30)
    assert st["key_shift"] > 0 and st["n_unsafe"] >= 1, st
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
    assert np.isfinite(st["filter_tin"]) and np.isfinite(st["filter_tout"]), st
    assert (st["filter_tout"] - st["filter_tin"]) < 1e-5, st
    assert st["pair_tests"] > 0 and st["fp64_rechecks"] * 100 <= st["pair_tests"], st


@pytest.mark.parametrize("mode", MODES)
def test_unsafe_split_with_sub_cell_order(mode, gpu_lib):
    """An unsafe cell first in cell order (its split renumbers every later cell)
    and large cells after it that are put into sub-cell order: the queue of large
    cells must survive the renumbering."""
    d, eps = UNSAFE_EPS[0]
    s = eps / np.sqrt(d)
    hi = np.nextafter(s, 0.0)
    rng = np.random.Generator(np.random.PCG64(308))
    corners = np.concatenate([np.zeros((6, d)), np.full((6, d), hi)])
    blobs = np.concatenate([rng.uniform(c * eps, c * eps + 1.2 * eps, size=(6000, d))
                            for c in (20.0, 24.0, 40.0)])
    far = rng.uniform(60 * eps, 90 * eps, size=(300, d))
    X = np.concatenate([corners, blobs, far])
    try:
        _set_opts(subcell_min=2)
        (got, st) = gpu_dbscan(X, eps, 10, mode=mode, tag="unsafe + sub-cell", want_stats=True)
    finally:
        _set_opts(subcell_min=-1)
    want = dbscan_o1(X, eps, 10)
    assert st["n_unsafe"] >= 1, st
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("big_first", [False, True])
def test_large_cell_bridge(mode, d, big_first, gpu_lib):
    """Two core cells joined by a single pair whose point in the large cell (10,000
    points: more than 64 chunks of 64 even after the unit is split in two) comes
    last in that cell, so that only a full scan of the large side finds it."""
    rng = np.random.Generator(np.random.PCG64(501 + d))
    side = 1.0 / np.sqrt(d)  # eps = 1
    small = 0.01 + rng.uniform(0, 0.02, size=(30, d))
    far = np.full(d, side - 0.03)
    far[0] += side  # far corner of the next cell along x
    big = far + rng.uniform(0, 0.02, size=(10000, d))
    bridge = np.full((1, d), 0.05)
    bridge[0, 0] = side + 0.015
    if big_first:  # mirrored: the large cell gets the lower Morton index
        m = 2 * side
        small, big, bridge = m - small, m - big, m - bridge
    X = np.concatenate([small, big, bridge])
    want = dbscan_o1(X, 1.0, 5)
    assert np.unique(want[1]).size == 1, "test data must form one cluster"
    _assert_parity(X, 1.0, 5, mode, f"large cell bridge d={d} big_first={big_first}")


@pytest.mark.parametrize("mode", MODES)
def test_edge_cases(mode, gpu_lib):
    import torch

    from paper_1912_06255_amd import binding

    log("edge n=0")
    core, lab = binding.dbscan(torch.zeros((0, 3), dtype=torch.float64, device="cuda"), 1.0, 5, mode=mode)
    assert core.numel() == 0 and lab.numel() == 0
    _assert_parity(np.array([[1.0, 2.0]]), 0.5, 1, mode, "single point mp=1")
    _assert_parity(np.array([[1.0, 2.0]]), 0.5, 2, mode, "single point mp=2")
    _assert_parity(np.full((3000, 2), 7.5), 0.1, 10, mode, "all duplicates")
    rng = np.random.Generator(np.random.PCG64(206))
    X = rng.uniform(0, 10, size=(4000, 3))
    _assert_parity(X, 0.7, 4001, mode, "minPts > n")
    _assert_parity(X, 0.7, 1, mode, "minPts = 1")
    _assert_parity(X, 100.0, 50, mode, "eps above diameter")
    _assert_parity(X, 1e-6, 2, mode, "tiny eps", oracle=dbscan_brute)
    # sparse cells with more than 64 points: minPts far above the per-cell count
    Y = rng.uniform(0, 4, size=(20000, 2))
    _assert_parity(Y, 0.3, 300, mode, "minPts 300")
    _assert_parity(rng.uniform(0, 100, size=(7000, 1)), 0.05, 3, mode, "d=1")
    _assert_parity(rng.normal(0, 1, size=(5000, 8)), 2.0, 6, mode, "d=8")
    # ragged sizes around tile edges (radix tiles of 4096 points, waves of 64)
    for n in (63, 64, 65, 2047, 2049, 4095, 4096, 4097, 8193):
        Z = rng.uniform(0, 30, size=(n, 2))
        _assert_parity(Z, 1.0, 3, mode, f"ragged n={n}")


def test_device_errors(gpu_lib):
    import torch

    from paper_1912_06255_amd import binding

    X = torch.zeros((100, 2), dtype=torch.float64, device="cuda")
    X[7, 1] = float("nan")
    log("error nonfinite")
    with pytest.raises(binding.DbscanError) as e:
        binding.dbscan(X, 1.0, 3)
    assert e.value.code == binding.ENONFINITE
    # extreme extent: the key is coarsened and the result still matches the oracle
    for mp in (1, 2):
        Y = np.array([[0.0, 0.0], [1e300, 1e300], [1e300, 1e300 + 1e284]])
        (got, st) = gpu_dbscan(Y, 1.0, mp, tag=f"extreme extent mp={mp}", want_stats=True)
        want = dbscan_brute(Y, 1.0, mp)
        assert st["key_shift"] > 0, st
        assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
    Z = torch.zeros((10, 2), dtype=torch.float64, device="cuda")
    for eps, mp in ((0.0, 3), (-1.0, 3), (float("inf"), 3), (float("nan"), 3), (1.0, 0)):
        with pytest.raises(binding.DbscanError) as e:
            binding.dbscan(Z, eps, mp)
        assert e.value.code == binding.EINVAL
    with pytest.raises(binding.DbscanError) as e:
        binding.dbscan(torch.zeros((10, 9), dtype=torch.float64, device="cuda"), 1.0, 2)
    assert e.value.code == binding.EINVAL
    # the context still works after errors
    _assert_parity(np.random.default_rng(1).uniform(0, 5, (500, 2)), 0.4, 4, "fp64", "after errors")


def test_determinism(gpu_lib):
    n = 100_000
    X = seed_spreader_3d(n, domain=1e5 * (n / 1e6) ** (1 / 3), seed=207)
    ref = gpu_dbscan(X, 150.0, 10, tag="determinism 0")
    for r in range(1, 6):
        got = gpu_dbscan(X, 150.0, 10, tag=f"determinism {r}")
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


_WORKLOAD_CACHE: dict = {}


def _workload_cached(config, scale):
    key = (config, scale)
    if key not in _WORKLOAD_CACHE:
        _WORKLOAD_CACHE.clear()  # one full-size workload in host memory at a time
        _WORKLOAD_CACHE[key] = config_workload(config, scale)
    return _WORKLOAD_CACHE[key]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("name", sorted(k for k, v in full_size_cases().items() if "eps" in v))
def test_full_size_against_oracle_hash(name, mode, gpu_lib):
    """One dbscan() call per oracle hash (the batched launch configuration is in
    test_gpu_full_size_hashes.py)."""
    case = full_size_cases()[name]
    X = _workload_cached(case["config"], case["scale"])[case.get("instance", 0)].X
    assert len(X) == case["n"]
    core, lab = gpu_dbscan(X, case["eps"], case["min_pts"], mode=mode, tag=name)
    summary = {
        "n_core": int(core.sum()),
        "n_noise": int((lab < 0).sum()),
        "n_clusters": int(len(np.unique(lab[core.astype(bool)]))),
    }
    assert summary == {k: case[k] for k in summary}, (summary, case)
    assert digest(core, lab) == case["sha256"]


def _set_opts(**kw):
    from paper_1912_06255_amd import binding

    for k, v in kw.items():
        binding.set_option(k, v)


@pytest.mark.parametrize("d", [2, 3, 5, 7])
def test_filter_forced_recheck_equals_plain(d, gpu_lib):
    """With every pair sent to the float64 recheck the filter path must equal plain."""
    rng = np.random.Generator(np.random.PCG64(301 + d))
    X = gaussian_mixture(6000, d, 10, 1.0, 12.0, 0.05, rng)
    eps = 1.2 if d <= 3 else 2.0
    plain, st0 = gpu_dbscan(X, eps, 8, mode="fp64", tag=f"plain d={d}", want_stats=True)
    try:
        _set_opts(force_recheck=1, filter_max_d=8)
        forced, st1 = gpu_dbscan(X, eps, 8, mode="fp32_filter", tag=f"forced d={d}", want_stats=True)
    finally:
        _set_opts(force_recheck=0, filter_max_d=-1)
    assert st1["fp64_rechecks"] > 0
    assert np.array_equal(plain[0], forced[0]) and np.array_equal(plain[1], forced[1])


def test_filter_rechecks_exact_boundaries(gpu_lib):
    """Integer lattice with eps = 1: every axis pair sits exactly at eps, so the
    float32 band must send them to float64 and the result must stay exact."""
    rng = np.random.Generator(np.random.PCG64(302))
    P = rng.integers(0, 40, size=(30000, 3)).astype(np.float64)
    want = dbscan_o1(P, 1.0, 4)
    got, st = gpu_dbscan(P, 1.0, 4, mode="fp32_filter", tag="lattice filter", want_stats=True)
    assert st["fp64_rechecks"] > 0, st
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


@pytest.mark.parametrize("mode", MODES)
def test_exact_boundaries_4d_lattice(mode, gpu_lib):
    """4D integer lattice with eps = 1: most neighbour pairs sit exactly at eps."""
    rng = np.random.Generator(np.random.PCG64(305))
    P = rng.integers(0, 12, size=(12000, 4)).astype(np.float64)
    _assert_parity(P, 1.0, 6, mode, "4d lattice")


_SUB_RESET = dict(fine_bits=-1, subcell_min=-1)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("eps,mp,opts", [
    (400.0, 100, dict(fine_bits=2)), (800.0, 1000, dict(fine_bits=2)),
    (400.0, 400, dict(fine_bits=1)), (400.0, 400, dict(fine_bits=3)),
    (200.0, 60, dict(fine_bits=2)), (120.0, 30, dict(fine_bits=2)),
    (400.0, 100, dict(subcell_min=2)), (800.0, 1000, dict(subcell_min=2)),
    (200.0, 60, dict(subcell_min=2)), (800.0, 300, dict(subcell_min=-1)),
    (800.0, 300, dict(subcell_min=0))])
def test_sub_cell_order_large_cells(eps, mp, opts, mode, gpu_lib):
    """Sub-cell order over cells of hundreds to thousands of points (several walks,
    5% noise), from sort-time fine bits or regrouped after the grid is built:
    MarkCore counts whole chunks whose box lies within eps and skips far ones,
    ClusterCore prunes chunk pairs by their boxes; the labels must not change."""
    X = seed_spreader_3d(30_000, domain=3e4, restart=0.03, noise_frac=0.05, seed=306)
    try:
        _set_opts(**opts)
        _assert_parity(X, eps, mp, mode, f"sub-cell {opts} eps={eps} mp={mp}")
    finally:
        _set_opts(**_SUB_RESET)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("opts", [dict(fine_bits=2), dict(subcell_min=2)])
def test_sub_cell_order_exact_boundaries(opts, mode, gpu_lib):
    """Integer lattice with about 60 copies of each site and eps = 3: many pairs and
    chunk-box corners sit exactly at eps, where a whole chunk may be counted only if
    every one of its points passes the float64 test.  minPts is above every cell's
    size, so every count comes from the neighbour walk."""
    rng = np.random.Generator(np.random.PCG64(307))
    P = rng.integers(0, 10, size=(60000, 3)).astype(np.float64)
    try:
        _set_opts(**opts)
        for mp in (3000, 5000):
            _assert_parity(P, 3.0, mp, mode, f"lattice sub-cell {opts} mp={mp}")
    finally:
        _set_opts(**_SUB_RESET)


# Above 3 dimensions: Gaussian clusters tight enough for cells of hundreds of points
# (d, n, components, sigma, spread, eps, minPts values).  The larger minPts sits near
# the component sizes, so that core and non-core points mix and the counts through
# whole chunks decide.
_HD_SUB = [
    (4, 30_000, 4, 0.5, 15.0, 1.5, (10, 4000)),
    (5, 30_000, 4, 0.4, 20.0, 2.0, (10, 6800)),
    (7, 20_000, 3, 0.4, 15.0, 2.5, (10, 6200)),
    (8, 16_000, 2, 0.4, 12.0, 3.0, (10, 7400)),
]
_HD_SUB_WANT = {}


def _hd_sub_case(i):
    d, n, k, sig, spread, eps, mps = _HD_SUB[i]
    rng = np.random.Generator(np.random.PCG64(900 + d))
    X = gaussian_mixture(n, d, k, sig, spread, 0.05, rng)
    for mp in mps:
        if (i, mp) not in _HD_SUB_WANT:
            _HD_SUB_WANT[(i, mp)] = dbscan_o1(X, eps, mp)
    return X, eps, mps


@pytest.mark.parametrize("mode,filter_max_d", [("fp64", -1), ("fp32_filter", 8)])
@pytest.mark.parametrize("opts", [dict(subcell_min=2), dict(subcell_min=512, bcp_rounds=0),
                                  dict(subcell_min=2, bcp_rounds=1, unit_level=0)])
@pytest.mark.parametrize("case", range(len(_HD_SUB)))
def test_sub_cell_order_high_d(case, opts, mode, filter_max_d, gpu_lib):
    """Sub-cell order above 3 dimensions: the coordinates regrouped one dimension at
    a time, and MarkCore and ClusterCore kernels of their own with the chunk-box
    paths, in float64 and with the float32 filter taking the decisions."""
    X, eps, mps = _hd_sub_case(case)
    d = X.shape[1]
    try:
        _set_opts(filter_max_d=filter_max_d, **opts)
        for mp in mps:
            tag = f"{d}d sub-cell {opts} {mode} eps={eps} mp={mp}"
            want = _HD_SUB_WANT[(case, mp)]
            got = gpu_dbscan(X, eps, mp, mode=mode, tag=tag)
            assert np.array_equal(got[0], want[0]), f"{tag}: core flags differ"
            assert np.array_equal(got[1], want[1]), f"{tag}: labels differ"
    finally:
        _set_opts(filter_max_d=-1, bcp_rounds=-1, unit_level=-1, **_SUB_RESET)


@pytest.mark.parametrize("opts", [dict(bcp_rounds=0), dict(bcp_rounds=1, unit_level=0),
                                  dict(bcp_rounds=1, unit_level=1), dict(bcp_rounds=1, unit_level=2),
                                  dict(fine_bits=3), dict(fine_bits=0), dict(bcp_split=1),
                                  dict(bcp_split=4), dict(bcp_split=2, bcp_rounds=1),
                                  dict(sparse=0, bcp_rounds=1, unit_level=2),
                                  dict(sparse=0, bcp_rounds=0), dict(sparse=1),
                                  dict(mark_split=1), dict(mark_split=2), dict(mark_split=8),
                                  dict(dense_group=1), dict(dense_group=64)])
@pytest.mark.parametrize("mode", MODES)
def test_tuning_options_do_not_change_results(opts, mode, gpu_lib):
    n = 40_000
    X = seed_spreader_3d(n, domain=1e5 * (n / 1e6) ** (1 / 3), seed=303)
    rng = np.random.Generator(np.random.PCG64(304))
    Y = gaussian_mixture(8000, 5, 10, 1.0, 12.0, 0.05, rng)
    # dense 2D blobs: hundreds of points per cell, so MarkCore splits its cells over
    # waves and ClusterCore takes groups cell by cell
    Z = gaussian_mixture(20_000, 2, 4, 1.0, 40.0, 0.0, rng)  # 59 points per cell at eps 1
    wantX = dbscan_o1(X, 200.0, 10)
    wantY = dbscan_o1(Y, 2.0, 10)
    wantZ = dbscan_o1(Z, 1.0, 400)  # 87 % core, 4 clusters
    try:
        _set_opts(**opts)
        gx = gpu_dbscan(X, 200.0, 10, mode=mode, tag=f"opts {opts} 3d")
        gy = gpu_dbscan(Y, 2.0, 10, mode=mode, tag=f"opts {opts} 5d")
        gz = gpu_dbscan(Z, 1.0, 400, mode=mode, tag=f"opts {opts} dense 2d")
    finally:
        _set_opts(bcp_rounds=-1, unit_level=1, fine_bits=-1, bcp_split=-1, sparse=-1,
                  mark_split=-1, dense_group=-1)
    assert np.array_equal(gx[0], wantX[0]) and np.array_equal(gx[1], wantX[1])
    assert np.array_equal(gy[0], wantY[0]) and np.array_equal(gy[1], wantY[1])
    assert np.array_equal(gz[0], wantZ[0]) and np.array_equal(gz[1], wantZ[1])


def test_option_ranges(gpu_lib):
    """Out-of-range option values are refused and leave the option unchanged."""
    from paper_1912_06255_amd import binding

    bad = {"bcp_rounds": [2, -2], "unit_level": [-2, 6], "fine_bits": [-2, 9],
           "force_recheck": [2], "batch_graph": [-1], "bcp_split": [0, 65],
           "filter_max_d": [-2, 9], "subcell_min": [-2, 1], "sparse": [-2, 2],
           "group_clouds": [-2, 2], "mark_split": [0, 3, 16], "dense_group": [0, 65],
           "cells": [-2, 2]}
    for name, values in bad.items():
        before = binding.get_option(name)
        for v in values:
            with pytest.raises(binding.DbscanError):
                binding.set_option(name, v)
            assert binding.get_option(name) == before, name
    binding.set_option("subcell_min", 2)
    assert binding.get_option("subcell_min") == 2
    binding.set_option("subcell_min", -1)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("sparse", [0, 1])
@pytest.mark.parametrize("d", [2, 3, 5, 7])
def test_sparse_kernels_match_oracle(d, sparse, mode, gpu_lib):
    """MarkCore, ClusterCore and ClusterBorder batched over 64 consecutive cells per
    tree walk (sparse = 1) and one cell per wave (sparse = 0), on the same clouds:
    eps small against the spread (about one point per cell) and larger (tens of
    points per cell), with ragged sizes and noise; the float32 filter takes the
    decisions in every dimension in filter mode."""
    rng = np.random.Generator(np.random.PCG64(910 + d))
    n = {2: 7001, 3: 9003, 5: 6007, 7: 5003}[d]
    X = gaussian_mixture(n, d, 12, 1.0, 15.0, 0.05, rng)
    cases = [(0.45, 3), (0.45, 10), (1.6, 10)] if d <= 3 else [(1.0, 5), (2.0, 10), (3.0, 20)]
    try:
        _set_opts(sparse=sparse, filter_max_d=8)
        for eps, mp in cases:
            (got, st) = gpu_dbscan(X, eps, mp, mode=mode, tag=f"sparse={sparse} d={d} eps={eps}",
                                   want_stats=True)
            want = dbscan_o1(X, eps, mp)
            assert np.array_equal(got[0], want[0]), (d, eps, mp, "core")
            assert np.array_equal(got[1], want[1]), (d, eps, mp, "labels")
    finally:
        _set_opts(sparse=-1, filter_max_d=-1)
