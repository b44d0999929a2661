"""Batches of clouds and settings (one captured HIP graph) against the oracle."""

import numpy as np
import pytest

from oracle import dbscan_o1
from tests.gpu_helpers import gpu_dbscan, log
from workloads import gaussian_mixture, multi_cloud_batch, seed_spreader_3d

pytestmark = pytest.mark.gpu


def _batch(clouds, settings, mode):
    import torch

    from paper_1912_06255_amd import binding

    return binding.Batch([torch.from_numpy(X).to("cuda") for X in clouds], settings, mode=mode)


def _mismatch(core, lab, want):
    """A short description of how a result differs from the oracle's."""
    bad = np.flatnonzero(lab != want[1])
    wc = want[0].astype(bool)
    return (f"{bad.size} labels differ ({int(wc[bad].sum())} at core points), first at "
            f"{bad[:5].tolist()}: got {lab[bad[:5]].tolist()} want {want[1][bad[:5]].tolist()}; "
            f"clusters got {len(np.unique(lab[core.astype(bool)]))} want {len(np.unique(want[1][wc]))}")


def _check_batch(b, clouds, settings, tag):
    for i, (X, st) in enumerate(zip(clouds, settings)):
        for s, (eps, mp) in enumerate(st):
            want = dbscan_o1(X, eps, mp)
            core = b.core[i][s].cpu().numpy()
            lab = b.label[i][s].cpu().numpy()
            assert np.array_equal(core, want[0]), f"{tag}: cloud {i} setting {s} core"
            assert np.array_equal(lab, want[1]), \
                f"{tag}: cloud {i} setting {s} labels: {_mismatch(core, lab, want)}"


def _clouds():
    rng = np.random.Generator(np.random.PCG64(401))
    n = 30_000
    A = seed_spreader_3d(n, domain=1e5 * (n / 1e6) ** (1 / 3), seed=402)
    B = gaussian_mixture(5000, 2, 8, 0.5, 10.0, 0.05, rng)
    C = gaussian_mixture(4000, 5, 6, 1.0, 10.0, 0.05, rng)
    E = np.zeros((0, 3))
    settings = [
        [(200.0, 5), (200.0, 10), (400.0, 50), (200.0, 100), (400.0, 5)],
        [(0.3, 4)],
        [(1.5, 10), (2.0, 10)],
        [(1.0, 3)],
    ]
    return [A, B, C, E], settings


@pytest.mark.parametrize("mode,filter_max_d", [("fp64", -1), ("fp32_filter", -1), ("fp32_filter", 8)])
def test_batch_matches_oracle(mode, filter_max_d, gpu_lib):
    from paper_1912_06255_amd import binding

    clouds, settings = _clouds()
    binding.set_option("filter_max_d", filter_max_d)
    try:
        b = _batch(clouds, settings, mode)
        log(f"batch mode={mode} filter_max_d={filter_max_d} clouds={len(clouds)}")
        b.run()
        _check_batch(b, clouds, settings, f"batch {mode}")
    finally:
        binding.set_option("filter_max_d", -1)


@pytest.mark.parametrize("mode", ["fp64", "fp32_filter"])
def test_graph_replays_match_eager(mode, gpu_lib):
    """Replay the captured graph several times with eager work between replays;
    every replay must equal the eager (uncaptured) batch."""
    import torch

    from paper_1912_06255_amd import binding

    clouds, settings = _clouds()
    b = _batch(clouds, settings, mode)
    binding.set_option("batch_graph", 0)
    try:
        log(f"eager batch mode={mode}")
        b.run()
        ref = [(c.clone(), l.clone()) for c, l in zip(b.core, b.label)]
    finally:
        binding.set_option("batch_graph", 1)
    rng = np.random.default_rng(5)
    for r in range(4):
        for c, l in zip(b.core, b.label):
            c.fill_(7)
            l.fill_(-7)
        log(f"graph replay {r} mode={mode}")
        b.run()
        for (c, l), (rc, rl) in zip(zip(b.core, b.label), ref):
            assert torch.equal(c, rc) and torch.equal(l, rl), f"replay {r} differs"
        # eager work on the same context between replays
        Y = rng.uniform(0, 10, (3000, 2))
        got = gpu_dbscan(Y, 0.4, 5, mode=mode, tag=f"eager between replays {r}")
        want = dbscan_o1(Y, 0.4, 5)
        assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
        torch.cuda.synchronize()


def test_batch_recaptures_when_description_changes(gpu_lib):
    clouds, settings = _clouds()
    b1 = _batch(clouds[:2], settings[:2], "fp32_filter")
    b2 = _batch(clouds[2:], settings[2:], "fp32_filter")
    for r in range(2):
        log(f"alternate batches {r}")
        b1.run()
        _check_batch(b1, clouds[:2], settings[:2], "b1")
        b2.run()
        _check_batch(b2, clouds[2:], settings[2:], "b2")


def test_multi_cloud_batch_small(gpu_lib):
    inst = multi_cloud_batch(n_clouds=40, size_scale=0.01)
    clouds = [i.X for i in inst]
    settings = [list(zip(i.eps, i.min_pts)) for i in inst]
    b = _batch(clouds, settings, "fp32_filter")
    log("multi-cloud batch 40 clouds")
    b.run()
    b.run()
    _check_batch(b, clouds, settings, "multi-cloud")


def _many_minpts_case():
    rng = np.random.Generator(np.random.PCG64(411))
    n = 30_000
    A = seed_spreader_3d(n, domain=1e5 * (n / 1e6) ** (1 / 3), seed=412)
    B = gaussian_mixture(4000, 5, 6, 1.0, 10.0, 0.05, rng)
    # dense 2D blobs: cells of hundreds of points (sub-cell order from 256 points)
    Cd = gaussian_mixture(20_000, 2, 3, 1.0, 10.0, 0.05, rng)
    settings = [
        # ten settings of one eps (more than one group of eight), a repeated minPts
        [(200.0, m) for m in (3, 5, 8, 10, 15, 20, 30, 50, 100, 10)] + [(400.0, 5), (400.0, 50)],
        [(1.5, m) for m in (2, 5, 10, 20)],
        [(3.0, m) for m in (5, 50, 500, 1000)],
    ]
    return [A, B, Cd], settings


@pytest.mark.parametrize("mode", ["fp64", "fp32_filter"])
@pytest.mark.parametrize("rounds,sparse", [(-1, -1), (1, -1), (-1, 1), (1, 1)])
def test_batch_many_minpts_per_eps(mode, rounds, sparse, gpu_lib):
    """Settings of one eps share their grid: they are taken by decreasing minPts,
    each ClusterCore starting from the union-find the previous one left, with the
    core flags of all of them set at once and their outputs written together in
    input order.  Covers more settings than one group holds, a repeated minPts, both
    ClusterCore schedules (one pass, rounds), d = 2, 3, 5, and large cells in
    sub-cell order (the inverse permutation of the outputs follows the regrouping)."""
    from paper_1912_06255_amd import binding

    clouds, settings = _many_minpts_case()
    binding.set_option("bcp_rounds", rounds)
    binding.set_option("subcell_min", 256)
    binding.set_option("sparse", sparse)
    tag = f"{mode} rounds={rounds} sparse={sparse}"
    try:
        b = _batch(clouds, settings, mode)
        log(f"many-minPts batch {tag}")
        b.run()
        _check_batch(b, clouds, settings, f"many minPts {tag}")
        b.run()  # graph replay
        _check_batch(b, clouds, settings, f"many minPts replay {tag}")
    finally:
        binding.set_option("bcp_rounds", -1)
        binding.set_option("subcell_min", -1)
        binding.set_option("sparse", -1)


@pytest.mark.parametrize("mode,filter_max_d", [("fp64", -1), ("fp32_filter", 8)])
def test_batch_sub_cell_order_high_d(mode, filter_max_d, gpu_lib):
    """Sub-cell order above 3 dimensions in a batch: settings of one eps (the warm
    ClusterCore kernel), an eps twice as large (a grid cut from the finer one's
    keys, regrouped again), and a 7D cloud; captured and replayed."""
    from paper_1912_06255_amd import binding

    rng = np.random.Generator(np.random.PCG64(905))
    A = gaussian_mixture(30_000, 5, 4, 0.4, 20.0, 0.05, rng)
    B = gaussian_mixture(20_000, 7, 3, 0.4, 15.0, 0.05, rng)
    clouds = [A, B]
    settings = [[(2.0, 6800), (2.0, 1000), (2.0, 10), (4.0, 7000), (1.0, 50)],
                [(2.5, 6200), (2.5, 10)]]
    binding.set_option("subcell_min", 2)
    binding.set_option("filter_max_d", filter_max_d)
    try:
        b = _batch(clouds, settings, mode)
        for r in range(2):
            log(f"high-d sub-cell batch {mode} run {r}")
            b.run()
            _check_batch(b, clouds, settings, f"high-d sub-cell {mode} run {r}")
    finally:
        binding.set_option("subcell_min", -1)
        binding.set_option("filter_max_d", -1)


def test_batch_invalid_arguments(gpu_lib):
    import torch

    from paper_1912_06255_amd import binding

    X = torch.zeros((10, 2), dtype=torch.float64, device="cuda")
    for st in ([(0.0, 3)], [(1.0, 0)], [(float("nan"), 2)]):
        b = binding.Batch([X], [st], mode="fp64")
        with pytest.raises(binding.DbscanError) as e:
            b.run()
        assert e.value.code == binding.EINVAL
