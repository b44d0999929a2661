"""Grouped batches: single-setting clouds of one dimension sharing every kernel launch
(ManyWork), against the oracle and against the same batch run one cloud at a time."""

import numpy as np
import pytest

from oracle import dbscan_o1
from tests.gpu_helpers import gpu_dbscan, log
from workloads import gaussian_mixture, multi_cloud_batch, seed_spreader_3d

pytestmark = pytest.mark.gpu


def _set(**opts):
    from paper_1912_06255_amd import binding

    for k, v in opts.items():
        binding.set_option(k, v)


def _mixed_case():
    """Clouds of d = 2, 3 and 5 with one setting each (ragged sizes from 1 point to
    several sort tiles, an empty cloud, a cloud of identical points), interleaved
    with clouds of several settings, which take the one-cloud path."""
    rng = np.random.Generator(np.random.PCG64(731))
    clouds, settings = [], []

    def add(X, st):
        clouds.append(np.ascontiguousarray(X, dtype=np.float64))
        settings.append(st)

    add(gaussian_mixture(9000, 2, 6, 0.5, 10.0, 0.05, rng), [(0.3, 4)])
    add(rng.uniform(0, 1, (1, 2)), [(0.5, 1)])
    add(rng.uniform(0, 1, (2, 2)), [(0.5, 2)])
    add(gaussian_mixture(63, 2, 2, 0.2, 3.0, 0.1, rng), [(0.2, 3)])
    add(gaussian_mixture(4097, 2, 3, 0.3, 5.0, 0.05, rng), [(0.25, 5)])
    add(np.zeros((0, 2)), [(1.0, 3)])
    add(np.full((300, 2), 2.5), [(0.1, 10)])
    n = 20_000
    add(seed_spreader_3d(n, domain=1e5 * (n / 1e6) ** (1 / 3), seed=732), [(200.0, 10)])
    add(seed_spreader_3d(5000, domain=1e5 * (5000 / 1e6) ** (1 / 3), seed=733),
        [(200.0, 5), (400.0, 20)])  # two settings: not grouped
    add(gaussian_mixture(7000, 3, 5, 1.0, 20.0, 0.1, rng), [(0.6, 8)])
    add(gaussian_mixture(65, 3, 2, 0.5, 4.0, 0.0, rng), [(0.7, 2)])
    add(gaussian_mixture(6000, 5, 6, 1.0, 10.0, 0.05, rng), [(1.5, 10)])
    add(gaussian_mixture(3000, 5, 4, 1.0, 10.0, 0.05, rng), [(2.0, 5)])
    add(gaussian_mixture(2500, 5, 4, 1.0, 10.0, 0.05, rng), [(1.0, 5), (1.0, 20)])
    return clouds, settings


def _batch(clouds, settings, mode):
    import torch

    from paper_1912_06255_amd import binding

    return binding.Batch([torch.from_numpy(X).to("cuda") for X in clouds], settings, mode=mode)


def _check(b, clouds, settings, tag, want=None):
    for i, (X, st) in enumerate(zip(clouds, settings)):
        for s, (eps, mp) in enumerate(st):
            w = want[i][s] if want is not None else dbscan_o1(X, eps, mp)
            core = b.core[i][s].cpu().numpy()
            lab = b.label[i][s].cpu().numpy()
            assert np.array_equal(core, w[0]), f"{tag}: cloud {i} (n={len(X)}) setting {s} core"
            assert np.array_equal(lab, w[1]), f"{tag}: cloud {i} (n={len(X)}) setting {s} labels"


def _oracle(clouds, settings):
    return [[dbscan_o1(X, e, m) for e, m in st] for X, st in zip(clouds, settings)]


@pytest.mark.parametrize("mode,filter_max_d", [("fp64", -1), ("fp32_filter", -1), ("fp32_filter", 8)])
def test_grouped_batch_matches_oracle(mode, filter_max_d, gpu_lib):
    """Every grouping (automatic, every single-setting cloud, none), captured and
    replayed, eager, and profiled (eager with phase events) gives the oracle's
    result for every cloud."""
    from paper_1912_06255_amd import binding

    clouds, settings = _mixed_case()
    want = _oracle(clouds, settings)
    try:
        for group in (-1, 1, 0):
            _set(group_clouds=group, filter_max_d=filter_max_d)
            b = _batch(clouds, settings, mode)
            for r in range(2):
                for c, l in zip(b.core, b.label):
                    c.fill_(7)
                    l.fill_(-7)
                log(f"grouped batch mode={mode} filter_max_d={filter_max_d} group={group} run {r}")
                b.run()
                _check(b, clouds, settings, f"group={group} run {r}", want)
        _set(group_clouds=1, batch_graph=0)
        b = _batch(clouds, settings, mode)
        log(f"grouped batch eager mode={mode}")
        b.run()
        _check(b, clouds, settings, "eager", want)
        binding.set_profiling(True)
        log(f"grouped batch profiled mode={mode}")
        b.run()
        _check(b, clouds, settings, "profiled", want)
        ph = binding.phase_stats()
        assert ph["markcore"][0] > 0.0 and ph["border"][1] >= 1
    finally:
        binding.set_profiling(False)
        _set(group_clouds=-1, filter_max_d=-1, batch_graph=1)


def test_grouped_batch_after_a_larger_single_call(gpu_lib):
    """A single call whose arrays reach into the group area is followed by the
    grouped batch again: its tables and descriptors are laid out anew (the captured
    graph is dropped), and the results stay exact."""
    clouds, settings = _mixed_case()
    want = _oracle(clouds, settings)
    b = _batch(clouds, settings, "fp32_filter")
    log("grouped batch before a large single call")
    b.run()
    _check(b, clouds, settings, "before", want)
    rng = np.random.Generator(np.random.PCG64(741))
    Y = gaussian_mixture(400_000, 3, 20, 1.0, 60.0, 0.05, rng)
    got = gpu_dbscan(Y, 0.8, 10, mode="fp32_filter", tag="large single call between batches")
    w = dbscan_o1(Y, 0.8, 10)
    assert np.array_equal(got[0], w[0]) and np.array_equal(got[1], w[1])
    for r in range(2):
        log(f"grouped batch after the large call, run {r}")
        b.run()
        _check(b, clouds, settings, f"after {r}", want)


def test_grouped_batch_reports_nonfinite(gpu_lib):
    """A non-finite coordinate in one grouped cloud fails the batch; the next clean
    batch on the same context succeeds (the status is cleared again)."""
    from paper_1912_06255_amd import binding

    clouds, settings = _mixed_case()
    bad = [X.copy() for X in clouds]
    bad[4][17, 1] = np.nan
    b = _batch(bad, settings, "fp64")
    log("grouped batch with a NaN")
    with pytest.raises(binding.DbscanError) as e:
        b.run()
    assert e.value.code == binding.ENONFINITE
    ok = _batch(clouds, settings, "fp64")
    log("clean grouped batch after the failure")
    ok.run()
    _check(ok, clouds, settings, "clean after failure")


def test_grouped_multi_cloud_small(gpu_lib):
    """The 256-cloud workload at 1% size (2, 3 and 5 dimensions), grouped against
    one cloud at a time and against the oracle."""
    inst = multi_cloud_batch(n_clouds=60, size_scale=0.01)
    clouds = [i.X for i in inst]
    settings = [list(zip(i.eps, i.min_pts)) for i in inst]
    want = _oracle(clouds, settings)
    try:
        for group in (-1, 0):
            _set(group_clouds=group)
            b = _batch(clouds, settings, "fp32_filter")
            log(f"multi-cloud 60 clouds group={group}")
            b.run()
            b.run()
            _check(b, clouds, settings, f"multi-cloud group={group}", want)
    finally:
        _set(group_clouds=-1)
