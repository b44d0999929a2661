"""The box method's cells in two dimensions (section "Box Computation"): strips by x,
boxes by y, both cut by binary search and pointer jumping.  The DBSCAN result is
unique, so it must equal the oracle's bit for bit whatever the cells; the cell
counts show that the boxes, not the grid, were used."""

import numpy as np
import pytest

from oracle import dbscan_o1
from tests.gpu_helpers import gpu_dbscan, log
from workloads import gaussian_mixture, seed_spreader_3d

pytestmark = pytest.mark.gpu

MODES = ["fp64", "fp32_filter"]


def _set(**opts):
    from paper_1912_06255_amd import binding

    for k, v in opts.items():
        binding.set_option(k, v)


def _cases():
    """(name, points, eps, minPts values)."""
    rng = np.random.Generator(np.random.PCG64(951))
    out = [
        ("mixture", gaussian_mixture(20_000, 2, 6, 0.5, 10.0, 0.05, rng), 0.3, (4, 30)),
        # integer sites with many copies: ties in x and in y everywhere, and strip and
        # box starts that coincide with whole groups of equal coordinates
        ("lattice", rng.integers(0, 30, size=(20_000, 2)).astype(np.float64), 1.5, (20, 60)),
        ("lattice fine", rng.integers(0, 200, size=(30_000, 2)).astype(np.float64) * 0.25,
         0.25 * np.sqrt(2.0), (2, 5)),
        # negative and large coordinates
        ("wide", rng.uniform(-1e6, 1e6, size=(30_000, 2)), 2e4, (3, 8)),
        # one strip (all x equal) and one row (all y equal)
        ("one strip", np.column_stack([np.full(5000, 3.0), rng.uniform(0, 100, 5000)]), 0.5, (2, 4)),
        ("one row", np.column_stack([rng.uniform(0, 100, 5000), np.full(5000, -7.0)]), 0.5, (2, 4)),
        ("single", np.array([[1.0, 2.0]]), 1.0, (1, 2)),
        ("pair", np.array([[0.0, 0.0], [0.5, 0.5]]), 1.0, (1, 2, 3)),
        ("ragged", gaussian_mixture(4097, 2, 3, 0.3, 5.0, 0.05, rng), 0.2, (3, 10)),
        ("small", gaussian_mixture(65, 2, 2, 0.2, 3.0, 0.1, rng), 0.3, (2, 3)),
    ]
    return out


_CASES = _cases()
_WANT = {}


def _want(i, mp):
    name, X, eps, _ = _CASES[i]
    if (i, mp) not in _WANT:
        _WANT[(i, mp)] = dbscan_o1(X, eps, mp)
    return _WANT[(i, mp)]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("case", range(len(_CASES)))
def test_box_cells_match_oracle(case, mode, gpu_lib):
    name, X, eps, mps = _CASES[case]
    try:
        for mp in mps:
            _set(cells=1)
            tag = f"box cells {name} n={len(X)} eps={eps} mp={mp} {mode}"
            got, st = gpu_dbscan(X, eps, mp, mode=mode, tag=tag, want_stats=True)
            want = _want(case, mp)
            assert np.array_equal(got[0], want[0]), f"{tag}: core flags differ"
            assert np.array_equal(got[1], want[1]), f"{tag}: labels differ"
            assert 1 <= st["n_cells"] <= len(X), st
    finally:
        _set(cells=0)


def test_box_cells_are_boxes(gpu_lib):
    """The box method cuts other cells than the grid (fewer here: a box starts at a
    point, not at a fixed grid line), with the same result; the option reads back."""
    from paper_1912_06255_amd import binding

    name, X, eps, mps = _CASES[0]
    try:
        _set(cells=0)
        g, sg = gpu_dbscan(X, eps, mps[0], tag="grid cells", want_stats=True)
        _set(cells=1)
        assert binding.get_option("cells") == 1
        b, sb = gpu_dbscan(X, eps, mps[0], tag="box cells", want_stats=True)
    finally:
        _set(cells=0)
    assert binding.get_option("cells") == 0
    assert np.array_equal(g[0], b[0]) and np.array_equal(g[1], b[1])
    assert sb["n_cells"] != sg["n_cells"], (sb["n_cells"], sg["n_cells"])
    assert sb["n_cells"] < sg["n_cells"], (sb["n_cells"], sg["n_cells"])


@pytest.mark.parametrize("mode", MODES)
def test_box_cells_in_a_batch(mode, gpu_lib):
    """A batch with box cells: a 2D cloud with several minPts and a chain of eps
    values (each eps gets a grid of its own), single-setting 2D clouds (built one at
    a time, not grouped), and a 3D cloud (grid cells: the option is 2D only)."""
    import torch

    from paper_1912_06255_amd import binding

    rng = np.random.Generator(np.random.PCG64(952))
    A = gaussian_mixture(20_000, 2, 6, 0.5, 10.0, 0.05, rng)
    B = gaussian_mixture(3000, 2, 3, 0.4, 6.0, 0.05, rng)
    C = gaussian_mixture(500, 2, 2, 0.3, 3.0, 0.05, rng)
    D3 = seed_spreader_3d(10_000, domain=1e5 * (1e4 / 1e6) ** (1 / 3), seed=953)
    clouds = [A, B, C, D3]
    settings = [[(0.15, 5), (0.3, 5), (0.3, 40), (0.6, 10)], [(0.25, 4)], [(0.3, 3)], [(200.0, 10)]]
    want = [[dbscan_o1(X, e, m) for e, m in st] for X, st in zip(clouds, settings)]
    try:
        _set(cells=1)
        b = binding.Batch([torch.from_numpy(X).cuda() for X in clouds], settings, mode=mode)
        for r in range(2):
            log(f"box-cell batch {mode} run {r}")
            b.run()
            for i, st in enumerate(settings):
                for s in range(len(st)):
                    core = b.core[i][s].cpu().numpy()
                    lab = b.label[i][s].cpu().numpy()
                    assert np.array_equal(core, want[i][s][0]), f"run {r} cloud {i} setting {s} core"
                    assert np.array_equal(lab, want[i][s][1]), f"run {r} cloud {i} setting {s} labels"
    finally:
        _set(cells=0)
