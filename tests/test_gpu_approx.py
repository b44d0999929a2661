"""Approximate DBSCAN on the GPU (dbscan_approx) against the relaxed definition
(oracle/approx.py: Gan and Tao's approximate DBSCAN in the paper's preliminaries),
whose output is not unique: every output must pass the checker, rho = 0 must give
the exact output, and an approximate clustering can only merge exact clusters."""

import numpy as np
import pytest

from oracle import check_approx, dbscan_o1
from tests.gpu_helpers import log
from workloads import blobs_2d, gaussian_mixture, seed_spreader_3d

pytestmark = pytest.mark.gpu

MODES = ["fp64", "fp32_filter"]


def _cases():
    rng = np.random.Generator(np.random.PCG64(601))
    n = 15_000
    yield "blobs", blobs_2d(6000, seed=602), 100.0, 10
    yield "spreader", seed_spreader_3d(n, domain=1e5 * (n / 1e6) ** (1 / 3), seed=603), 200.0, 10
    yield "mixture5", gaussian_mixture(6000, 5, 10, 1.0, 12.0, 0.05, rng), 2.0, 10
    yield "lattice", rng.integers(0, 25, size=(8000, 3)).astype(np.float64), 1.0, 4


CASES = list(_cases())


def _approx(X, eps, mp, rho, mode):
    import torch

    from paper_1912_06255_amd import binding

    log(f"approx n={X.shape[0]} d={X.shape[1]} eps={eps} mp={mp} rho={rho} mode={mode}")
    core, lab = binding.dbscan(torch.from_numpy(X).cuda(), eps, mp, mode=mode, rho=rho)
    return core.cpu().numpy(), lab.cpu().numpy()


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("rho", [0.01, 0.1, 0.5])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_approx_output_is_valid(case, rho, mode, gpu_lib):
    name, X, eps, mp = CASES[case]
    core, lab = _approx(X, eps, mp, rho, mode)
    fails = check_approx(X, eps, mp, rho, core, lab)
    assert not fails, f"{name} rho={rho}: {fails}"
    # approximate clusters are unions of exact ones
    want = dbscan_o1(X, eps, mp)
    c = want[0].astype(bool)
    exact_ids = np.unique(want[1][c]).size
    got_ids = np.unique(lab[c]).size
    assert got_ids <= exact_ids
    log(f"{name} rho={rho} {mode}: {exact_ids} exact clusters, {got_ids} approximate")


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("case", range(len(CASES)))
def test_rho_zero_is_exact(case, mode, gpu_lib):
    name, X, eps, mp = CASES[case]
    got = _approx(X, eps, mp, 0.0, mode)
    want = dbscan_o1(X, eps, mp)
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1]), name


def test_bad_rho_is_refused(gpu_lib):
    import torch

    from paper_1912_06255_amd import binding

    X = torch.zeros((4, 2), dtype=torch.float64, device="cuda")
    for rho in (-0.1, float("nan"), float("inf"), 1e200):
        with pytest.raises(binding.DbscanError) as e:
            binding.dbscan(X, 1.0, 2, rho=rho)
        assert e.value.code == binding.EINVAL


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("rho", [0.1, 0.5])
def test_approx_through_sub_cell_order(rho, mode, gpu_lib):
    """Large cells in sub-cell order, so ClusterCore takes its leaf path (chunk-box
    pruning at the relaxed radius); the output must still pass the checker."""
    from paper_1912_06255_amd import binding

    X = seed_spreader_3d(8000, domain=1.5e4, restart=0.03, noise_frac=0.05, seed=604)
    try:
        binding.set_option("subcell_min", 2)
        core, lab = _approx(X, 400.0, 100, rho, mode)
    finally:
        binding.set_option("subcell_min", -1)
    fails = check_approx(X, 400.0, 100, rho, core, lab)
    assert not fails, fails


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("d", [1, 8])
def test_approx_extreme_dimensions(d, mode, gpu_lib):
    rng = np.random.Generator(np.random.PCG64(605 + d))
    X = gaussian_mixture(3000, d, 6, 1.0, 10.0, 0.05, rng)
    eps = 0.3 if d == 1 else 2.5
    for rho in (0.0, 0.3):
        core, lab = _approx(X, eps, 8, rho, mode)
        fails = check_approx(X, eps, 8, rho, core, lab)
        assert not fails, f"d={d} rho={rho}: {fails}"


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("rho", [0.1, 0.5])
def test_approx_through_sparse_kernels(rho, mode, gpu_lib):
    """ClusterCore at radius eps (1 + rho) in the batched sparse kernels (forced on
    for 2D and 3D clouds), checked against the relaxed definition."""
    from paper_1912_06255_amd import binding

    for case in (0, 3):
        name, X, eps, mp = CASES[case]
        binding.set_option("sparse", 1)
        try:
            core, lab = _approx(X, eps, mp, rho, mode)
        finally:
            binding.set_option("sparse", -1)
        fails = check_approx(X, eps, mp, rho, core, lab)
        assert not fails, f"{name} sparse rho={rho}: {fails}"
