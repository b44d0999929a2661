"""O1 (C, bucketed candidates) must equal O0 (numpy brute force) everywhere O0 runs.

Inputs are small draws of every workload generator plus adversarial lattices where
many pairs sit exactly at eps.
"""

import numpy as np
import pytest

from oracle import dbscan_brute, dbscan_o1
from workloads import blobs_2d, gaussian_mixture, seed_spreader_3d, multi_cloud_batch


def _same(X, eps, mp):
    a = dbscan_brute(X, eps, mp)
    b = dbscan_o1(X, eps, mp)
    assert np.array_equal(a[0], b[0]), "core flags differ"
    assert np.array_equal(a[1], b[1]), "labels differ"
    return a


@pytest.mark.parametrize("mp", [1, 4, 10, 30])
def test_blobs(mp):
    X = blobs_2d(3000, seed=101)
    _same(X, 100.0, mp)


@pytest.mark.parametrize("eps,mp", [(200.0, 10), (400.0, 50), (120.0, 5)])
def test_seed_spreader(eps, mp):
    X = seed_spreader_3d(4000, domain=1e5 * (4000 / 1e6) ** (1 / 3), seed=102)
    _same(X, eps, mp)


@pytest.mark.parametrize("d", [4, 5, 7])
@pytest.mark.parametrize("eps", [1.5, 3.0])
def test_high_dim(d, eps):
    rng = np.random.Generator(np.random.PCG64(103 + d))
    X = gaussian_mixture(2500, d, 8, 1.0, 12.0, 0.05, rng)
    _same(X, eps, 10)


def test_multi_cloud_small():
    for inst in multi_cloud_batch(n_clouds=12, size_scale=0.002)[:12]:
        _same(inst.X, inst.eps[0], inst.min_pts[0])


@pytest.mark.parametrize("d", [1, 2, 3, 5])
def test_lattice_exact_boundaries(d):
    # integer lattice with eps = 1: every axis neighbour is exactly at eps
    rng = np.random.Generator(np.random.PCG64(104))
    P = rng.integers(0, 6, size=(1500, d)).astype(np.float64)
    for mp in (2, 3, 2 * d + 1):
        _same(P, 1.0, mp)


def test_empty_and_tiny():
    assert dbscan_o1(np.zeros((0, 3)), 1.0, 1)[0].shape == (0,)
    _same(np.array([[0.5, 0.5]]), 1.0, 1)
    _same(np.array([[0.5, 0.5]]), 1.0, 2)
