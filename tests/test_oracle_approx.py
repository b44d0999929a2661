"""Pins of the approximate-DBSCAN checker (oracle/approx.py) against the relaxed
definition of the paper's preliminaries (Gan and Tao): hand-worked cases where the
valid outputs are known, the exact output as a valid one, uniqueness at rho = 0, and
outputs broken in each way the definition forbids."""

import numpy as np
import pytest

from oracle import check_approx, dbscan_brute, relaxed_e2
from oracle.brute import border_labels
from workloads import blobs_2d, gaussian_mixture

# Two chains of three points on a line, all core at eps = 1, minPts = 2, with a gap
# of 1.3 between them: exactly two DBSCAN clusters, ids 0 and 3.
TWO = np.array([[0.0], [0.6], [1.2], [2.5], [3.1], [3.7]])
SEPARATE = (np.ones(6, np.uint8), np.array([0, 0, 0, 3, 3, 3], np.int32))
MERGED = (np.ones(6, np.uint8), np.zeros(6, np.int32))


def test_relaxed_radius_reading():
    assert relaxed_e2(1.0, 0.5) == 2.25
    assert relaxed_e2(1.0, 0.0) == 1.0
    assert relaxed_e2(2.0, 1.0) == 16.0


@pytest.mark.parametrize("rho,merged_ok", [(0.5, True), (0.2, False), (0.0, False)])
def test_gap_inside_and_outside_the_relaxation(rho, merged_ok):
    # the gap 1.3 is within eps(1 + rho) = 1.5 but not within 1.2 or 1
    assert check_approx(TWO, 1.0, 2, rho, *SEPARATE) == []
    assert (check_approx(TWO, 1.0, 2, rho, *MERGED) == []) == merged_ok


def test_gap_exactly_at_the_outer_radius():
    # eps (1 + rho) = 2 exactly and D = 4 = fl(2^2): the pair may join the clusters
    X = np.array([[0.0], [1.0], [3.0], [4.0]])
    merged = (np.ones(4, np.uint8), np.zeros(4, np.int32))
    assert check_approx(X, 1.0, 2, 1.0, *merged) == []
    Xf = np.array([[0.0], [1.0], [np.nextafter(3.0, 4.0)], [np.nextafter(4.0, 5.0)]])
    assert check_approx(Xf, 1.0, 2, 1.0, *merged) != []


def _datasets():
    rng = np.random.Generator(np.random.PCG64(501))
    yield blobs_2d(1500, seed=502), 100.0, 5
    yield gaussian_mixture(1200, 3, 6, 1.0, 12.0, 0.05, rng), 0.8, 6
    yield gaussian_mixture(900, 5, 5, 1.0, 10.0, 0.05, rng), 1.5, 5


@pytest.mark.parametrize("rho", [0.0, 0.01, 0.5])
def test_exact_output_is_valid(rho):
    for X, eps, mp in _datasets():
        core, lab = dbscan_brute(X, eps, mp)
        assert check_approx(X, eps, mp, rho, core, lab) == []


def _two_clusters(lab, core):
    ids = np.unique(lab[core.astype(bool)])
    assert ids.size >= 2
    return ids[0], ids[1]


def test_mutants_fail():
    X, eps, mp = next(_datasets())
    core, lab = dbscan_brute(X, eps, mp)
    c = core.astype(bool)
    a, b = _two_clusters(lab, core)
    bad = []
    # a core flag flipped
    k = core.copy(); k[np.flatnonzero(c)[0]] ^= 1
    bad.append((k, lab))
    # a cluster split: one of its core points (not the smallest) given its own id
    members = np.flatnonzero(c & (lab == a))
    l2 = lab.copy(); l2[members[1]] = members[1]
    bad.append((core, l2))
    # a non-canonical id for a whole cluster
    l3 = lab.copy(); l3[lab == a] = members[1]
    bad.append((core, l3))
    # two far clusters merged (at rho = 0 nothing beyond eps may merge)
    l4 = lab.copy(); l4[lab == b] = min(a, b)
    bad.append((core, l4))
    # a border point with a wrong id, and a noise point given an id
    border = np.flatnonzero(~c & (lab >= 0))
    if border.size:
        l5 = lab.copy(); l5[border[0]] = -1
        bad.append((core, l5))
    noise = np.flatnonzero(lab < 0)
    if noise.size:
        l6 = lab.copy(); l6[noise[0]] = a
        bad.append((core, l6))
    for k_, l_ in bad:
        assert check_approx(X, eps, mp, 0.0, k_, l_) != []


def test_unique_at_rho_zero():
    """At rho = 0 the relaxation is empty: every valid output is the exact one, so
    the checker accepts the exact output and rejects every merge of two clusters
    (with border ids recomputed for the merged clustering, as the definition asks)."""
    for X, eps, mp in _datasets():
        core, lab = dbscan_brute(X, eps, mp)
        c = core.astype(bool)
        E2 = float(np.float64(eps) * np.float64(eps))
        ids = np.unique(lab[c])
        for a, b in zip(ids[:-1], ids[1:]):
            merged = np.where(c, np.where(lab == b, a, lab), -1)
            l2 = border_labels(np.asarray(X, np.float64), c, merged, E2)
            assert check_approx(X, eps, mp, 0.0, core, l2) != []
