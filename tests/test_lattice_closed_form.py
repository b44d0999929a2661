"""The closed form of tests/lattice_case.py against the oracle on small lattices
(the same construction the maximum-size GPU test uses at 268 million points)."""

import numpy as np
import pytest

from oracle import dbscan_brute, dbscan_o1
from tests.lattice_case import expected, lattice, points


@pytest.mark.parametrize("side,gap,seed", [(12, 5, 1), (40, 20, 2), (64, 3, 3)])
def test_closed_form_matches_oracle(side, gap, seed):
    gx, gy = lattice(seed, side, gap)
    X = points(gx, gy)
    want = expected(gx, gy, side, gap)
    for impl in (dbscan_o1, dbscan_brute):
        got = impl(X, 1.0, 5)
        assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1]), impl.__name__


def test_closed_form_has_every_kind_of_point():
    """Core, border and noise points all occur (exactly the 8 corners are noise), so
    the large test tells apart readings that would change any of them: a strict <
    at eps (every point noise), corners as border, or one cluster across the gap."""
    gx, gy = lattice(4, 20, 10)
    want_core, want_label = expected(gx, gy, 20, 10)
    assert want_core.sum() > 0 and (want_label >= 0).sum() > want_core.sum()
    assert (want_label == -1).sum() == 8  # four corners per half
    assert np.unique(want_label[want_label >= 0]).size == 2
