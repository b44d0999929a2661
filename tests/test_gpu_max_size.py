"""Near the largest supported input: 538 million points (the 23200 x 23200 lattice
without one column; above 2^29, so n times the four MarkCore waves per cell exceeds
2^31), where every 32-bit position, cell and chunk index is in its upper range.  The expected output is the closed form of tests/lattice_case.py
(pinned to the oracle on small lattices by test_lattice_closed_form.py); the oracle
itself cannot cluster this many points in test time."""

import numpy as np
import pytest

from tests.gpu_helpers import gpu_dbscan, log
from tests.lattice_case import expected, lattice, points

pytestmark = pytest.mark.gpu

SIDE = 23200
GAP = 11600


@pytest.fixture(scope="module")
def case():
    log(f"max-size lattice: building {SIDE}x{SIDE - 1} points")
    gx, gy = lattice(309, SIDE, GAP)
    X = points(gx, gy)
    want = expected(gx, gy, SIDE, GAP)
    del gx, gy
    return X, want


@pytest.mark.parametrize("mode", ["fp64", "fp32_filter"])
def test_lattice_5e8_closed_form(mode, case, gpu_lib):
    X, (want_core, want_label) = case
    (core, label), st = gpu_dbscan(X, 1.0, 5, mode=mode, tag=f"max-size lattice {mode}",
                                   want_stats=True)
    assert st["n_points"] == want_core.size
    bad_core = np.flatnonzero(core != want_core)
    assert bad_core.size == 0, f"{bad_core.size} core flags differ, first {bad_core[:5]}"
    bad = np.flatnonzero(label != want_label)
    assert bad.size == 0, f"{bad.size} labels differ, first {bad[:5]}: {label[bad[:5]]} vs {want_label[bad[:5]]}"
    if mode == "fp32_filter":
        # every neighbour pair sits exactly at eps: the float32 band sends them to float64
        assert st["fp64_rechecks"] > 0
