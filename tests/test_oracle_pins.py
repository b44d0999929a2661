"""The oracle against facts fixed outside of it (see tests/pins.py)."""

import pytest

from oracle import dbscan_brute, dbscan_o1, membership
from tests.pins import ALL_PINS, MEMBER_PINS

IMPLS = {"O0_brute": dbscan_brute, "O1_c": dbscan_o1}


@pytest.mark.parametrize("impl", sorted(IMPLS))
@pytest.mark.parametrize("pin", sorted(ALL_PINS))
def test_oracle_pin(pin, impl):
    fails = ALL_PINS[pin](IMPLS[impl])
    assert not fails, "\n".join(fails)


@pytest.mark.parametrize("pin", sorted(MEMBER_PINS))
def test_oracle_membership_pin(pin):
    fails = MEMBER_PINS[pin](membership)
    assert not fails, "\n".join(fails)


def test_membership_agrees_with_labels():
    """The smallest id of each point's set is its label; core points have exactly
    their own id; noise has none (on random clouds, against the label oracle)."""
    import numpy as np

    from workloads import blobs_2d

    for seed in (3, 4):
        X = blobs_2d(600, seed=seed)
        core, lab = dbscan_brute(X, 100.0, 8)
        off, ids = membership(X, 100.0, 8)
        for i in range(len(X)):
            s = ids[off[i]:off[i + 1]].tolist()
            assert s == sorted(set(s))
            if core[i]:
                assert s == [lab[i]]
            else:
                assert (s[0] if s else -1) == lab[i]


def test_membership_mutants_are_caught():
    """Two plausible mistakes in a membership implementation fail a pin: keeping only
    the smallest id, and letting a border point join its clusters into one."""
    import numpy as np

    def as_csr(sets):
        off = np.zeros(len(sets) + 1, np.int64)
        off[1:] = np.cumsum([len(t) for t in sets])
        return off, np.array([v for t in sets for v in t], np.int32)

    def min_only(X, eps, mp):
        _, lab = dbscan_brute(X, eps, mp)
        return as_csr([[int(v)] if v >= 0 else [] for v in lab])

    def merged(X, eps, mp):
        off, ids = membership(X, eps, mp)
        sets = [ids[off[i]:off[i + 1]].tolist() for i in range(len(off) - 1)]
        return as_csr([[min(t)] * (len(t) > 0) if len(t) > 1 else t for t in sets])

    for bad in (min_only, merged):
        assert any(MEMBER_PINS[p](bad) for p in MEMBER_PINS), bad.__name__
