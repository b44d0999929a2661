"""Plant plausible mistakes in the CPU oracle and require the pins to catch each.

Each mutant replaces one piece of oracle.brute (on the CPU only) and must fail at
least one pin of tests/pins.py; a mutant that passes every pin would show a hole
in what pins the oracle.
"""

import numpy as np
import pytest

import oracle.brute as ob
from tests.pins import ALL_PINS


def _sq_reversed(X, rows, cols=None):
    Xc = X if cols is None else X[cols]
    Xr = X[rows]
    acc = np.zeros((Xr.shape[0], Xc.shape[0]))
    for k in reversed(range(X.shape[1])):
        t = Xr[:, k][:, None] - Xc[:, k][None, :]
        acc = acc + t * t
    return acc


def _sq_fused(X, rows, cols=None):
    # each square added to the running sum before rounding (extended precision)
    Xc = X if cols is None else X[cols]
    Xr = X[rows]
    acc = np.zeros((Xr.shape[0], Xc.shape[0]))
    for k in range(X.shape[1]):
        t = (Xr[:, k][:, None] - Xc[:, k][None, :]).astype(np.longdouble)
        acc = (acc.astype(np.longdouble) + t * t).astype(np.float64)
    return acc


def _sq_float32(X, rows, cols=None):
    Xc = (X if cols is None else X[cols]).astype(np.float32)
    Xr = X[rows].astype(np.float32)
    acc = np.zeros((Xr.shape[0], Xc.shape[0]), np.float32)
    for k in range(X.shape[1]):
        t = Xr[:, k][:, None] - Xc[:, k][None, :]
        acc = acc + t * t
    return acc.astype(np.float64)


def _sq_drop_last_dim(X, rows, cols=None):
    return _orig["sqdist_rows"](X[:, :-1] if X.shape[1] > 1 else X * 0, rows, cols)


def _counts_without_self(X, E2):
    return _orig["neighbour_counts"](X, E2) - 1


def _within_sqrt(D, E2):
    return np.sqrt(D) <= np.sqrt(E2)


def _border_max(X, core, label, E2):
    out = label.copy()
    non, cidx = np.flatnonzero(~core), np.flatnonzero(core)
    if cidx.size:
        w = ob._within(ob.sqdist_rows(X, non, cidx), E2)
        cand = np.where(w, label[cidx][None, :], -1)
        out[non] = cand.max(axis=1) if non.size else out[non]
    return out


def _border_none(X, core, label, E2):
    return label.copy()


def _components_max_id(X, core, E2):
    lab = _orig["core_components"](X, core, E2)
    out = lab.copy()
    for c in np.unique(lab[lab >= 0]):
        m = lab == c
        out[m] = np.flatnonzero(m).max()
    return out


def _components_through_all(X, core, E2):
    # treat every point as a chain member: border points then bridge clusters
    lab = _orig["core_components"](X, np.ones_like(core), E2)
    return np.where(core, lab, -1)


_orig = {
    "sqdist_rows": ob.sqdist_rows,
    "neighbour_counts": ob.neighbour_counts,
    "core_components": ob.core_components,
}

MUTANTS = {
    "strict_less": ("_within", lambda D, E2: D < E2),
    "sqrt_compare": ("_within", _within_sqrt),
    "reverse_dim_order": ("sqdist_rows", _sq_reversed),
    "fused_multiply_add": ("sqdist_rows", _sq_fused),
    "float32_distance": ("sqdist_rows", _sq_float32),
    "drop_last_dim": ("sqdist_rows", _sq_drop_last_dim),
    "self_not_counted": ("neighbour_counts", _counts_without_self),
    "border_max_id": ("border_labels", _border_max),
    "border_unassigned": ("border_labels", _border_none),
    "cluster_max_id": ("core_components", _components_max_id),
    "chain_through_border": ("core_components", _components_through_all),
}

@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, monkeypatch):
    attr, fn = MUTANTS[name]
    monkeypatch.setattr(ob, attr, fn)
    failed = []
    for pin_name, pin in ALL_PINS.items():
        if pin(ob.dbscan_brute):
            failed.append(pin_name)
            break
    assert failed, f"mutant {name} passed every pin"
