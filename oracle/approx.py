"""Checker for approximate DBSCAN (test infrastructure only).

The paper's preliminaries give Gan and Tao's approximate DBSCAN: the same as DBSCAN
except for the connectivity of core points.  Core points within eps of each other
must be in one cluster; core points farther apart than eps(1 + rho) must not be joined
by that pair; pairs in between may or may not be.  Several outputs are valid, so the
oracle for it is a checker of that definition rather than one expected output.

A clustering of the core points is valid exactly when it is the set of connected
components of some graph G with  E_eps <= G <= E_eps(1+rho)  (edges between core
points).  Equivalently:

  (i)  every pair of core points within eps has the same cluster id;
  (ii) the core points of each cluster are connected by pairs within eps(1 + rho)
       that stay inside the cluster.

(If (i) and (ii) hold, G = E_eps plus the within-cluster pairs of E_eps(1+rho) has
exactly the clusters as components; conversely components of such a G satisfy both.)

Readings, as for the exact oracle: "within eps" is the float64 test D <= fl(eps^2);
"within eps(1 + rho)" is D <= fl(R^2) with R = fl(eps * fl(1 + rho)).  The rest is as
in DBSCAN: core flags are exact, a cluster's id is its smallest core input index, a
non-core point takes the smallest id among clusters with a core point within eps, and
noise is -1.
"""

from __future__ import annotations

import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

from .brute import _row_blocks, core_flags, sqdist_rows


def relaxed_e2(eps: float, rho: float) -> float:
    """fl(R^2), R = fl(eps * fl(1 + rho)): the squared outer radius of the relaxation."""
    R = np.float64(eps) * (np.float64(1.0) + np.float64(rho))
    return float(R * R)


def check_approx(X, eps: float, min_pts: int, rho: float, core, label) -> list[str]:
    """Reasons why (core, label) is not a valid approximate DBSCAN output; [] if valid."""
    X = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
    if X.ndim == 1:
        X = X[:, None]
    n = X.shape[0]
    core = np.asarray(core).astype(bool)
    label = np.asarray(label).astype(np.int64)
    fails: list[str] = []
    if core.shape != (n,) or label.shape != (n,):
        return ["output shapes differ from the input"]
    if n == 0:
        return fails
    E2 = float(np.float64(eps) * np.float64(eps))
    E2r = relaxed_e2(eps, rho)

    want_core = core_flags(X, eps, min_pts)
    if not np.array_equal(core, want_core):
        bad = np.flatnonzero(core != want_core)
        fails.append(f"core flags differ at {bad.size} points, first {bad[:5].tolist()}")
        return fails

    ci = np.flatnonzero(core)
    cl = label[ci]
    if (cl < 0).any():
        fails.append("a core point has no cluster")
        return fails

    # (i) pairs within eps share a cluster; collect the pairs within eps(1 + rho)
    # inside a cluster for (ii)
    rows, cols = [], []
    for s, e in _row_blocks(ci.size, ci.size):
        D = sqdist_rows(X, ci[s:e], ci)
        near = D <= E2
        split = near & (cl[s:e, None] != cl[None, :])
        if split.any():
            a, b = np.argwhere(split)[0]
            fails.append(f"core points {ci[s + a]} and {ci[b]} are within eps but in "
                         f"clusters {cl[s + a]} and {cl[b]}")
            return fails
        r, c = np.nonzero((D <= E2r) & (cl[s:e, None] == cl[None, :]))
        rows.append(r + s)
        cols.append(c)
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    g = coo_matrix((np.ones(r.size, dtype=np.int8), (r, c)), shape=(ci.size, ci.size))
    _, comp = connected_components(g, directed=False)
    for lab in np.unique(cl):
        members = np.flatnonzero(cl == lab)
        if np.unique(comp[members]).size != 1:
            fails.append(f"cluster {lab} is not connected by pairs within eps(1 + rho)")
            return fails
        if lab != ci[members].min():
            fails.append(f"cluster {lab}: id is not its smallest core index {ci[members].min()}")
            return fails

    # non-core points: smallest id among clusters with a core point within eps
    non = np.flatnonzero(~core)
    big = np.iinfo(np.int64).max
    for s, e in _row_blocks(non.size, ci.size):
        w = sqdist_rows(X, non[s:e], ci) <= E2
        m = np.where(w, cl[None, :], big).min(axis=1)
        want = np.where(m == big, -1, m)
        got = label[non[s:e]]
        if not np.array_equal(got, want):
            k = int(np.flatnonzero(got != want)[0])
            fails.append(f"non-core point {non[s + k]} has id {got[k]}, expected {want[k]}")
            return fails
    return fails
