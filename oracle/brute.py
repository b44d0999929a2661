"""O0: brute-force exact DBSCAN from the definition (test infrastructure only).

Follows the DBSCAN definition in the paper's preliminaries section:

* core: p is core iff |{q : d(p, q) <= eps}| >= minPts (the set includes p);
* cluster: core points p, q share a cluster iff a chain of core points joins them
  with consecutive distances <= eps; every core point is in exactly one cluster;
* border: a non-core point within eps of a core point of a cluster belongs to it;
  noise: a non-core point within eps of no core point.

Every pairwise decision is the float64 test D <= E2 described in the package
docstring.  No shortcut of the grid method is used here.
"""

from __future__ import annotations

import numpy as np

# Rows per block when a block of distance rows is materialised (memory bound only).
_BLOCK_ELEMS = 1 << 22


def _within(D: np.ndarray, E2: float) -> np.ndarray:
    """The distance decision: inclusive, as "no more than eps" in the definition."""
    return D <= E2


def sqdist_rows(X: np.ndarray, rows: np.ndarray, cols: np.ndarray | None = None) -> np.ndarray:
    """D(i, j) for i in ``rows`` and j in ``cols`` (all points when None).

    Per dimension k in order: t = x_ik - x_jk (one rounding), acc = acc + t * t (two
    roundings).  numpy's elementwise float64 operations are single IEEE operations,
    so there is no contraction and no reordering across dimensions.
    """
    Xc = X if cols is None else X[cols]
    Xr = X[rows]
    acc = np.zeros((Xr.shape[0], Xc.shape[0]), dtype=np.float64)
    for k in range(X.shape[1]):
        t = Xr[:, k][:, None] - Xc[:, k][None, :]
        acc = acc + t * t
    return acc


def _row_blocks(n_rows: int, n_cols: int):
    step = max(1, _BLOCK_ELEMS // max(1, n_cols))
    for s in range(0, n_rows, step):
        yield s, min(n_rows, s + step)


def neighbour_counts(X: np.ndarray, E2: float) -> np.ndarray:
    """|N(i)| for every i, N(i) = {j : D(i, j) <= E2}, i itself included."""
    n = X.shape[0]
    cnt = np.zeros(n, dtype=np.int64)
    for s, e in _row_blocks(n, n):
        cnt[s:e] = _within(sqdist_rows(X, np.arange(s, e)), E2).sum(axis=1)
    return cnt


def core_flags(X: np.ndarray, eps: float, min_pts: int) -> np.ndarray:
    """Core test of the definition: at least minPts points within eps, self included."""
    E2 = float(np.float64(eps) * np.float64(eps))
    return neighbour_counts(X, E2) >= min_pts


def core_components(X: np.ndarray, core: np.ndarray, E2: float) -> np.ndarray:
    """Cluster id of every core point (-1 elsewhere) by breadth-first search.

    Clusters are the connected components of the graph on core points with an edge
    wherever D <= E2.  Searches start from core points in increasing index order, so
    the start of each search is the smallest index in its component and becomes the
    component's id.
    """
    n = X.shape[0]
    label = np.full(n, -1, dtype=np.int64)
    core_idx = np.flatnonzero(core)
    for s in core_idx:
        if label[s] >= 0:
            continue
        label[s] = s
        frontier = np.array([s])
        while frontier.size:
            unl = core_idx[label[core_idx] < 0]
            if unl.size == 0:
                break
            reached = np.zeros(unl.size, dtype=bool)
            for a, b in _row_blocks(frontier.size, unl.size):
                reached |= _within(sqdist_rows(X, frontier[a:b], unl), E2).any(axis=0)
            frontier = unl[reached]
            label[frontier] = s
    return label


def border_labels(X: np.ndarray, core: np.ndarray, label: np.ndarray, E2: float) -> np.ndarray:
    """Give each non-core point the smallest id among clusters with a core point within eps."""
    out = label.copy()
    non = np.flatnonzero(~core)
    core_idx = np.flatnonzero(core)
    if core_idx.size == 0:
        return out
    core_lab = label[core_idx]
    for s, e in _row_blocks(non.size, core_idx.size):
        w = _within(sqdist_rows(X, non[s:e], core_idx), E2)
        cand = np.where(w, core_lab[None, :], np.iinfo(np.int64).max)
        m = cand.min(axis=1)
        out[non[s:e]] = np.where(m == np.iinfo(np.int64).max, -1, m)
    return out


def membership(X, eps: float, min_pts: int):
    """Every cluster each point belongs to, from the definition (paper, section
    "Preliminaries"): a core point belongs to its own cluster only; a non-core point
    belongs to every cluster that has a core point within eps (it can be several:
    border points do not merge clusters); noise belongs to none.

    Returns CSR arrays in input order: offsets int64[n+1] and ids int32[offsets[n]],
    the ids of each point ascending.  Cluster ids are those of ``dbscan_brute``.
    """
    X = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
    if X.ndim == 1:
        X = X[:, None]
    n = X.shape[0]
    if n == 0:
        return np.zeros(1, np.int64), np.zeros(0, np.int32)
    E2 = float(np.float64(eps) * np.float64(eps))
    core = neighbour_counts(X, E2) >= min_pts
    label = core_components(X, core, E2)
    core_idx = np.flatnonzero(core)
    sets = [[] for _ in range(n)]
    for i in core_idx:
        sets[i] = [int(label[i])]
    non = np.flatnonzero(~core)
    if core_idx.size:
        for s, e in _row_blocks(non.size, core_idx.size):
            w = _within(sqdist_rows(X, non[s:e], core_idx), E2)
            for r in range(e - s):
                sets[non[s + r]] = sorted(set(label[core_idx[w[r]]].tolist()))
    offsets = np.zeros(n + 1, np.int64)
    offsets[1:] = np.cumsum([len(t) for t in sets])
    ids = np.array([v for t in sets for v in t], dtype=np.int32)
    return offsets, ids


def dbscan_brute(X, eps: float, min_pts: int):
    """Exact DBSCAN by definition.  Returns (core uint8[n], cluster id int32[n])."""
    X = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
    if X.ndim == 1:
        X = X[:, None]
    n = X.shape[0]
    if n == 0:
        return np.zeros(0, np.uint8), np.zeros(0, np.int32)
    E2 = float(np.float64(eps) * np.float64(eps))
    core = neighbour_counts(X, E2) >= min_pts
    label = core_components(X, core, E2)
    label = border_labels(X, core, label, E2)
    return core.astype(np.uint8), label.astype(np.int32)
