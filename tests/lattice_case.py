"""A lattice with a gap, in a seeded random order, whose DBSCAN output at eps = 1,
minPts = 5 has a closed form (DBSCAN definition, section "Preliminaries").

The points are the integer lattice [0, side)^2 without the column x = gap.  A point
has itself and its lattice neighbours at distance exactly 1 (float64 D = 1 <= fl(1^2))
in its eps-ball: interior points have 5, edge points 4, corners 3, so exactly the
interior points are core.  The two halves are 2 apart, so each half's core points form
one cluster, whose id is the smallest input index among them.  An edge point that is
not a corner has an interior neighbour at distance 1 and takes its half's id; a
corner's nearest core point is at sqrt(2) > eps, so corners are noise (-1).
"""

import numpy as np


def lattice(seed: int, side: int, gap: int):
    xs = np.concatenate([np.arange(gap), np.arange(gap + 1, side)]).astype(np.int32)
    ys = np.arange(side, dtype=np.int32)
    gx = np.repeat(xs, side)
    gy = np.tile(ys, xs.size)
    order = np.random.Generator(np.random.PCG64(seed)).permutation(gx.size)
    return gx[order], gy[order]


def points(gx, gy):
    X = np.empty((gx.size, 2), dtype=np.float64)
    X[:, 0] = gx
    X[:, 1] = gy
    return X


def expected(gx, gy, side: int, gap: int):
    left = gx < gap
    lo_x = np.where(left, 0, gap + 1)
    hi_x = np.where(left, gap - 1, side - 1)
    on_x_edge = (gx == lo_x) | (gx == hi_x)
    on_y_edge = (gy == 0) | (gy == side - 1)
    core = ~on_x_edge & ~on_y_edge
    corner = on_x_edge & on_y_edge
    idx = np.arange(gx.size)
    id_left = int(idx[core & left].min())
    id_right = int(idx[core & ~left].min())
    label = np.where(left, id_left, id_right).astype(np.int32)
    label[corner] = -1
    return core.astype(np.uint8), label
