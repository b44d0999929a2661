"""Pins: checks of a DBSCAN implementation against facts fixed outside of it.

Every check takes ``impl(X, eps, min_pts) -> (core uint8[n], label int32[n])`` and
returns a list of failure messages (empty when the check passes).  The oracle must
pass all of them; ``test_oracle_mutations`` plants plausible mistakes in the oracle
and requires each mutant to fail at least one.

Sources of truth used here (none of them calls the implementation under test to
produce an expected value):

* hand-worked examples in ``golden/`` from the DBSCAN definition (paper,
  Preliminaries section);
* rounding-sensitive pairs in ``golden/rounding_pairs.txt`` whose decisions were
  derived in exact rational arithmetic;
* an exact integer-coordinate brute force using transitive closure (a different
  algorithm from the oracle's breadth-first search);
* library reductions: for minPts = 1 the clusters are the connected components of
  the eps-graph (scipy), and sklearn's DBSCAN agrees on core points and on the core
  partition when no pair lies near the eps boundary;
* closed forms and metamorphic invariants.
"""

from __future__ import annotations

import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
GOLDEN_CASES = [
    "ex1_1d_chain.txt",
    "ex2_2d_border_tie.txt",
    "ex3_fp64_rounding.txt",
    "ex4_exact_boundary.txt",
    "ex5_duplicates.txt",
    "ex6_border_bridge.txt",
]


def load_golden(name: str, with_members: bool = False):
    """Fixture rows "coords | core label [| clusters]"; the optional third field is
    the full membership (ascending ids, "-" for none)."""
    eps = mp = None
    X, core, label, members = [], [], [], []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line:
                continue
            if line.startswith("#"):
                body = line[1:].strip()
                if body.startswith("eps:"):
                    eps = float(body.split(":", 1)[1])
                elif body.startswith("minpts:"):
                    mp = int(body.split(":", 1)[1])
                continue
            fields = line.split("|")
            coords, out = fields[0], fields[1]
            X.append([float(v) for v in coords.split()])
            c, lab = out.split()
            core.append(int(c))
            label.append(int(lab))
            if len(fields) > 2:
                m = fields[2].split()
                members.append([] if m == ["-"] else [int(v) for v in m])
            else:
                members.append(None)
    res = (np.array(X, dtype=np.float64), eps, mp, np.array(core, np.uint8), np.array(label, np.int32))
    return res + (members,) if with_members else res


def load_rounding_pairs():
    rows = []
    with open(os.path.join(GOLDEN, "rounding_pairs.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            head, p, q, within = line.split("|")
            kind, d, eps = head.split()
            rows.append(
                (
                    kind,
                    int(d),
                    float.fromhex(eps),
                    [float.fromhex(v) for v in p.split()],
                    [float.fromhex(v) for v in q.split()],
                    int(within),
                )
            )
    return rows


def _as_np(res):
    core, label = res
    return np.asarray(core).astype(np.uint8), np.asarray(label).astype(np.int32)


def pin_golden(impl):
    fails = []
    for name in GOLDEN_CASES:
        X, eps, mp, core, label = load_golden(name)
        c, lab = _as_np(impl(X, eps, mp))
        if not (np.array_equal(c, core) and np.array_equal(lab, label)):
            fails.append(f"{name}: core {c.tolist()} label {lab.tolist()}")
    return fails


def pin_rounding(impl):
    fails = []
    for kind, d, eps, p, q, within in load_rounding_pairs():
        c, lab = _as_np(impl(np.array([p, q]), eps, 2))
        want_lab = [0, 0] if within else [-1, -1]
        if c.tolist() != [within, within] or lab.tolist() != want_lab:
            fails.append(f"{kind} d={d} eps={eps!r}: core {c.tolist()} want {within}")
    return fails


def integer_reference(P, eps_int: int, min_pts: int, with_members: bool = False):
    """DBSCAN on integer coordinates with exact integer arithmetic.

    Reachability between core points is the transitive closure (Warshall) of the
    core-core adjacency; a core point's id is the smallest core index it reaches.
    """
    n = len(P)
    E2 = eps_int * eps_int
    adj = [[sum((a - b) * (a - b) for a, b in zip(P[i], P[j])) <= E2 for j in range(n)] for i in range(n)]
    core = [sum(adj[i]) >= min_pts for i in range(n)]
    R = [[core[i] and core[j] and adj[i][j] for j in range(n)] for i in range(n)]
    for k in range(n):
        for i in range(n):
            if R[i][k]:
                for j in range(n):
                    if R[k][j]:
                        R[i][j] = True
    cid = [min(j for j in range(n) if R[i][j]) if core[i] else None for i in range(n)]
    label, members = [], []
    for i in range(n):
        if core[i]:
            label.append(cid[i])
            members.append([cid[i]])
        else:
            ids = sorted({cid[j] for j in range(n) if core[j] and adj[i][j]})
            label.append(ids[0] if ids else -1)
            members.append(ids)
    if with_members:
        return members
    return np.array(core, np.uint8), np.array(label, np.int32)


def pin_integer_bruteforce(impl, cases: int = 60, seed: int = 7):
    rng = np.random.Generator(np.random.PCG64(seed))
    fails = []
    for case in range(cases):
        d = int(rng.integers(1, 4))
        n = int(rng.integers(1, 14))
        P = rng.integers(-4, 5, size=(n, d)).tolist()
        eps = int(rng.integers(1, 4))
        mp = int(rng.integers(1, 5))
        want = integer_reference(P, eps, mp)
        got = _as_np(impl(np.array(P, dtype=np.float64), float(eps), mp))
        if not (np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])):
            fails.append(f"case {case}: P={P} eps={eps} minPts={mp}")
    return fails


def _members_of(offsets, ids):
    offsets = np.asarray(offsets, dtype=np.int64)
    ids = np.asarray(ids, dtype=np.int64)
    return [ids[offsets[i]:offsets[i + 1]].tolist() for i in range(len(offsets) - 1)]


def pin_members_golden(impl_members):
    """Hand-worked memberships in the fixtures that carry them."""
    fails = []
    for name in GOLDEN_CASES:
        X, eps, mp, _, _, members = load_golden(name, with_members=True)
        if any(m is None for m in members):
            continue
        got = _members_of(*impl_members(X, eps, mp))
        if got != members:
            fails.append(f"{name}: membership {got} want {members}")
    return fails


def pin_members_integer(impl_members, cases: int = 40, seed: int = 17):
    """Exact integer transitive closure: every point's full set of clusters.

    Random integer clouds almost never hold a point in two clusters, so each case
    starts from one of the two hand-worked geometries that do (ex2 in 2D, ex6 scaled
    by 10 onto an integer line), embedded in d = 1..3 dimensions, moved by a random
    integer translation, reflected and permuted per axis, with far integer noise and
    small clusters added and the point order shuffled."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ex2, _, _, _, _ = load_golden("ex2_2d_border_tie.txt")
    ex6, _, _, _, _ = load_golden("ex6_border_bridge.txt")
    bases = [(ex2.astype(np.int64), 1, 4), (np.rint(ex6 * 10).astype(np.int64), 10, 4)]
    fails = []
    multi = 0
    for case in range(cases):
        B, eps, mp = bases[case % 2]
        d = int(rng.integers(max(1, B.shape[1]), 4))
        P = np.zeros((B.shape[0], d), dtype=np.int64)
        P[:, :B.shape[1]] = B
        P = P[:, rng.permutation(d)] * rng.choice([-1, 1], size=d) + rng.integers(-50, 51, size=d)
        far = rng.integers(200, 260, size=(int(rng.integers(0, 8)), d)) * rng.choice([-1, 1], size=d)
        P = np.concatenate([P, far])[rng.permutation(len(P) + len(far))].tolist()
        want = integer_reference(P, eps, mp, with_members=True)
        multi += sum(len(m) > 1 for m in want)
        got = _members_of(*impl_members(np.array(P, dtype=np.float64), float(eps), mp))
        if got != want:
            fails.append(f"case {case}: P={P} eps={eps} minPts={mp}: {got} want {want}")
    if multi == 0:
        fails.append("no point in two clusters: the cases do not exercise full membership")
    return fails


MEMBER_PINS = {"members_golden": pin_members_golden, "members_integer": pin_members_integer}


def _canonical_components(n, edges):
    """Component id = smallest member index, from an explicit edge list."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components

    if len(edges):
        e = np.asarray(edges)
        A = coo_matrix((np.ones(len(e)), (e[:, 0], e[:, 1])), shape=(n, n))
    else:
        A = coo_matrix((n, n))
    _, comp = connected_components(A, directed=False)
    first = np.full(comp.max() + 1, n, dtype=np.int64)
    np.minimum.at(first, comp, np.arange(n))
    return first[comp].astype(np.int32)


def pin_scipy_minpts1(impl, seed: int = 11):
    """minPts = 1: every point is core and clusters are eps-graph components."""
    rng = np.random.Generator(np.random.PCG64(seed))
    fails = []
    for d in (1, 2, 3, 5):
        P = rng.integers(0, 40, size=(300, d))
        eps = 3
        diff = P[:, None, :] - P[None, :, :]
        adj = (diff * diff).sum(axis=2) <= eps * eps
        want = _canonical_components(len(P), np.argwhere(adj))
        c, lab = _as_np(impl(P.astype(np.float64), float(eps), 1))
        if not c.all() or not np.array_equal(lab, want):
            fails.append(f"d={d}: minPts=1 components differ")
    return fails


def _margin_safe(X, eps, rel=1e-9):
    from scipy.spatial.distance import pdist

    dist = pdist(X)
    return np.min(np.abs(dist - eps)) > rel * eps


def pin_sklearn(impl, seed: int = 13):
    """sklearn DBSCAN (kd-tree) agrees on core points and on how they are grouped."""
    from sklearn.cluster import DBSCAN

    rng = np.random.Generator(np.random.PCG64(seed))
    fails = []
    for d, eps, mp in ((2, 0.6, 5), (3, 0.9, 8), (5, 1.6, 6)):
        k = 6
        centres = rng.uniform(0, 10, size=(k, d))
        X = centres[rng.integers(0, k, 900)] + rng.standard_normal((900, d)) * 0.5
        X = np.concatenate([X, rng.uniform(0, 10, size=(100, d))])
        if not _margin_safe(X, eps):
            fails.append(f"d={d}: data not margin safe, pick another seed")
            continue
        sk = DBSCAN(eps=eps, min_samples=mp, algorithm="kd_tree").fit(X)
        sk_core = np.zeros(len(X), bool)
        sk_core[sk.core_sample_indices_] = True
        c, lab = _as_np(impl(X, eps, mp))
        if not np.array_equal(c.astype(bool), sk_core):
            fails.append(f"d={d}: core flags differ from sklearn")
            continue
        a, b = lab[sk_core], sk.labels_[sk_core]
        pairs = set(zip(a.tolist(), b.tolist()))
        if len(pairs) != len(set(a.tolist())) or len(pairs) != len(set(b.tolist())):
            fails.append(f"d={d}: core partition differs from sklearn")
    return fails


def pin_closed_forms(impl, seed: int = 17):
    rng = np.random.Generator(np.random.PCG64(seed))
    fails = []
    X = rng.uniform(0, 1, size=(50, 3))
    c, lab = _as_np(impl(X, 0.2, 51))
    if c.any() or (lab != -1).any():
        fails.append("minPts > n must give all noise")
    c, lab = _as_np(impl(X, 0.05, 1))
    if not c.all():
        fails.append("minPts = 1 must make every point core")
    c, lab = _as_np(impl(X, 2.0, 50))
    if not c.all() or (lab != 0).any():
        fails.append("eps above the diameter must give one cluster with id 0")
    c, lab = _as_np(impl(np.array([[3.0, -1.0]]), 1.0, 1))
    if c.tolist() != [1] or lab.tolist() != [0]:
        fails.append("a single point with minPts = 1 is its own cluster 0")
    # well separated singletons: each its own cluster, id = own index
    Y = np.arange(20, dtype=np.float64)[:, None] * 10.0
    c, lab = _as_np(impl(Y, 1.0, 1))
    if not np.array_equal(lab, np.arange(20, dtype=np.int32)):
        fails.append("isolated points with minPts = 1 must carry their own index")
    return fails


def _core_partition(core, lab):
    idx = np.flatnonzero(core)
    groups = {}
    for i in idx.tolist():
        groups.setdefault(int(lab[i]), []).append(i)
    return sorted(tuple(sorted(g)) for g in groups.values())


def pin_metamorphic(impl, seed: int = 19):
    rng = np.random.Generator(np.random.PCG64(seed))
    fails = []
    k = 5
    centres = rng.uniform(0, 20, size=(k, 3))
    X = centres[rng.integers(0, k, 600)] + rng.standard_normal((600, 3))
    eps, mp = 0.8, 6
    base = _as_np(impl(X, eps, mp))
    for p2 in (-3, 7):
        s = 2.0 ** p2
        got = _as_np(impl(X * s, eps * s, mp))
        if not (np.array_equal(got[0], base[0]) and np.array_equal(got[1], base[1])):
            fails.append(f"scaling by 2^{p2} changed the result")
    perm = rng.permutation(len(X))
    got = _as_np(impl(X[perm], eps, mp))
    if not np.array_equal(got[0], base[0][perm]):
        fails.append("permuting points must permute core flags")
    else:
        inv = np.empty_like(perm)
        inv[perm] = np.arange(len(perm))
        p_old = _core_partition(base[0], base[1])
        p_new = [tuple(sorted(perm[list(g)].tolist())) for g in _core_partition(got[0], got[1])]
        if sorted(p_new) != p_old:
            fails.append("permuting points changed the core partition")
        # ids are the smallest new index of a core point of the cluster
        for g in _core_partition(got[0], got[1]):
            if got[1][g[0]] != g[0]:
                fails.append("cluster id is not its smallest core index after permuting")
                break
        noise_old = set(np.flatnonzero(base[1] < 0).tolist())
        noise_new = set(perm[np.flatnonzero(got[1] < 0)].tolist())
        if noise_old != noise_new:
            fails.append("permuting points changed the noise set")
    # integer data: translation, axis permutation and reflection are exact
    P = rng.integers(0, 30, size=(400, 3)).astype(np.float64)
    b2 = _as_np(impl(P, 2.0, 4))
    for name, Q in (
        ("translate", P + np.array([1024.0, -77.0, 5.0])),
        ("axes", P[:, [2, 0, 1]]),
        ("reflect", -P),
    ):
        got = _as_np(impl(Q, 2.0, 4))
        if not (np.array_equal(got[0], b2[0]) and np.array_equal(got[1], b2[1])):
            fails.append(f"integer data: {name} changed the result")
    return fails


ALL_PINS = {
    "golden": pin_golden,
    "rounding": pin_rounding,
    "integer_bruteforce": pin_integer_bruteforce,
    "scipy_minpts1": pin_scipy_minpts1,
    "sklearn": pin_sklearn,
    "closed_forms": pin_closed_forms,
    "metamorphic": pin_metamorphic,
}
