"""Write rounding_pairs.txt: point pairs whose eps decision depends on rounding order.

The decision is D(p,q) <= E2, where D sums the rounded squares of the rounded
coordinate differences in dimension order, with no fused multiply-add, and
E2 = fl(eps * eps).  Each pair kept here flips if the sum is taken in reverse
dimension order ("order" rows) or if each square is fused into the running sum
("fma" rows).  Expected decisions come from exact rational arithmetic with one
explicit round-to-nearest-even per operation (Python's Fraction -> float conversion
is correctly rounded), not from any implementation under test; the script then
asserts that the oracle agrees.

Run:  python tests/golden/make_rounding_pairs.py
"""

from __future__ import annotations

import os
import sys
from fractions import Fraction as F

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "rounding_pairs.txt")


def fl(x: F) -> float:
    return float(x)


def model_D(p, q, order, fused: bool) -> float:
    acc = 0.0
    for k in order:
        t = fl(F(p[k]) - F(q[k]))
        if fused:
            acc = fl(F(acc) + F(t) * F(t))
        else:
            acc = fl(F(acc) + F(fl(F(t) * F(t))))
    return acc


def search(rng, d, want, count):
    found = []
    tries = 0
    while len(found) < count and tries < 200_000:
        tries += 1
        eps = float(rng.uniform(0.5, 3.0))
        E2 = fl(F(eps) * F(eps))
        p = rng.uniform(0.0, 16.0, d)
        u = rng.standard_normal(d)
        u /= np.sqrt((u * u).sum())
        q = p + eps * u * (1.0 + rng.uniform(-4e-16, 4e-16))
        p = [float(v) for v in p]
        q = [float(v) for v in q]
        fwd = model_D(p, q, range(d), False)
        if want == "order":
            alt = model_D(p, q, range(d - 1, -1, -1), False)
        else:
            alt = model_D(p, q, range(d), True)
        if (fwd <= E2) != (alt <= E2):
            found.append((want, d, eps, p, q, int(fwd <= E2)))
    return found


def main() -> None:
    rng = np.random.Generator(np.random.PCG64(20200614))
    rows = []
    for d in (2, 3, 5, 7):
        rows += search(rng, d, "order", 4)
        rows += search(rng, d, "fma", 4)
    sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
    from oracle import dbscan_brute

    lines = [
        "# Point pairs whose float64 eps decision flips under reversed dimension order",
        "# ('order') or under fused multiply-add ('fma').  Expected 'within' comes from",
        "# exact rational arithmetic with one round-to-nearest-even per operation, sum",
        "# in dimension order, no fusion; written by make_rounding_pairs.py.",
        "# As a DBSCAN input [p, q] with minPts = 2, both points are core iff within.",
        "# kind d eps(hex) | p(hex)... | q(hex)... | within",
    ]
    for kind, d, eps, p, q, within in rows:
        core, _ = dbscan_brute(np.array([p, q]), eps, 2)
        assert int(core[0]) == within and int(core[1]) == within, (kind, d, eps, p, q)
        lines.append(
            f"{kind} {d} {eps.hex()} | {' '.join(v.hex() for v in p)} | "
            f"{' '.join(v.hex() for v in q)} | {within}"
        )
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {len(rows)} pairs to {OUT}")


if __name__ == "__main__":
    main()
