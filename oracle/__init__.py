"""CPU oracle for exact Euclidean DBSCAN — TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may import,
call, link or run anything in this package.  The GPU library never depends on it, and
this package shares no code with the GPU library.

What it computes is the DBSCAN definition of the paper's preliminaries section
(core points, clusters as components of core points chained at distance <= eps,
border and noise points), with these readings where the paper leaves room:

* a distance decision "d(p, q) <= eps" is the float64 test D(p, q) <= E2, where
  D = (((0 + t_0^2) + t_1^2) + ...) with t_k = p_k - q_k, every operation rounded to
  nearest-even, the sum taken in dimension order, no fused multiply-add, and
  E2 = eps * eps rounded once; no square root is ever taken;
* a point counts itself (D(p, p) = 0);
* the id of a cluster is the smallest input index of a core point in it;
* a border point, which the paper lets belong to several clusters, gets the smallest
  id among the clusters it belongs to; noise gets -1.  ``brute.membership`` gives the
  full set of clusters of every point as well.

Two implementations:

* ``brute`` (O0): numpy, every point against every point.  Plain and slow; use for
  n up to a few 10^4.
* ``o1`` (O1): plain C with OpenMP.  Same decisions, but candidates for each range
  query come from the 3^d buckets of side slightly above eps around the point, which
  provably contain every point within eps.  Pinned to O0 by the tests.

For approximate DBSCAN (Gan and Tao's relaxation, also in the preliminaries), whose
output is not unique, ``approx.check_approx`` checks an output against the relaxed
definition instead.
"""

from .approx import check_approx, relaxed_e2  # noqa: F401
from .brute import dbscan_brute, membership, sqdist_rows  # noqa: F401
from .o1 import dbscan_o1, o1_available, build_o1  # noqa: F401
