/*
 * O1: exact DBSCAN oracle in plain C with OpenMP — TEST INFRASTRUCTURE ONLY.
 *
 * Computes the DBSCAN definition of the paper's preliminaries section with the same
 * float64 decision as the numpy oracle O0:
 *
 *   D(p,q) = (((0 + t_0*t_0) + t_1*t_1) + ...),  t_k = p_k - q_k,
 *   "within eps"  <=>  D(p,q) <= E2,  E2 = eps*eps (one rounding),
 *
 * every operation rounded to nearest-even in dimension order.  This file must be
 * compiled with -ffp-contract=off and without -ffast-math so that no multiply-add
 * is fused and no sum is reordered.
 *
 * The only difference from O0 is where candidates come from: points are put in
 * buckets of side w = eps * (1 + 2^-20) and a range query around p scans the 3^d
 * buckets whose integer coordinates differ from p's by at most one.  Any q with
 * D(p,q) <= E2 has |q_k - p_k| <= eps * (1 + 2^-50) in every dimension, so with the
 * slack of w over eps it lies at most one bucket away as long as bucket indices stay
 * below 2^28 (checked; larger extents return O1_ERANGE).
 *
 *   core:    |{q : D(p,q) <= E2}| >= minPts, p itself counted;
 *   cluster: components of core points under D <= E2 (union-find, links only
 *            between pairs that pass the decision); id = smallest input index of a
 *            core point in the component;
 *   border:  a non-core point takes the smallest id among core points within eps;
 *            noise gets -1.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define O1_OK 0
#define O1_EINVAL (-1)
#define O1_ENOMEM (-2)
#define O1_ERANGE (-4)
#define O1_ENONFINITE (-5)

static double sqdist(const double *a, const double *b, int d) {
  double acc = 0.0;
  for (int k = 0; k < d; ++k) {
    double t = a[k] - b[k];
    acc = acc + t * t;
  }
  return acc;
}

/* ---- bucket table: integer coordinates -> contiguous run of sorted points ---- */

typedef struct {
  int d;
  int64_t nb;          /* number of non-empty buckets */
  int64_t *coord;      /* [nb*d] bucket coordinates */
  int64_t *start;      /* [nb+1] runs in the sorted point order */
  int64_t cap;         /* hash capacity (power of two) */
  int64_t *slot;       /* [cap] bucket id or -1 */
} buckets_t;

static uint64_t hash_coord(const int64_t *c, int d) {
  uint64_t h = 0x9E3779B97F4A7C15ull;
  for (int k = 0; k < d; ++k) {
    h ^= (uint64_t)c[k] + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
    h *= 0xBF58476D1CE4E5B9ull;
  }
  return h ^ (h >> 31);
}

static int64_t bucket_find(const buckets_t *B, const int64_t *c) {
  uint64_t m = (uint64_t)B->cap - 1;
  for (uint64_t h = hash_coord(c, B->d) & m;; h = (h + 1) & m) {
    int64_t b = B->slot[h];
    if (b < 0) return -1;
    if (memcmp(B->coord + b * B->d, c, sizeof(int64_t) * (size_t)B->d) == 0) return b;
  }
}

static const int64_t *g_sort_keys;
static int g_sort_d;

static int cmp_points(const void *pa, const void *pb) {
  int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
  const int64_t *ka = g_sort_keys + a * g_sort_d, *kb = g_sort_keys + b * g_sort_d;
  for (int k = 0; k < g_sort_d; ++k) {
    if (ka[k] != kb[k]) return ka[k] < kb[k] ? -1 : 1;
  }
  return a < b ? -1 : (a > b);
}

/* ---- union-find on sorted positions, parent[x] <= x always ---- */

static int64_t uf_find(int64_t *parent, int64_t x) {
  while (parent[x] != x) {
    parent[x] = parent[parent[x]];
    x = parent[x];
  }
  return x;
}

static void uf_union(int64_t *parent, int64_t a, int64_t b) {
  a = uf_find(parent, a);
  b = uf_find(parent, b);
  if (a == b) return;
  if (a < b) parent[b] = a;
  else parent[a] = b;
}

/* Enumerate the 3^d neighbour buckets of bucket coordinate c; returns the count of
 * non-empty ones written to out (at most 3^d). */
static int neighbour_buckets(const buckets_t *B, const int64_t *c, int64_t *out) {
  int d = B->d;
  int64_t t[8];
  int digit[8];
  int total = 1, cnt = 0;
  for (int k = 0; k < d; ++k) total *= 3;
  for (int k = 0; k < d; ++k) digit[k] = 0;
  for (int e = 0; e < total; ++e) {
    for (int k = 0; k < d; ++k) t[k] = c[k] + digit[k] - 1;
    int64_t b = bucket_find(B, t);
    if (b >= 0) out[cnt++] = b;
    for (int k = 0; k < d; ++k) {
      if (++digit[k] < 3) break;
      digit[k] = 0;
    }
  }
  return cnt;
}

int o1_dbscan(const double *X, int64_t n, int32_t d, double eps, int32_t min_pts,
              int32_t nthreads, uint8_t *core_out, int32_t *label_out) {
  if (n < 0 || d < 1 || d > 8 || !(eps > 0.0) || !isfinite(eps) || min_pts < 1)
    return O1_EINVAL;
  if (n == 0) return O1_OK;
  if (!X || !core_out || !label_out) return O1_EINVAL;
  if (nthreads > 0) omp_set_num_threads(nthreads);
  for (int64_t i = 0; i < n * d; ++i)
    if (!isfinite(X[i])) return O1_ENONFINITE;

  int rc = O1_OK;
  const double E2 = eps * eps;
  const double w = eps * (1.0 + 0x1p-20);
  double org[8];
  for (int k = 0; k < d; ++k) org[k] = X[k];
  for (int64_t i = 0; i < n; ++i)
    for (int k = 0; k < d; ++k)
      if (X[i * d + k] < org[k]) org[k] = X[i * d + k];

  int64_t *key = malloc(sizeof(int64_t) * (size_t)(n * d));
  int64_t *order = malloc(sizeof(int64_t) * (size_t)n);
  double *Xs = malloc(sizeof(double) * (size_t)(n * d));
  int64_t *pb = malloc(sizeof(int64_t) * (size_t)n);       /* bucket of sorted pos */
  uint8_t *cs = malloc((size_t)n);                         /* core flag, sorted pos */
  int64_t *ls = malloc(sizeof(int64_t) * (size_t)n);       /* label, sorted pos */
  buckets_t B = {d, 0, NULL, NULL, 0, NULL};
  if (!key || !order || !Xs || !pb || !cs || !ls) { rc = O1_ENOMEM; goto done; }

  for (int64_t i = 0; i < n; ++i) {
    order[i] = i;
    for (int k = 0; k < d; ++k) {
      double q = floor((X[i * d + k] - org[k]) / w);
      if (q > (double)(1 << 28)) { rc = O1_ERANGE; goto done; }
      key[i * d + k] = (int64_t)q;
    }
  }
  g_sort_keys = key;
  g_sort_d = d;
  qsort(order, (size_t)n, sizeof(int64_t), cmp_points);

  /* runs of equal bucket coordinates */
  B.coord = malloc(sizeof(int64_t) * (size_t)(n * d));
  B.start = malloc(sizeof(int64_t) * (size_t)(n + 1));
  if (!B.coord || !B.start) { rc = O1_ENOMEM; goto done; }
  for (int64_t s = 0; s < n; ++s) {
    int64_t i = order[s];
    for (int k = 0; k < d; ++k) Xs[s * d + k] = X[i * d + k];
    if (s == 0 || memcmp(key + order[s - 1] * d, key + i * d, sizeof(int64_t) * (size_t)d)) {
      memcpy(B.coord + B.nb * d, key + i * d, sizeof(int64_t) * (size_t)d);
      B.start[B.nb++] = s;
    }
    pb[s] = B.nb - 1;
  }
  B.start[B.nb] = n;
  B.cap = 1;
  while (B.cap < 2 * B.nb) B.cap <<= 1;
  B.slot = malloc(sizeof(int64_t) * (size_t)B.cap);
  if (!B.slot) { rc = O1_ENOMEM; goto done; }
  for (int64_t h = 0; h < B.cap; ++h) B.slot[h] = -1;
  for (int64_t b = 0; b < B.nb; ++b) {
    uint64_t m = (uint64_t)B.cap - 1;
    uint64_t h = hash_coord(B.coord + b * d, d) & m;
    while (B.slot[h] >= 0) h = (h + 1) & m;
    B.slot[h] = b;
  }

  int max_nb = 1;
  for (int k = 0; k < d; ++k) max_nb *= 3;

  /* core flags: count every point within eps, self included */
#pragma omp parallel
  {
    int64_t *nbr = malloc(sizeof(int64_t) * (size_t)max_nb);
#pragma omp for schedule(dynamic, 256)
    for (int64_t s = 0; s < n; ++s) {
      int m = neighbour_buckets(&B, B.coord + pb[s] * d, nbr);
      int64_t cnt = 0;
      for (int e = 0; e < m; ++e)
        for (int64_t q = B.start[nbr[e]]; q < B.start[nbr[e] + 1]; ++q)
          cnt += sqdist(Xs + s * d, Xs + q * d, d) <= E2;
      cs[s] = cnt >= min_pts;
    }
    free(nbr);
  }

  /* clusters: each thread unions the core pairs of its share of points in its own
   * union-find; the partitions are then joined into thread 0's structure. */
  {
    int T = omp_get_max_threads();
    int64_t *par = malloc(sizeof(int64_t) * (size_t)n * (size_t)T);
    if (!par) { rc = O1_ENOMEM; goto done; }
#pragma omp parallel num_threads(T)
    {
      int t = omp_get_thread_num();
      int64_t *P = par + (size_t)t * (size_t)n;
      for (int64_t x = 0; x < n; ++x) P[x] = x;
      int64_t *nbr = malloc(sizeof(int64_t) * (size_t)max_nb);
#pragma omp for schedule(dynamic, 256)
      for (int64_t s = 0; s < n; ++s) {
        if (!cs[s]) continue;
        int m = neighbour_buckets(&B, B.coord + pb[s] * d, nbr);
        for (int e = 0; e < m; ++e)
          for (int64_t q = B.start[nbr[e]]; q < B.start[nbr[e] + 1]; ++q) {
            if (q == s || !cs[q]) continue;
            if (uf_find(P, s) == uf_find(P, q)) continue;
            if (sqdist(Xs + s * d, Xs + q * d, d) <= E2) uf_union(P, s, q);
          }
      }
      free(nbr);
    }
    for (int t = 1; t < T; ++t) {
      int64_t *P = par + (size_t)t * (size_t)n;
      for (int64_t x = 0; x < n; ++x) uf_union(par, x, uf_find(P, x));
    }
    /* smallest input index per component */
    for (int64_t s = 0; s < n; ++s) ls[s] = INT64_MAX;
    for (int64_t s = 0; s < n; ++s) {
      if (!cs[s]) continue;
      int64_t r = uf_find(par, s);
      if (order[s] < ls[r]) ls[r] = order[s];
    }
    for (int64_t s = 0; s < n; ++s) {
      if (cs[s]) ls[s] = ls[uf_find(par, s)];
    }
    for (int64_t s = 0; s < n; ++s) if (!cs[s]) ls[s] = -1;
    free(par);
  }

  /* border points: smallest id among core points within eps */
#pragma omp parallel
  {
    int64_t *nbr = malloc(sizeof(int64_t) * (size_t)max_nb);
#pragma omp for schedule(dynamic, 256)
    for (int64_t s = 0; s < n; ++s) {
      if (cs[s]) continue;
      int m = neighbour_buckets(&B, B.coord + pb[s] * d, nbr);
      int64_t best = INT64_MAX;
      for (int e = 0; e < m; ++e)
        for (int64_t q = B.start[nbr[e]]; q < B.start[nbr[e] + 1]; ++q) {
          if (!cs[q] || ls[q] >= best) continue;
          if (sqdist(Xs + s * d, Xs + q * d, d) <= E2) best = ls[q];
        }
      ls[s] = best == INT64_MAX ? -1 : best;
    }
    free(nbr);
  }

  for (int64_t s = 0; s < n; ++s) {
    core_out[order[s]] = cs[s];
    label_out[order[s]] = (int32_t)ls[s];
  }

done:
  free(key); free(order); free(Xs); free(pb); free(cs); free(ls);
  free(B.coord); free(B.start); free(B.slot);
  return rc;
}

int o1_max_threads(void) { return omp_get_max_threads(); }
