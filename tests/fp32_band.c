/*
 * Host emulation of the float32 distance filter, to pin its error band on the CPU
 * (test infrastructure; compiled by tests/test_fp32_band.py with
 * -O2 -ffp-contract=off -fopenmp).
 *
 * The filter (added to the paper's method: its exact distance decision is the
 * float64 test of the definition in the preliminaries section) stores every point
 * as float32 coordinates relative to the float64 corner of its cell and decides a
 * pair (p in cell g, q in cell h) from
 *
 *   a = f32(f64(p - A_g)),  b = f32(f64(q - A_h)),  T = f32(f64(A_g - A_h)),
 *   D32 = float32 sum over k of (f32(f32(a_k - b_k) + T_k))^2, accumulated with
 *         fused multiply-adds (fmaf: one rounding per term),
 *
 * against thresholds T_in <= E2 <= T_out.  The proof bounds D32 in terms of the
 * defined float64 value D64 (sum of squared float64 differences in dimension order,
 * no fused operation):
 *
 *   lo(D64) = (1 - g_d) (sqrt(D64 / (1 + gb)) - sqrt(d) eta)^2 <= D32
 *   D32 <= hi(D64) = (1 + g_d) (sqrt(D64 / (1 - gb)) + sqrt(d) eta)^2
 *
 * with u = 2^-24, v = 2^-53, g_d = d u / (1 - d u), gb = (d + 2) v / (1 - (d + 2) v),
 * eta = (1 + 2^-20) u (6 M + 2 Tm), M bounding every |coordinate - anchor| and Tm
 * bounding |A_g - A_h| per dimension (eps (1 + 2^-20) + 2 M near the boundary).
 * T_in = lo(E2) and T_out = hi(E2), widened by 2^-40 and rounded outwards to
 * float32.
 *
 * band_check() draws pairs at distance eps (1 + delta) with small delta (most
 * within a few 1e-6 of the boundary) from a counter-based generator (splitmix64)
 * and reports the largest violations of both bounds and of the two decisions.
 * drop_eta = 1 plants a mistake for the tests: the coordinate error term is left
 * out of the bounds, as if the float32 coordinates were exact.
 */
#include <math.h>
#include <stdint.h>

static uint64_t splitmix64(uint64_t *s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static double unif(uint64_t *s) { return (double)(splitmix64(s) >> 11) * 0x1p-53; }

static double gauss(uint64_t *s) {
  double a = unif(s), b = unif(s);
  if (a < 1e-300) a = 1e-300;
  return sqrt(-2.0 * log(a)) * cos(6.283185307179586 * b);
}

static double d64(const double *p, const double *q, int d) {
  double acc = 0.0;
  for (int k = 0; k < d; ++k) {
    double t = p[k] - q[k];
    acc = acc + t * t;
  }
  return acc;
}

typedef struct {
  double gd, gb, r; /* gamma_d, gamma-bar, sqrt(d) * eta */
} band_t;

static band_t band_of(int d, double eps, double M, int drop_eta) {
  const double u = 0x1p-24, v = 0x1p-53;
  band_t b;
  b.gd = d * u / (1.0 - d * u);
  b.gb = (d + 2) * v / (1.0 - (d + 2) * v);
  double Tm = eps * (1.0 + 0x1p-20) + 2.0 * M;
  double eta = (1.0 + 0x1p-20) * u * (6.0 * M + 2.0 * Tm);
  b.r = drop_eta ? 0.0 : sqrt((double)d) * eta;
  return b;
}

static double lo_of(const band_t *b, double D) {
  double a = sqrt(D / (1.0 + b->gb)) * (1.0 - 0x1p-40) - b->r * (1.0 + 0x1p-40);
  return a > 0.0 ? (1.0 - b->gd) * a * a * (1.0 - 0x1p-40) : -1.0;
}

static double hi_of(const band_t *b, double D) {
  double a = sqrt(D / (1.0 - b->gb)) * (1.0 + 0x1p-40) + b->r * (1.0 + 0x1p-40);
  return (1.0 + b->gd) * a * a * (1.0 + 0x1p-40);
}

static float down32(double x) {
  float f = (float)x;
  return (double)f > x ? nextafterf(f, -INFINITY) : f;
}

static float up32(double x) {
  float f = (float)x;
  return (double)f < x ? nextafterf(f, INFINITY) : f;
}

/*
 * out[0] max (D32 - hi(D64)) / E2      (<= 0 when the upper bound holds)
 * out[1] max (lo(D64) - D32) / E2      (<= 0 when the lower bound holds)
 * out[2] pairs with D32 <= T_in but D64 > E2   (wrong IN: must be 0)
 * out[3] pairs with D32 > T_out but D64 <= E2  (wrong OUT: must be 0)
 * out[4] pairs inside the band (rechecked in float64)
 * out[5] max |D32 - D64| / E2
 * out[6] T_in / E2, out[7] T_out / E2
 * out[8] pairs with D64 <= E2
 */
void band_check(int d, double eps, double M, double domain, int64_t npairs, uint64_t seed,
                int drop_eta, double *out) {
  const double E2 = eps * eps;
  const band_t B = band_of(d, eps, M, drop_eta);
  const float tin = down32(lo_of(&B, E2));
  const float tout = up32(hi_of(&B, E2));
  double mx_hi = -INFINITY, mx_lo = -INFINITY, mx_abs = 0.0;
  int64_t wrong_in = 0, wrong_out = 0, band = 0, inside = 0;
#pragma omp parallel for schedule(static) reduction(max : mx_hi, mx_lo, mx_abs) \
    reduction(+ : wrong_in, wrong_out, band, inside)
  for (int64_t i = 0; i < npairs; ++i) {
    uint64_t s = seed * 0x2545F4914F6CDD1Dull + (uint64_t)i * 0x9E3779B97F4A7C15ull;
    double Ag[8], Ah[8], p[8], q[8], dir[8];
    double nrm = 0.0;
    /* a direction from the unit cube (uniformity on the sphere is not needed) */
    for (int k = 0; k < d; ++k) {
      dir[k] = 2.0 * unif(&s) - 1.0;
      nrm += dir[k] * dir[k];
    }
    if (nrm < 1e-6) {
      dir[0] = 1.0;
      nrm = 1.0;
    }
    nrm = sqrt(nrm);
    /* 9 in 10 pairs within a few 1e-6 of eps, the rest up to 20% either side */
    const double delta = (splitmix64(&s) % 10) ? 3e-6 * gauss(&s) : 0.4 * (unif(&s) - 0.5);
    const double len = eps * (1.0 + delta);
    for (int k = 0; k < d; ++k) {
      Ag[k] = domain * unif(&s);
      p[k] = Ag[k] + 0.999 * M * unif(&s);
      q[k] = p[k] + len * dir[k] / nrm;
      Ah[k] = q[k] - 0.999 * M * unif(&s);
    }
    float acc = 0.0f;
    for (int k = 0; k < d; ++k) {
      const float a = (float)(p[k] - Ag[k]);
      const float b = (float)(q[k] - Ah[k]);
      const float T = (float)(Ag[k] - Ah[k]);
      const float s1 = a - b;
      const float df = s1 + T;
      acc = fmaf(df, df, acc);
    }
    const double D = d64(p, q, d);
    const double D32 = (double)acc;
    const double h = (D32 - hi_of(&B, D)) / E2;
    const double l = (lo_of(&B, D) - D32) / E2;
    const double ab = fabs(D32 - D) / E2;
    if (h > mx_hi) mx_hi = h;
    if (l > mx_lo) mx_lo = l;
    if (ab > mx_abs) mx_abs = ab;
    if (acc <= tin && D > E2) ++wrong_in;
    if (acc > tout && D <= E2) ++wrong_out;
    if (acc > tin && acc <= tout) ++band;
    if (D <= E2) ++inside;
  }
  out[0] = mx_hi;
  out[1] = mx_lo;
  out[2] = (double)wrong_in;
  out[3] = (double)wrong_out;
  out[4] = (double)band;
  out[5] = mx_abs;
  out[6] = (double)tin / E2;
  out[7] = (double)tout / E2;
  out[8] = (double)inside;
}
