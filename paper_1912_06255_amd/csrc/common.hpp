// Device-side building blocks shared by the DBSCAN kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define DB_DEV __device__ __forceinline__

namespace db {

constexpr int kWave = 64;
constexpr int kMaxD = 8;
constexpr int kTreeLevels = 5;  // node levels above the cells; 64^6 cells max

// ---------------------------------------------------------------------------
// Device-resident state of one call, written by the kernels themselves so that no
// host read is needed between phases.
// ---------------------------------------------------------------------------
struct GridDesc {
  double origin[kMaxD];   // per-dimension minimum of the points
  double side;            // cell side s = eps / sqrt(d), rounded
  int32_t bits[kMaxD];    // bits of each cell coordinate in the Morton key
  int32_t total_bits;     // sum of bits
  int32_t shift;          // key coordinate = floor(q / 2^shift), q = cell index
  int32_t fine_bits;      // sub-cell bits per dimension appended below the cell key
  int32_t cell_key_shift; // = fine_bits * d: key >> cell_key_shift is the cell key
  int32_t passes;         // 8-bit radix passes needed
  uint32_t epoch;         // bumped once per call; tags look-back words
  uint32_t status;        // DBSCAN_STATUS_* bits
  int32_t n_cells;        // C before/after splitting
  int32_t n_unsafe;       // cells whose float64 diameter test failed
  int32_t n_sub;          // cells queued for sub-cell order (k_cell_safe, k_subsort)
  unsigned long long max_extent_bits;  // largest cell extent (float64 bits, >= 0)
  float tin, tout;        // float32 filter thresholds (IN if <= tin, OUT if > tout)
  float tinb, toutb;      // the same for ClusterCore's radius (sqrt(E2b))
  // Counters, spread over kCtrSlots addresses (by workgroup) so that concurrent
  // updates do not serialise on one address; the host sums the slots.
  unsigned long long ctr[5][256];
};

constexpr int kCtrSlots = 256;
enum { kCtrBcp = 0, kCtrLinks = 1, kCtrRechecks = 2, kCtrPairs = 3, kCtrCore = 4 };

DB_DEV void stat_add_slot(GridDesc* g, int which, int slot, unsigned long long v) {
  if (v) atomicAdd(&g->ctr[which][slot & (kCtrSlots - 1)], v);
}

DB_DEV void stat_add(GridDesc* g, int which, unsigned long long v) {
  stat_add_slot(g, which, (int)blockIdx.x, v);
}

// ---------------------------------------------------------------------------
// Wave helpers
// ---------------------------------------------------------------------------
DB_DEV int lane_id() { return __lane_id(); }

DB_DEV uint64_t ballot(bool p) { return __ballot(p); }

DB_DEV uint64_t lanemask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

DB_DEV int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Orders LDS traffic between lanes of one wave.
DB_DEV void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Value of v in lane t (t wave-uniform), through scalar registers.
DB_DEV double bcast(double v, int t) {
  const int tt = __builtin_amdgcn_readfirstlane(t);
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), tt);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), tt);
  return __hiloint2double(hi, lo);
}

DB_DEV int bcast(int v, int t) {
  return __builtin_amdgcn_readlane(v, __builtin_amdgcn_readfirstlane(t));
}

DB_DEV float bcast(float v, int t) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), __builtin_amdgcn_readfirstlane(t)));
}

DB_DEV int wave_incl_scan(int v) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    int t = __shfl_up(v, o, kWave);
    if (l >= o) v += t;
  }
  return v;
}

DB_DEV int wave_sum(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

DB_DEV int wave_min(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, kWave));
  return v;
}

DB_DEV int wave_max(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, kWave));
  return v;
}

DB_DEV uint64_t wave_or(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, kWave);
  return v;
}

DB_DEV double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, kWave));
  return v;
}

DB_DEV double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}

// ---------------------------------------------------------------------------
// Coherent (L2, device scope) loads and stores for data other waves update.
// ---------------------------------------------------------------------------
template <class T>
DB_DEV T ld_acq(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
DB_DEV void st_rel(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

DB_DEV void atomic_min_double(double* addr, double v) {
  unsigned long long* a = reinterpret_cast<unsigned long long*>(addr);
  unsigned long long old = ld_acq(a);
  while (v < __longlong_as_double((long long)old)) {
    unsigned long long prev = atomicCAS(a, old, (unsigned long long)__double_as_longlong(v));
    if (prev == old) break;
    old = prev;
  }
}

DB_DEV void atomic_max_double(double* addr, double v) {
  unsigned long long* a = reinterpret_cast<unsigned long long*>(addr);
  unsigned long long old = ld_acq(a);
  while (v > __longlong_as_double((long long)old)) {
    unsigned long long prev = atomicCAS(a, old, (unsigned long long)__double_as_longlong(v));
    if (prev == old) break;
    old = prev;
  }
}

// ---------------------------------------------------------------------------
// The float64 distance decision: t_k = p_k - q_k, acc = acc + t_k*t_k in dimension
// order, each operation rounded once (the library is built with
// -ffp-contract=off; the pragma keeps it so if that flag is ever dropped).
// ---------------------------------------------------------------------------
template <int D>
DB_DEV double sqdist(const double (&p)[D], const double (&q)[D]) {
#pragma clang fp contract(off)
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double t = p[k] - q[k];
    acc = acc + t * t;
  }
  return acc;
}

// Float32 filter.  a and b are float32 coordinates of p and q relative to the
// float64 anchors A_g, A_h of their cells, T = fl32(fl64(A_g - A_h)); the value
// computed is fl32 of sum_k (fl32(fl32(a_k - b_k) + T_k))^2, in any order with
// fused multiply-adds allowed (its error bound covers that).  Returns 1 (within
// eps), 0 (not within) or 2 (inside the error band: decide again in float64).
template <int D>
DB_DEV int decide32(const float (&a)[D], const float (&b)[D], const float (&T)[D], float tin,
                    float tout) {
  float acc = 0.0f;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const float s1 = a[k] - b[k];
    const float df = s1 + T[k];
    acc = __builtin_fmaf(df, df, acc);
  }
  return acc <= tin ? 1 : (acc > tout ? 0 : 2);
}

// Lower bound of D(p, q) over p in box [alo, ahi] and q in box [blo, bhi], with
// the second box given as float32 bounds that contain the float64 box (rounded
// outwards): the gaps are computed in float64 from the widened bounds, so the
// result is at most the float64 one below and remains a lower bound.
template <int D>
DB_DEV double box_sqdist(const double (&alo)[D], const double (&ahi)[D], const float* blo,
                         const float* bhi, int stride, int j) {
#pragma clang fp contract(off)
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double l = (double)blo[(size_t)k * stride + j];
    const double h = (double)bhi[(size_t)k * stride + j];
    double t = 0.0;
    if (alo[k] > h) t = alo[k] - h;
    else if (l > ahi[k]) t = l - ahi[k];
    acc = acc + t * t;
  }
  return acc;
}

// Lower bound of D(p, q) over p in box [alo, ahi] and q in box [blo, bhi].
// Rounding is monotone, so the rounded per-dimension gap is at most |fl(p_k - q_k)|
// for every such pair, and squares and sums preserve the order: a box distance
// above E2 proves every pair between the boxes is farther than eps.
template <int D>
DB_DEV double box_sqdist(const double (&alo)[D], const double (&ahi)[D], const double* blo,
                         const double* bhi, int stride, int j) {
#pragma clang fp contract(off)
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double l = blo[(size_t)k * stride + j];
    const double h = bhi[(size_t)k * stride + j];
    double t = 0.0;
    if (alo[k] > h) t = alo[k] - h;
    else if (l > ahi[k]) t = l - ahi[k];
    acc = acc + t * t;
  }
  return acc;
}

// Upper bound of D(p, q) over q in the box [lo, hi].  Rounding is monotone, so
// fl(p_k - q_k) lies between fl(p_k - hi_k) and fl(p_k - lo_k) and its magnitude is
// at most the larger of theirs; squares and sums keep the order, so a bound of at
// most E2 proves every point of the box within eps of p (the float64 test, exactly).
template <int D>
DB_DEV double box_maxdist(const double (&p)[D], const double* lo, const double* hi, int stride,
                          int j) {
#pragma clang fp contract(off)
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double a = fabs(p[k] - lo[(size_t)k * stride + j]);
    const double b = fabs(p[k] - hi[(size_t)k * stride + j]);
    const double t = a > b ? a : b;
    acc = acc + t * t;
  }
  return acc;
}

// ---------------------------------------------------------------------------
// Decoupled look-back: each tile publishes a 64-bit word
//   [epoch:30 | flag:2 | value:32]
// flag 1 = tile aggregate only, flag 2 = inclusive prefix.  Words whose epoch is
// not the current call's count as "not yet published", so the state array never
// needs clearing.  The wait is bounded; on expiry the status bit is raised and the
// partial sum is used (the call then reports DBSCAN_EINTERNAL).
// ---------------------------------------------------------------------------
constexpr uint64_t kFlagAgg = 1, kFlagIncl = 2;
constexpr int kSpinLimit = 1 << 22;

DB_DEV uint64_t lb_word(uint32_t epoch, uint64_t flag, uint32_t value) {
  return ((uint64_t)(epoch & 0x3fffffffu) << 34) | (flag << 32) | value;
}

DB_DEV uint32_t lookback_exclusive(uint64_t* state, int stride, int tile, uint32_t epoch,
                                   uint32_t* status) {
  uint32_t excl = 0;
  int j = tile - 1;
  int spins = 0;
  const uint32_t ep = epoch & 0x3fffffffu;
  while (j >= 0) {
    uint64_t w = ld_acq(&state[(size_t)j * stride]);
    const uint32_t wep = (uint32_t)(w >> 34);
    const uint64_t flag = (w >> 32) & 3;
    if (wep != ep || flag == 0) {
      if (++spins > kSpinLimit) {
        atomicOr(status, 4u);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    excl += (uint32_t)w;
    if (flag == kFlagIncl) break;
    --j;
  }
  return excl;
}

}  // namespace db
