// Grid construction (paper: section "Grid Computation"; Algorithm 1, Cells):
// bounding box, Morton cell keys, LSD radix sort of (key, index), cell runs with a
// float64 diameter guard, and a 64-ary bounding-box tree over the sorted cells that
// plays the role of the paper's k-d tree over cells (section "Finding Neighboring
// Cells"): it returns exactly the non-empty cells that can hold a point within eps.
#pragma once

#include "common.hpp"

namespace db {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kXcds = 8;  // accelerator complex dies, each with its own L2

// Units [0, total) of a wave-per-unit kernel in an XCD-aware order.  Workgroup b
// runs on XCD b mod 8, so the units are cut into one contiguous range per XCD and
// that XCD's waves stride through it: units that are close in Morton order (and
// read each other's points) then share one L2 instead of being spread over all
// eight.  Every unit is visited by exactly one wave for any grid size.
struct UnitRange {
  long long first, end, step;
};

// (for G workgroups of which this is number bid: part of a launch shared by two jobs)
DB_DEV UnitRange xcd_units_of(long long total, int G, int bid) {
  const int X = G < kXcds ? G : kXcds;
  const int x = bid % X;
  const int r = bid / X;
  const int per = (G - x + X - 1) / X;  // workgroups b < G with b mod X == x
  const long long chunk = (total + X - 1) / X;
  const long long b = total < (long long)x * chunk ? total : (long long)x * chunk;
  const long long e = total < b + chunk ? total : b + chunk;
  return UnitRange{b + (long long)r * kWavesPerBlock + (long long)(threadIdx.x / kWave), e,
                   (long long)per * kWavesPerBlock};
}

DB_DEV UnitRange xcd_units(long long total) {
  return xcd_units_of(total, (int)gridDim.x, (int)blockIdx.x);
}
#ifndef DB_SORT_ITEMS
#define DB_SORT_ITEMS 16
#endif
constexpr int kSortItems = DB_SORT_ITEMS;
constexpr int kTile = kBlock * kSortItems;  // keys per radix / scan tile

constexpr int kIntMax = 0x7fffffff;

// Sub-cell order after the grid is built (k_subsort): default size threshold,
// workgroups of the launch, and the most Morton bits (summed over dimensions).
constexpr int kSubMinAuto = 2048;
constexpr int kSubBlocks = 256;
constexpr int kSubMaxBits = 12;
// Groups of sub-cell leaves: 64 chunks of 64 sorted positions (k_group_box).
constexpr int kGroupChunks = 64;
constexpr int kGroupPts = kGroupChunks * kWave;
static_assert(kGroupChunks == kWave, "a group's chunks are one per lane of a wave");

// Look-back epoch slots within one call: 0..7 radix passes, 8..9 cell scans.
constexpr uint32_t kEpochSlots = 16;

struct TreeView {
  const double* lo[kTreeLevels + 1];  // level 0 = cells, SoA [D][cap]
  const double* hi[kTreeLevels + 1];
  // float32 copies rounded outwards (lo down, hi up) for the walks: half the bytes,
  // and a box that contains the float64 one only weakens pruning
  const float* flo[kTreeLevels + 1];
  const float* fhi[kTreeLevels + 1];
  int cap[kTreeLevels + 1];
};

// All device pointers of one call.  Point and cell arrays use stride n (C <= n).
struct Work {
  int n;
  int minPts;
  int fine_max;       // at most this many sub-cell key bits per dimension
  int unit_max_level; // largest tree level acting as one ClusterCore unit
  int force_recheck;  // filter mode: decide every pair in float64
  int count_cap;      // MarkCore counts neighbours up to this value (largest minPts of the eps)
  int bcp_split;      // waves per ClusterCore unit
  int mark_split;     // MarkCore waves per cell (a power of two; grids of many points per cell)
  int dense_group;    // ClusterCore takes a group cell by cell from this many points per live cell
  int sub_min;        // cells of at least this many points get sub-cell order (k_subsort); kIntMax: none
  int warm;           // ClusterCore starts from the union-find the previous setting left (a larger
                      // minPts of the same eps: its core points, hence its links, are a subset)
  const int32_t* prev_core_count;  // warm: that setting's per-cell core counts (or null)
  int sparse_mode;    // 0: per-cell kernels, 1: batched sparse kernels
  int box_cells;      // 1: the cells are the box method's (d = 2; see box.hpp)
  uint32_t core_mask; // bit of this setting in coreS (settings of one eps share one byte per point)
  int32_t* sublist;   // [n / 2 + 1] first sorted positions of the cells queued for sub-cell order
  double eps;
  double E2;
  double E2b;         // ClusterCore's pair test: E2, or fl(R^2), R = fl(eps fl(1 + rho)), for approximate DBSCAN
  double E2leaf;      // approximate DBSCAN: leaves of squared diameter up to this are taken whole
                      // (about (eps rho / 2)^2; 0 when exact)
  double side;
  const double* pts;  // input, [n][D]
  uint8_t* core_out;
  int32_t* label_out;

  GridDesc* desc;
  double* bbox_part;  // [kBBoxBlocks][2*kMaxD]
  uint32_t* bbox_flag; // [kBBoxBlocks] a non-finite coordinate was seen by that workgroup
  uint32_t* ghist;    // [8][256]
  uint32_t* tilectr;  // [16]
  uint64_t* lbstate;  // [tiles * 256]
  uint64_t* keyA;
  uint64_t* keyB;
  uint32_t* idxA;
  uint32_t* idxB;
  double* X;          // [D][n] points in cell order
  float* X32;         // [D][n] float32 coordinates relative to the cell anchor (filter mode)
  double* chunkLo;    // [D][chunkCap] box of each aligned 64-point chunk of X
  double* chunkHi;
  double* runBox;     // [4][D][chunkCap] boxes of each chunk's first and last cell runs
                      // (first lo, first hi, last lo, last hi)
  int chunkCap;
  double* groupLo;    // [D][groupCap] boxes of the aligned groups of 64 chunks (k_group_box;
  double* groupHi;    // in the room of runBox, which is free by then)
  int groupCap;
  int32_t* perm;      // sorted position -> input index
  int32_t* inv;       // input index -> sorted position (kept only when several settings share a grid)
  uint64_t* pk;       // [n] with inv: cell << 8 | core bits of each sorted position (one word for
                      // the output pass to gather)
  uint64_t* skey;     // [n] sorted keys of the finest grid of a chain of eps values that differ by
                      // powers of two (coarser grids of the chain are cut from them), or null
  int32_t* cellOf;    // [n]
  int32_t* cellStart; // [n+1]
  int32_t* cellOf2;
  int32_t* cellStart2;
  uint8_t* unsafe;    // [n] per cell
  TreeView tree;      // tree.lo[0] / hi[0] = cell boxes
  uint8_t* coreS;     // [n] core flag, cell order
  int32_t* coreCount; // [n] per cell
  int32_t* parent;    // [n] union-find over cells
  int32_t* minIdx;    // [n] per root: smallest input index of a core point
  int32_t* cellLabel; // [n] per cell: cluster id of its core points or -1
  int32_t* cellMin;   // [n] per cell: smallest input index of its core points
  int32_t* nroot[kTreeLevels + 1];  // per tree node (levels 1..): common root or -1/-2
  int32_t* nlist;     // [cap1][64] level-1 nodes within reach of each level-1 node
  int32_t* nlen;      // [cap1] list length, -1 when longer than 64
  int32_t* blabel;    // [n] border label, cell order
  int32_t* cnt;       // [n] neighbours within eps, capped at count_cap, cell order
};

// What a kernel runs on: one grid (OneWork, the Work passed by value) or a group of
// grids (ManyWork: a table of Works in device memory).  A group shares each launch:
// every workgroup takes its share of each grid in turn, so small grids fill the
// chip together instead of one launch each.  Kernels size their launch for the
// largest grid of a group; the parts of a launch a smaller grid does not need find
// no work (or no tile) in it.
// each(): for kernels that share memory between the waves of a workgroup (a barrier
// separates the grids); each_wave(): for kernels whose waves work alone (shared
// memory per wave, no barrier), so that a wave goes on to the next grid as soon as
// its own share of this one is done.
struct OneWork {
  Work W;
  template <class F>
  DB_DEV void each(F&& f) const {
    f(W);
  }
  template <class F>
  DB_DEV void each_wave(F&& f) const {
    f(W);
  }
};

// The table is read through the constant address space: it is not written while a
// kernel runs, and the compiler then loads each grid's fields into scalar registers,
// as it does for a Work passed by value.
using ConstWork = const __attribute__((address_space(4))) Work;

struct ManyWork {
  ConstWork* Ws;
  int k;
  template <class F>
  DB_DEV void each(F&& f) const {
    for (int c = 0; c < k; ++c) {
      if (c) __syncthreads();  // the previous grid's use of shared memory is over
      f(*(const Work*)&Ws[c]);
    }
  }
  template <class F>
  DB_DEV void each_wave(F&& f) const {
    for (int c = 0; c < k; ++c) f(*(const Work*)&Ws[c]);
  }
};

constexpr int kBBoxBlocks = 512;

DB_DEV uint32_t epoch_of(const GridDesc* desc, uint32_t slot) {
  return (desc->epoch * kEpochSlots + slot) & 0x3fffffffu;
}

// ---------------------------------------------------------------------------
// Call initialisation: counters, histograms and the epoch.
// ---------------------------------------------------------------------------
// `first`: the first grid of a call (or of a batch) also clears the status and the
// cumulative counters.
DB_DEV void init_call(const Work& W, int first) {
  const int t = threadIdx.x;
  for (int i = t; i < 8 * 256; i += blockDim.x) W.ghist[i] = 0;
  if (t < 16) W.tilectr[t] = 0;
  GridDesc* g = W.desc;
  for (int i = t; i < 5 * kCtrSlots; i += blockDim.x) {
    const int which = i / kCtrSlots;
    if (first || which == kCtrCore) g->ctr[which][i % kCtrSlots] = 0;
  }
  if (t == 0) {
    g->epoch = g->epoch + 1;
    g->n_cells = 0;
    g->n_unsafe = 0;
    g->n_sub = 0;
    g->max_extent_bits = 0;
    if (first) g->status = 0;
  }
}

// ---------------------------------------------------------------------------
// Bounding box (partials per block, then one block finalises the grid).
// ---------------------------------------------------------------------------
template <int D, class WS>
__global__ __launch_bounds__(kBlock) void k_bbox_partial(WS ws, int first) {
  ws.each([&](const Work& W) {
    __shared__ double s_lo[kWavesPerBlock][D], s_hi[kWavesPerBlock][D];
    __shared__ int s_bad;
    if (blockIdx.x == 0) init_call(W, first);  // nothing below reads what it resets
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    double lo[D], hi[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
      lo[k] = __builtin_inf();
      hi[k] = -__builtin_inf();
    }
    bool bad = false;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < W.n; i += gridDim.x * kBlock) {
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const double v = W.pts[(size_t)i * D + k];
        bad |= !__builtin_isfinite(v);
        lo[k] = fmin(lo[k], v);
        hi[k] = fmax(hi[k], v);
      }
    }
    if (ballot(bad) && lane_id() == 0) s_bad = 1;
    const int w = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const double a = wave_min(lo[k]), b = wave_max(hi[k]);
      if (lane_id() == 0) {
        s_lo[w][k] = a;
        s_hi[w][k] = b;
      }
    }
    __syncthreads();
    if (threadIdx.x < D) {
      const int k = threadIdx.x;
      double a = s_lo[0][k], b = s_hi[0][k];
      for (int j = 1; j < kWavesPerBlock; ++j) {
        a = fmin(a, s_lo[j][k]);
        b = fmax(b, s_hi[j][k]);
      }
      W.bbox_part[blockIdx.x * 2 * kMaxD + k] = a;
      W.bbox_part[blockIdx.x * 2 * kMaxD + kMaxD + k] = b;
    }
    if (threadIdx.x == 0) W.bbox_flag[blockIdx.x] = (uint32_t)s_bad;
  });
}

// Grid: origin o = min corner, q_k = floor((x_k - o_k) / s).  The Morton key holds
// c_k = floor(q_k / 2^shift) with the smallest shift that fits all dimensions in
// 64 bits; shift = 0 (cells of side s) unless the extent is extreme.  A coarser
// key only makes cells larger: the diameter guard then splits them into single
// points, so the result is unchanged.
struct KeyGrid {
  double origin[kMaxD];
  double side;
  int bits[kMaxD];
  int total, shift, fine, passes, bad;
};

// Every workgroup of k_keys reduces the partials and derives the same grid
// (deterministically); workgroup 0 also publishes it in the descriptor.
template <int D>
DB_DEV void grid_from_partials(const Work& W, int nparts, KeyGrid& G) {
  __shared__ double s_lo[kWavesPerBlock][D], s_hi[kWavesPerBlock][D];
  __shared__ int s_bad;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  {
    double lo[D], hi[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
      lo[k] = __builtin_inf();
      hi[k] = -__builtin_inf();
    }
    bool bad = false;
    for (int j = threadIdx.x; j < nparts; j += kBlock) {
      bad |= W.bbox_flag[j] != 0;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        lo[k] = fmin(lo[k], W.bbox_part[j * 2 * kMaxD + k]);
        hi[k] = fmax(hi[k], W.bbox_part[j * 2 * kMaxD + kMaxD + k]);
      }
    }
    if (ballot(bad) && lane_id() == 0) s_bad = 1;
    const int w = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const double a = wave_min(lo[k]), b = wave_max(hi[k]);
      if (lane_id() == 0) {
        s_lo[w][k] = a;
        s_hi[w][k] = b;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const bool bad = s_bad != 0 || (W.desc->status & 1u) != 0;
    int len[D];
    for (int k = 0; k < D; ++k) {
      double a = s_lo[0][k], b = s_hi[0][k];
      for (int j = 1; j < kWavesPerBlock; ++j) {
        a = fmin(a, s_lo[j][k]);
        b = fmax(b, s_hi[j][k]);
      }
      G.origin[k] = bad ? 0.0 : a;
      len[k] = 0;
      if (!bad) {
        const double qmax = floor((b - a) / W.side);
        if (!(qmax < 1e308)) len[k] = 1100;          // infinite extent ratio
        else if (qmax >= 1.0) len[k] = ilogb(qmax) + 1;  // bit length of qmax
      }
    }
    int shift = 0, total = 0;
    for (;;) {
      int t = 0;
      for (int k = 0; k < D; ++k) t += max(0, len[k] - shift);
      if (t <= 64) {
        total = t;
        break;
      }
      ++shift;
    }
    for (int k = 0; k < kMaxD; ++k) G.bits[k] = k < D ? max(0, len[k] - shift) : 0;
    // Sub-cell bits order the points inside each cell along a finer Morton curve, so
    // that aligned 64-point chunks are spatially compact (tight chunk boxes).
    int fine = 0;
    if (shift == 0) fine = max(0, min(W.fine_max, (64 - total) / D));
    G.side = W.side;
    G.shift = shift;
    G.fine = fine;
    G.total = total + fine * D;
    G.passes = (total + fine * D + 7) / 8;
    G.bad = s_bad;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Morton key of every point and the 8-bit digit histograms of all radix passes.
// ---------------------------------------------------------------------------
template <int D>
DB_DEV uint64_t morton_key(const double* x, const KeyGrid& g, const int (&bits)[D], int maxb,
                           int fine) {
  unsigned long long c[D];
  unsigned f[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double u = (x[k] - g.origin[k]) / g.side;
    const double qc = floor(u);
    const double q = floor(ldexp(qc, -g.shift));
    const unsigned long long lim = bits[k] >= 64 ? ~0ull : ((1ull << bits[k]) - 1ull);
    unsigned long long v = q > 0.0 ? (unsigned long long)q : 0ull;
    if (!(q < 18446744073709551616.0)) v = lim;
    c[k] = v > lim ? lim : v;
    // position inside the cell, in 2^fine steps (u - floor(u) is exact)
    const double fr = ldexp(u - qc, fine);
    const unsigned flim = (1u << fine) - 1u;
    unsigned fv = fr > 0.0 ? (unsigned)fmin(fr, (double)flim) : 0u;
    f[k] = fv > flim ? flim : fv;
  }
  uint64_t key = 0;
  for (int b = maxb - 1; b >= 0; --b) {
#pragma unroll
    for (int k = 0; k < D; ++k) {
      if (b < bits[k]) key = (key << 1) | ((c[k] >> b) & 1ull);
    }
  }
  for (int b = fine - 1; b >= 0; --b) {
#pragma unroll
    for (int k = 0; k < D; ++k) key = (key << 1) | ((f[k] >> b) & 1u);
  }
  return key;
}

template <int D, class WS>
__global__ __launch_bounds__(kBlock) void k_keys(WS ws, int nparts) {
  ws.each([&](const Work& W) {
    __shared__ uint32_t s_hist[8][256];
    __shared__ KeyGrid g;
    for (int i = threadIdx.x; i < 8 * 256; i += kBlock) (&s_hist[0][0])[i] = 0;
    // The look-back words of this grid's scans start cleared.  The region can hold
    // anything an earlier call left there (another grid's keys, for instance), and
    // a stale word whose high bits happen to equal a tag of this call would be read
    // as a predecessor's prefix, leaving the permutation with holes.
    {
      const size_t nlb = (size_t)((W.n + kTile - 1) / kTile) * 256;
      for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < nlb;
           i += (size_t)gridDim.x * kBlock)
        W.lbstate[i] = 0;
    }
    grid_from_partials<D>(W, nparts, g);  // ends with a barrier
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      GridDesc* d = W.desc;
      for (int k = 0; k < kMaxD; ++k) {
        d->origin[k] = k < D ? g.origin[k] : 0.0;
        d->bits[k] = g.bits[k];
      }
      d->side = g.side;
      d->shift = g.shift;
      d->fine_bits = g.fine;
      d->cell_key_shift = g.fine * D;
      d->total_bits = g.total;
      d->passes = g.passes;
      if (g.bad) d->status |= 1u;
    }
    int bits[D];
    int maxb = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      bits[k] = g.bits[k];
      maxb = max(maxb, bits[k]);
    }
    const int passes = g.passes;
    const int fine = g.fine;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < W.n; i += gridDim.x * kBlock) {
      double x[D];
#pragma unroll
      for (int k = 0; k < D; ++k) x[k] = W.pts[(size_t)i * D + k];
      const uint64_t key = morton_key<D>(x, g, bits, maxb, fine);
      W.keyA[i] = key;
      W.idxA[i] = (uint32_t)i;
      W.cnt[i] = 0;  // MarkCore's waves add their shares to it
      for (int p = 0; p < passes; ++p) atomicAdd(&s_hist[p][(key >> (8 * p)) & 255], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < passes * 256; i += kBlock) {
      const uint32_t v = (&s_hist[0][0])[i];
      if (v) atomicAdd(&W.ghist[i], v);
    }
  });
}

// ---------------------------------------------------------------------------
// One 8-bit LSD radix pass (stable), single kernel per pass: tiles are taken in
// order from an atomic counter, ranked inside the tile with wave ballots, and
// offset across tiles with decoupled look-back per digit.
// ---------------------------------------------------------------------------
DB_DEV uint32_t block_excl_scan_256(uint32_t v, uint32_t* s_tmp /*[kWavesPerBlock]*/) {
  const int w = threadIdx.x / kWave;
  const int incl = wave_incl_scan((int)v);
  if (lane_id() == kWave - 1) s_tmp[w] = incl;
  __syncthreads();
  uint32_t off = 0;
  for (int j = 0; j < w; ++j) off += s_tmp[j];
  __syncthreads();
  return off + (uint32_t)incl - v;
}

template <class WS>
__global__ __launch_bounds__(kBlock) void k_sort_pass(WS ws, int pass) {
  ws.each([&](const Work& W) {
    __shared__ uint32_t s_wcnt[kWavesPerBlock][256];
    __shared__ uint32_t s_base[256];
    __shared__ uint32_t s_tmp[kWavesPerBlock];
    __shared__ int s_tile;
    const GridDesc* g = W.desc;
    if (pass >= g->passes) return;
    const uint64_t* kin = (pass & 1) ? W.keyB : W.keyA;
    const uint32_t* vin = (pass & 1) ? W.idxB : W.idxA;
    uint64_t* kout = (pass & 1) ? W.keyA : W.keyB;
    uint32_t* vout = (pass & 1) ? W.idxA : W.idxB;
    const uint32_t epoch = epoch_of(g, pass);
    const int tid = threadIdx.x, w = tid / kWave, lane = lane_id();
    if (tid == 0) s_tile = atomicAdd(&W.tilectr[pass], 1);
    for (int i = tid; i < kWavesPerBlock * 256; i += kBlock) (&s_wcnt[0][0])[i] = 0;
    __syncthreads();
    const int tile = s_tile;
    // (a launch shared by several grids has as many workgroups as the largest needs)
    if (tile >= (W.n + kTile - 1) / kTile) return;
    const int shift = 8 * pass;
    const int n = W.n;

    uint64_t key[kSortItems];
    uint32_t val[kSortItems];
    uint32_t rnk[kSortItems];
    const int base_idx = tile * kTile + w * (kWave * kSortItems);
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      const int idx = base_idx + j * kWave + lane;
      const bool valid = idx < n;
      key[j] = valid ? kin[idx] : 0ull;
      val[j] = valid ? vin[idx] : 0u;
    }
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      const int idx = base_idx + j * kWave + lane;
      const bool valid = idx < n;
      const uint32_t digit = (uint32_t)(key[j] >> shift) & 255u;
      uint64_t peers = ballot(valid);
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const bool bit = (digit >> b) & 1u;
        const uint64_t bb = ballot(bit);
        peers &= bit ? bb : ~bb;
      }
      const uint32_t before = (uint32_t)__popcll(peers & lanemask_lt());
      const uint32_t cnt = (uint32_t)__popcll(peers);
      const uint32_t old = valid ? s_wcnt[w][digit] : 0u;
      wave_sync();
      if (valid && before == 0) s_wcnt[w][digit] = old + cnt;
      wave_sync();
      rnk[j] = old + before;
    }
    __syncthreads();
    // per digit: offsets of each wave inside the tile, tile total, look-back.
    {
      const int dg = tid;
      uint32_t run = 0;
#pragma unroll
      for (int w2 = 0; w2 < kWavesPerBlock; ++w2) {
        const uint32_t t = s_wcnt[w2][dg];
        s_wcnt[w2][dg] = run;
        run += t;
      }
      uint64_t* st = W.lbstate + (size_t)tile * 256 + dg;
      uint32_t excl = 0;
      if (tile == 0) {
        st_rel(st, lb_word(epoch, kFlagIncl, run));
      } else {
        st_rel(st, lb_word(epoch, kFlagAgg, run));
        excl = lookback_exclusive(W.lbstate + dg, 256, tile, epoch, &W.desc->status);
        st_rel(st, lb_word(epoch, kFlagIncl, excl + run));
      }
      const uint32_t gstart = block_excl_scan_256(W.ghist[pass * 256 + dg], s_tmp);
      s_base[dg] = gstart + excl;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      const int idx = base_idx + j * kWave + lane;
      if (idx < n) {
        const uint32_t digit = (uint32_t)(key[j] >> shift) & 255u;
        const uint32_t dst = s_base[digit] + s_wcnt[w][digit] + rnk[j];
        if (dst < (uint32_t)n) {  // always true unless a look-back wait expired
          kout[dst] = key[j];
          vout[dst] = val[j];
        }
      }
    }
  });
}

// ---------------------------------------------------------------------------
// Cell runs.  mode 0: a new cell starts where the sorted key changes, and
// the points are gathered into cell order (SoA).  mode 1 (only when some cell
// failed the diameter guard): additionally every point of an unsafe cell becomes
// a cell of its own, written to the second set of cell arrays.  mode 2: a grid
// derived from a finer one (k_derive): the points keep their order and the cells
// are the runs of equal kept keys (skey >> cell_key_shift).
// ---------------------------------------------------------------------------
template <int D, class WS>
__global__ __launch_bounds__(kBlock) void k_cells(WS ws, int mode) {
  ws.each([&](const Work& W) {
    __shared__ uint32_t s_tmp[kWavesPerBlock];
    __shared__ uint32_t s_excl;
    __shared__ uint32_t s_tot;
    __shared__ int s_tile;
    const GridDesc* g = W.desc;
    if (mode == 1 && g->n_unsafe == 0) return;
    const int n = W.n;
    const bool odd = (g->passes & 1) != 0;
    const uint64_t* keys = odd ? W.keyB : W.keyA;
    const uint32_t* idx = odd ? W.idxB : W.idxA;
    // (mode 1 writes the second set of cell arrays; modes 0 and 2 the first)
    int32_t* cof = mode == 1 ? W.cellOf2 : W.cellOf;
    int32_t* cst = mode == 1 ? W.cellStart2 : W.cellStart;
    const int tid = threadIdx.x;
    if (tid == 0) s_tile = atomicAdd(&W.tilectr[8 + mode], 1);
    __syncthreads();
    const int tile = s_tile;
    if (tile >= (n + kTile - 1) / kTile) return;  // (see k_sort_pass)
    const uint32_t epoch = epoch_of(g, 8 + mode);
    const int cks = g->cell_key_shift;

    bool head[kSortItems];
    uint32_t pre[kSortItems];
    uint32_t run = 0;
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      const int i = tile * kTile + j * kBlock + tid;
      bool h = false;
      if (i < n) {
        if (i == 0) {
          h = true;
        } else if (mode == 0) {
          h = (keys[i] >> cks) != (keys[i - 1] >> cks);
        } else if (mode == 2) {
          h = (W.skey[i] >> cks) != (W.skey[i - 1] >> cks);
        } else {
          const int c = W.cellOf[i];
          h = c != W.cellOf[i - 1] || W.unsafe[c];
        }
      }
      head[j] = h;
      const uint32_t ex = block_excl_scan_256(h ? 1u : 0u, s_tmp);
      pre[j] = run + ex;
      // block total for this j: last thread's exclusive + its flag
      if (tid == kBlock - 1) s_tot = ex + (h ? 1u : 0u);
      __syncthreads();
      run += s_tot;
      __syncthreads();
    }
    if (tid == 0) {
      uint64_t* st = W.lbstate + (size_t)tile * 256;
      uint32_t excl = 0;
      if (tile == 0) {
        st_rel(st, lb_word(epoch, kFlagIncl, run));
      } else {
        st_rel(st, lb_word(epoch, kFlagAgg, run));
        excl = lookback_exclusive(W.lbstate, 256, tile, epoch, &W.desc->status);
        st_rel(st, lb_word(epoch, kFlagIncl, excl + run));
      }
      s_excl = excl;
    }
    __syncthreads();
    const uint32_t texcl = s_excl;
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      const int i = tile * kTile + j * kBlock + tid;
      if (i >= n) continue;
      int cid = (int)(texcl + pre[j] + (head[j] ? 1u : 0u)) - 1;
      cid = cid < 0 ? 0 : (cid >= n ? n - 1 : cid);  // clamps only after an expired wait
      cof[i] = cid;
      if (head[j]) cst[cid] = i;
      if (i == n - 1) {
        cst[cid + 1] = n;
        W.desc->n_cells = cid + 1;
      }
      if (mode == 2) W.cnt[i] = 0;  // MarkCore's waves add their shares to it (k_keys did not run)
      if (mode == 0) {
        uint32_t src = idx[i];
        if (src >= (uint32_t)n) src = 0;  // only after an expired wait
        W.perm[i] = (int32_t)src;
        if (W.inv) W.inv[src] = i;
        if (W.skey) W.skey[i] = keys[i];
#pragma unroll
        for (int k = 0; k < D; ++k) W.X[(size_t)k * n + i] = W.pts[(size_t)src * D + k];
      }
    }
  });
}

// A grid for eps' = 2^j eps from the grid of eps of the same cloud (call
// initialisation included, as k_bbox_partial does for a new grid).  With the same
// origin and side s' = 2^j s, each cell index of the coarser grid is the finer one
// divided by 2^j (scaling by a power of two is exact), so the coarser Morton key
// is the finer key without its lowest j levels: those levels hold min(bits_k, j)
// bits of each dimension k.  The points stay in the finer grid's order, which is
// sorted by the coarser key too; k_cells mode 2 cuts the runs.  (Any cut is exact:
// the diameter guard and the box tree decide every pair as for a fresh grid.)
template <int D>
__global__ __launch_bounds__(kBlock) void k_derive(Work W, int j) {
  init_call(W, 0);
  if (threadIdx.x == 0) {
    GridDesc* g = W.desc;
    int cut = 0;
    for (int k = 0; k < D; ++k) {
      const int b = g->bits[k];
      cut += min(b, j);
      g->bits[k] = max(0, b - j);
    }
    g->cell_key_shift += cut;
    g->total_bits -= cut;
    g->side = ldexp(g->side, j);
  }
}

// After a split: the second set of cell arrays becomes the first.

// ---------------------------------------------------------------------------
// Per-cell float64 point boxes (and the boxes of the aligned 64-point chunks).
// Every cell's box is written exactly once, without atomics.
// ---------------------------------------------------------------------------
template <int D, class WS>
__global__ __launch_bounds__(kBlock) void k_cell_box(WS ws, int only_if_split) {
  ws.each_wave([&](const Work& W) {
    const GridDesc* g = W.desc;
    if (only_if_split && g->n_unsafe == 0) return;
    const int n = W.n;
    const int C = g->n_cells;
    double* lo = const_cast<double*>(W.tree.lo[0]);
    double* hi = const_cast<double*>(W.tree.hi[0]);
    const int lane = lane_id();
    const int wid = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    // after a split the new cells are read from the second arrays, which are also
    // copied over the first ones here
    const int32_t* cellOf = only_if_split ? W.cellOf2 : W.cellOf;
    if (only_if_split) {
      for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += gridDim.x * blockDim.x) {
        if (i < n) W.cellOf[i] = W.cellOf2[i];
        if (i <= C) W.cellStart[i] = W.cellStart2[i];
      }
    }
    const int nw = gridDim.x * kWavesPerBlock;
    const int nchunks = (n + kWave - 1) / kWave;
    const size_t rc = (size_t)D * W.chunkCap;
    // Per aligned 64-point chunk: boxes of the cells lying wholly inside it
    // (segmented wave reduction), the box of the chunk itself, and the boxes of its
    // first and last cell runs, from which k_cell_span builds the boxes of the cells
    // that span several chunks.
    for (int ch = wid; ch < nchunks; ch += nw) {
      const int base = ch * kWave;
      const int i = base + lane;
      const bool valid = i < n;
      const int c = valid ? cellOf[i] : -1;
      const int cn = (i + 1 < n && lane < kWave - 1) ? cellOf[i + 1] : -2;
      // the cells just before and just after the chunk (one load each for the wave)
      const int before = base > 0 ? cellOf[base - 1] : -1;
      const int after = base + kWave < n ? cellOf[base + kWave] : -1;
      double xs[D];  // every load issued before the first store
#pragma unroll
      for (int k = 0; k < D; ++k) xs[k] = valid ? W.X[(size_t)k * n + i] : 0.0;
      const bool last = valid && (lane == kWave - 1 || i + 1 >= n || cn != c);
      // (the shuffle runs on every lane: a lane it reads from must be active)
      const int c_first = __shfl(c, 0, kWave);
      const bool first_run = last && c == c_first;
      // a run lies wholly inside the chunk unless it is the first run and its cell
      // began before the chunk, or it is the last run and its cell goes on after it
      const bool owned = last && (!first_run || c != before) &&
                         (lane < kWave - 1 || c != after);
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const double x = xs[k];
        double a = x, b = x;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
          const double ua = __shfl_up(a, o, kWave);
          const double ub = __shfl_up(b, o, kWave);
          const int uc = __shfl_up(c, o, kWave);
          if (lane >= o && uc == c) {
            a = fmin(a, ua);
            b = fmax(b, ub);
          }
        }
        if (owned) {
          lo[(size_t)k * n + c] = a;
          hi[(size_t)k * n + c] = b;
        }
        const size_t r = (size_t)k * W.chunkCap + ch;
        if (first_run) {
          W.runBox[r] = a;
          W.runBox[rc + r] = b;
        }
        if (lane == kWave - 1) {  // (the last run of a chunk ends at its last lane)
          W.runBox[2 * rc + r] = a;
          W.runBox[3 * rc + r] = b;
        }
        if (!only_if_split) {
          const double ca = wave_min(valid ? x : __builtin_inf());
          const double cb = wave_max(valid ? x : -__builtin_inf());
          if (lane == 0) {
            W.chunkLo[r] = ca;
            W.chunkHi[r] = cb;
          }
        }
      }
    }

  });
}

// Boxes of the cells that span more than one 64-point chunk (after k_cell_box, which
// wrote every chunk's box and the boxes of its first and last cell runs): the last
// run of the cell's first chunk, the whole chunks inside it and the first run of its
// last chunk.  One wave per cell, 64 chunk boxes per step, so a cell of 128k points
// costs 32 steps of loads instead of a pass over its points.
template <int D, class WS>
__global__ __launch_bounds__(kBlock) void k_cell_span(WS ws, int only_if_split) {
  ws.each_wave([&](const Work& W) {
    const GridDesc* g = W.desc;
    if (only_if_split && g->n_unsafe == 0) return;
    const int n = W.n;
    const int C = g->n_cells;
    double* lo = const_cast<double*>(W.tree.lo[0]);
    double* hi = const_cast<double*>(W.tree.hi[0]);
    const int lane = lane_id();
    const int wid = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    const int nw = gridDim.x * kWavesPerBlock;
    const size_t cap = W.chunkCap;
    const size_t rc = (size_t)D * cap;
    for (int c = wid; c < C; c += nw) {
      const int s = W.cellStart[c], e = W.cellStart[c + 1];
      const int c0 = s >> 6, c1 = (e - 1) >> 6;
      if (c0 == c1) continue;  // inside one chunk: done by k_cell_box
      double a[D], b[D];
#pragma unroll
      for (int k = 0; k < D; ++k) {
        a[k] = __builtin_inf();
        b[k] = -__builtin_inf();
      }
      if (lane == 0) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
          a[k] = fmin(W.runBox[2 * rc + k * cap + c0], W.runBox[k * cap + c1]);
          b[k] = fmax(W.runBox[3 * rc + k * cap + c0], W.runBox[rc + k * cap + c1]);
        }
      }
      for (int j = c0 + 1 + lane; j < c1; j += kWave) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
          a[k] = fmin(a[k], W.chunkLo[k * cap + j]);
          b[k] = fmax(b[k], W.chunkHi[k * cap + j]);
        }
      }
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const double ra = wave_min(a[k]), rb = wave_max(b[k]);
        if (lane == 0) {
          lo[(size_t)k * n + c] = ra;
          hi[(size_t)k * n + c] = rb;
        }
      }
    }
  });
}

// Sub-cell order for large cells: the leaves of the paper's per-cell quadtree
// (section "Range Counting"), built only where a cell holds at least sub_min
// points.  The points of the cell's whole aligned 64-point chunks are regrouped
// by a Morton code over the cell's box, about one code per chunk, so that each
// chunk covers a compact part of the cell; then those chunks' boxes are computed
// again.  The partial chunks at the cell's two ends keep their points, so no
// chunk shared with another cell changes and one workgroup owns each cell (the
// cells come from the queue k_cell_safe fills; the unsafe-cell split, which only
// turns unsafe cells into singletons, leaves their points in place).  The
// order inside one code is arbitrary: no result depends on the order of the
// points of a cell.  Buffers that are free at this point hold the moved points:
// the sort's keys and indices, and the float32 coordinates (computed later).  Up
// to 3 dimensions every coordinate moves at once (one temporary per dimension);
// above, one dimension at a time through one temporary, after each point's new
// place is stored.  With at most kSubMaxBits code bits, a cell in 7 or 8
// dimensions is split once per dimension: the first level of the paper's tree.
constexpr int kSubThreads = 1024;
constexpr int kSubUnroll = 8;

template <int D>
struct SubCode {
  double lo[D], sc[D];
  unsigned top;
  int f;
  DB_DEV unsigned operator()(const double (&x)[D]) const {
    unsigned q[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
      // (a NaN from a subnormal extent lands in code 0)
      const double t = (x[k] - lo[k]) * sc[k];
      q[k] = t >= (double)top ? top : (t > 0.0 ? (unsigned)t : 0u);
    }
    unsigned code = 0;
    for (int bit = f - 1; bit >= 0; --bit)
#pragma unroll
      for (int k = 0; k < D; ++k) code = (code << 1) | ((q[k] >> bit) & 1u);
    return code;
  }
};

template <int D, class WS>
__global__ __launch_bounds__(kSubThreads) void k_subsort(WS ws) {
  ws.each([&](const Work& W) {
    constexpr int NW = kSubThreads / kWave;
    constexpr int U = D <= 3 ? kSubUnroll : 2;
    __shared__ int s_off[1 << kSubMaxBits];
    __shared__ uint32_t s_wsum[NW];
    const GridDesc* g = W.desc;
    const int nq = g->n_sub, n = W.n;
    const int tid = threadIdx.x, w = tid / kWave, lane = lane_id();
    // one float64 array of n per dimension (the float32 coordinates hold
    // 4 n D >= 8 n bytes for d >= 2) and the moved input indices
    double* tmp[3] = {reinterpret_cast<double*>(W.keyA), reinterpret_cast<double*>(W.keyB),
                      reinterpret_cast<double*>(W.X32)};
    int32_t* tperm = reinterpret_cast<int32_t*>(W.idxA);
    int32_t* dst = reinterpret_cast<int32_t*>(W.X32);  // d > 3: each point's new place
    for (int t = blockIdx.x; t < nq; t += gridDim.x) {
      const int s = W.sublist[t];
      const int c = W.cellOf[s];
      const int e = W.cellStart[c + 1];
      const int a = (s + kWave - 1) / kWave * kWave, b = e / kWave * kWave;
      // f bits per dimension: about one Morton code per chunk
      const int nck = (b - a) / kWave;
      int lg = 0;
      while ((1 << lg) < nck) ++lg;
      SubCode<D> code;
      code.f = max(1, min((lg + D - 1) / D, kSubMaxBits / D));
      code.top = (1u << code.f) - 1u;
      const int B = 1 << (code.f * D);
#pragma unroll
      for (int k = 0; k < D; ++k) {
        code.lo[k] = W.tree.lo[0][(size_t)k * n + c];
        const double ext = W.tree.hi[0][(size_t)k * n + c] - code.lo[k];
        code.sc[k] = ext > 0.0 ? ldexp(1.0, code.f) / ext : 0.0;
      }
      for (int j = tid; j < B; j += kSubThreads) s_off[j] = 0;
      __syncthreads();
      // (1) points per code
      for (int i0 = a + tid; i0 < b; i0 += U * kSubThreads) {
        double x[U][D];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = i0 + u * kSubThreads;
#pragma unroll
          for (int k = 0; k < D; ++k) x[u][k] = i < b ? W.X[(size_t)k * n + i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (i0 + u * kSubThreads < b) atomicAdd(&s_off[code(x[u])], 1);
      }
      __syncthreads();
      // (2) first position of each code: exclusive prefix over the codes, each
      // thread owning a run of B / kSubThreads of them
      {
        const int per = (B + kSubThreads - 1) / kSubThreads;
        const int j0 = min(B, tid * per), j1 = min(B, j0 + per);
        int run = 0;
        for (int j = j0; j < j1; ++j) run += s_off[j];
        const int incl = wave_incl_scan(run);
        if (lane == kWave - 1) s_wsum[w] = (uint32_t)incl;
        __syncthreads();
        int pre = a + incl - run;
        for (int k = 0; k < w; ++k) pre += (int)s_wsum[k];
        for (int j = j0; j < j1; ++j) {
          const int v = s_off[j];
          s_off[j] = pre;
          pre += v;
        }
      }
      __syncthreads();
      if constexpr (D > 3) {
        // (3) each point's new place, and its input index moved there
        for (int i = a + tid; i < b; i += kSubThreads) {
          double x[D];
#pragma unroll
          for (int k = 0; k < D; ++k) x[k] = W.X[(size_t)k * n + i];
          const int t = atomicAdd(&s_off[code(x)], 1);
          dst[i] = t;
          tperm[t] = W.perm[i];
        }
        __syncthreads();
        // (4) the coordinates, one dimension at a time through tmp[0]
        for (int k = 0; k < D; ++k) {
          for (int i = a + tid; i < b; i += kSubThreads) tmp[0][dst[i]] = W.X[(size_t)k * n + i];
          __syncthreads();
          for (int i = a + tid; i < b; i += kSubThreads) W.X[(size_t)k * n + i] = tmp[0][i];
          __syncthreads();
        }
        // (5) the input indices and the chunks' new boxes, one wave per chunk (a and
        // b are multiples of the chunk size)
        for (int ch = a / kWave + w; ch < b / kWave; ch += NW) {
          const int i = ch * kWave + lane;
          const int pm = tperm[i];
          W.perm[i] = pm;
          if (W.inv) W.inv[pm] = i;
#pragma unroll
          for (int k = 0; k < D; ++k) {
            const double x = W.X[(size_t)k * n + i];
            const double mn = wave_min(x), mx = wave_max(x);
            if (lane == 0) {
              W.chunkLo[(size_t)k * W.chunkCap + ch] = mn;
              W.chunkHi[(size_t)k * W.chunkCap + ch] = mx;
            }
          }
        }
        __syncthreads();
      } else {
        // (3) every point and its input index to its place in the temporaries
        for (int i0 = a + tid; i0 < b; i0 += U * kSubThreads) {
          int pm[U];
          double x[U][D];
  #pragma unroll
          for (int u = 0; u < U; ++u) {
            const int i = i0 + u * kSubThreads;
            const bool ok = i < b;
            pm[u] = ok ? W.perm[i] : 0;
  #pragma unroll
            for (int k = 0; k < D; ++k) x[u][k] = ok ? W.X[(size_t)k * n + i] : 0.0;
          }
  #pragma unroll
          for (int u = 0; u < U; ++u) {
            if (i0 + u * kSubThreads >= b) continue;
            const int t = atomicAdd(&s_off[code(x[u])], 1);
            tperm[t] = pm[u];
  #pragma unroll
            for (int k = 0; k < D; ++k) tmp[k][t] = x[u][k];
          }
        }
        __syncthreads();
        // (4) back into place, one wave per chunk, with the chunk's new box
        constexpr int V = 4;
        for (int ch0 = a / kWave + w * V; ch0 < b / kWave; ch0 += NW * V) {
          int pm[V];
          double x[V][D];
  #pragma unroll
          for (int v = 0; v < V; ++v) {
            const int i = (ch0 + v) * kWave + lane;
            const bool ok = i < b;
            pm[v] = ok ? tperm[i] : 0;
  #pragma unroll
            for (int k = 0; k < D; ++k) x[v][k] = ok ? tmp[k][i] : 0.0;
          }
  #pragma unroll
          for (int v = 0; v < V; ++v) {
            const int ch = ch0 + v;
            if (ch * kWave >= b) continue;
            const int i = ch * kWave + lane;
            W.perm[i] = pm[v];
            if (W.inv) W.inv[pm[v]] = i;
  #pragma unroll
            for (int k = 0; k < D; ++k) {
              W.X[(size_t)k * n + i] = x[v][k];
              const double mn = wave_min(x[v][k]), mx = wave_max(x[v][k]);
              if (lane == 0) {
                W.chunkLo[(size_t)k * W.chunkCap + ch] = mn;
                W.chunkHi[(size_t)k * W.chunkCap + ch] = mx;
              }
            }
          }
        }
        __syncthreads();
      }
    }
  });
}

// The level above the sub-cell leaves: boxes of the aligned groups of 64 chunks
// (4,096 sorted positions).  A group that lies inside one cell is a node of that
// cell's tree holding 4,096 of its points: MarkCore counts or skips it whole, and
// ClusterCore skips its chunks when its box is farther than eps.  Groups that span
// cells are never used.  One wave per group; built after the last change to the
// chunk boxes (sub-cell order), only where the leaves are used.
template <int D, class WS>
__global__ __launch_bounds__(kBlock) void k_group_box(WS ws) {
  ws.each_wave([&](const Work& W) {
    const int nch = (W.n + kWave - 1) / kWave;
    const int ng = (nch + kGroupChunks - 1) / kGroupChunks;
    const int lane = lane_id();
    const int nw = gridDim.x * (blockDim.x / kWave);
    for (int g = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; g < ng; g += nw) {
      const int ch = g * kGroupChunks + lane;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const double lo = ch < nch ? W.chunkLo[(size_t)k * W.chunkCap + ch] : __builtin_inf();
        const double hi = ch < nch ? W.chunkHi[(size_t)k * W.chunkCap + ch] : -__builtin_inf();
        const double a = wave_min(lo), b = wave_max(hi);
        if (lane == 0) {
          W.groupLo[(size_t)k * W.groupCap + g] = a;
          W.groupHi[(size_t)k * W.groupCap + g] = b;
        }
      }
    }
  });
}

// Diameter guard: D(lo, hi) <= E2 proves every pair in the cell is within eps
// (monotone rounding; see box_sqdist).  The paper's claim that all points of a
// cell are within eps holds in exact arithmetic only.
template <int D, class WS>
__global__ void k_cell_safe(WS ws) {
  ws.each_wave([&](const Work& W) {
    GridDesc* g = W.desc;
    const int C = g->n_cells, n = W.n;
    int bad = 0;
    double ext = 0.0;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < C; c += gridDim.x * blockDim.x) {
      double a[D], b[D];
#pragma unroll
      for (int k = 0; k < D; ++k) {
        a[k] = W.tree.lo[0][(size_t)k * n + c];
        b[k] = W.tree.hi[0][(size_t)k * n + c];
      }
      const bool uns = !(sqdist<D>(a, b) <= W.E2);
      W.unsafe[c] = uns;
      bad += uns;
      // safe cells with at least sub_min points and two whole chunks inside them
      // are queued for sub-cell order by their first sorted position, which the
      // split of unsafe cells (into singletons, renumbering the cells) keeps
      if (!uns && W.sub_min != kIntMax && g->fine_bits == 0) {
        const int s = W.cellStart[c], e = W.cellStart[c + 1];
        if (e - s >= W.sub_min && e / kWave - (s + kWave - 1) / kWave >= 2)
          W.sublist[atomicAdd(&g->n_sub, 1)] = s;
      }
      // the extent bounds |coordinate - anchor| in the float32 filter; a cell that
      // fails the guard becomes singletons, whose anchors are the points themselves
      if (!uns) {
#pragma unroll
        for (int k = 0; k < D; ++k) ext = fmax(ext, b[k] - a[k]);
      }
    }
    bad = wave_sum(bad);
    ext = wave_max(ext);
    if (lane_id() == 0 && bad) atomicAdd(&g->n_unsafe, bad);
    // extents are >= 0, so their bit patterns order like the values
    if (lane_id() == 0 && ext > 0.0)
      atomicMax(&g->max_extent_bits, (unsigned long long)__double_as_longlong(ext));
  });
}

// Float32 filter thresholds (see decide32).  With u = 2^-24, v = 2^-53,
// M = largest cell extent (bounds |coordinate - anchor|) and
// Tm = eps (1 + 2^-20) + 2 M (bounds |T| for every pair near the eps boundary),
// each float32 coordinate difference is within
//   eta = (1 + 2^-20) u (6 M + 2 Tm)
// of the exact difference (five roundings: the two stored coordinates, T, the
// subtraction and the addition; the factor absorbs the u^2 and v terms).  The
// float32 sum of squares is within gamma_d = d u / (1 - d u) of its exact value,
// and the defined float64 D within gammabar = (d+2) v / (1 - (d+2) v) of the exact
// squared distance S.  Hence
//   D32 <= T_in  = (1 - gamma_d) (sqrt(E2 / (1 + gammabar)) - sqrt(d) eta)^2  =>  D <= E2
//   D32 >  T_out = (1 + gamma_d) (sqrt(E2 / (1 - gammabar)) + sqrt(d) eta)^2  =>  D >  E2.
// Both are widened by 2^-40 for the rounding of this computation and rounded
// outwards to float32.  Outside a safe exponent range every pair is rechecked.
template <int D>
DB_DEV void threshold_pair(const Work& W, double eps, double E2, float& tin_out, float& tout_out) {
  const GridDesc* g = W.desc;
  const double u = 0x1p-24, v = 0x1p-53;
  const double M = __longlong_as_double((long long)g->max_extent_bits) * (1.0 + 0x1p-40);
  const double gd = D * u / (1.0 - D * u);
  const double gb = (D + 2) * v / (1.0 - (D + 2) * v);
  const double Tm = eps * (1.0 + 0x1p-20) + 2.0 * M;
  const double eta = (1.0 + 0x1p-20) * u * (6.0 * M + 2.0 * Tm);
  const double r = sqrt((double)D) * eta * (1.0 + 0x1p-40);
  const double ain = sqrt(E2 / (1.0 + gb)) * (1.0 - 0x1p-40) - r;
  const double aout = sqrt(E2 / (1.0 - gb)) * (1.0 + 0x1p-40) + r;
  double tin = ain > 0.0 ? (1.0 - gd) * ain * ain * (1.0 - 0x1p-40) : -1.0;
  double tout = (1.0 + gd) * aout * aout * (1.0 + 0x1p-40);
  const bool ok = E2 >= 0x1p-100 && E2 <= 0x1p100 && (eps + 2.0 * M) <= 0x1p60 &&
                  __builtin_isfinite(tout) && (g->status & 1u) == 0;
  if (!ok || W.force_recheck) {
    tin = -__builtin_inf();
    tout = __builtin_inf();
  }
  tin_out = __double2float_rd(tin);
  tout_out = __double2float_ru(tout);
}

// The thresholds of eps (MarkCore, ClusterBorder) and of ClusterCore's radius,
// which differs only for approximate DBSCAN (sqrt(E2b), rounded up, then bounds it).
template <int D>
DB_DEV void thresholds(const Work& W, double eps) {
  GridDesc* g = W.desc;
  threshold_pair<D>(W, eps, W.E2, g->tin, g->tout);
  const double epsb = W.E2b == W.E2 ? eps : sqrt(W.E2b) * (1.0 + 0x1p-40);
  threshold_pair<D>(W, epsb, W.E2b, g->tinb, g->toutb);
}

// Float32 coordinates relative to the anchor of each point's cell (its box corner);
// the first thread also sets the thresholds.
// (workgroup bid of the nwg doing this job)
template <int D>
DB_DEV void local32_part(const Work& W, double eps, int nwg, int bid) {
  if (bid == 0 && threadIdx.x == 0) thresholds<D>(W, eps);
  const int n = W.n;
  for (int i = bid * blockDim.x + threadIdx.x; i < n; i += nwg * blockDim.x) {
    const int c = W.cellOf[i];
#pragma unroll
    for (int k = 0; k < D; ++k)
      W.X32[(size_t)k * n + i] = (float)(W.X[(size_t)k * n + i] - W.tree.lo[0][(size_t)k * n + c]);
  }
}

template <int D, class WS>
__global__ void k_local32(WS ws) {
  ws.each_wave([&](const Work& W) {
    local32_part<D>(W, W.eps, (int)gridDim.x, (int)blockIdx.x);
  });
}

// ---------------------------------------------------------------------------
// Tree level l: node j bounds children [64 j, 64 j + 64) of level l - 1.
// ---------------------------------------------------------------------------
DB_DEV int level_count(int C, int l) {
  long long c = C;
  for (int i = 0; i < l; ++i) c = (c + 63) >> 6;
  return (int)c;
}

template <int D, class WS>
__global__ __launch_bounds__(kBlock) void k_tree_level(WS ws, int l) {
  ws.each_wave([&](const Work& W) {
    const int C = W.desc->n_cells;
    const int nchild = level_count(C, l - 1);
    const int nnode = (nchild + 63) >> 6;
    const double* clo = W.tree.lo[l - 1];
    const double* chi = W.tree.hi[l - 1];
    const int cs = W.tree.cap[l - 1];
    double* plo = const_cast<double*>(W.tree.lo[l]);
    double* phi = const_cast<double*>(W.tree.hi[l]);
    float* cflo = const_cast<float*>(W.tree.flo[l - 1]);
    float* cfhi = const_cast<float*>(W.tree.fhi[l - 1]);
    float* pflo = const_cast<float*>(W.tree.flo[l]);
    float* pfhi = const_cast<float*>(W.tree.fhi[l]);
    const int ps = W.tree.cap[l];
    const int lane = lane_id();
    for (int j = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; j < nnode;
         j += gridDim.x * kWavesPerBlock) {
      const int ch = j * 64 + lane;
      const bool v = ch < nchild;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const double ca = v ? clo[(size_t)k * cs + ch] : __builtin_inf();
        const double cb = v ? chi[(size_t)k * cs + ch] : -__builtin_inf();
        if (l == 1 && v) {  // float copies of the cell boxes
          cflo[(size_t)k * cs + ch] = __double2float_rd(ca);
          cfhi[(size_t)k * cs + ch] = __double2float_ru(cb);
        }
        const double a = wave_min(ca);
        const double b = wave_max(cb);
        if (lane == 0) {
          plo[(size_t)k * ps + j] = a;
          phi[(size_t)k * ps + j] = b;
          pflo[(size_t)k * ps + j] = __double2float_rd(a);
          pfhi[(size_t)k * ps + j] = __double2float_ru(b);
        }
      }
    }
  });
}

// Levels l0 .. top in one workgroup (they hold few nodes: C / 64^l0 at most), level
// after level, instead of one launch each.
template <int D, class WS>
__global__ __launch_bounds__(kBlock) void k_tree_tail(WS ws, int l0) {
  ws.each([&](const Work& W) {
    const int C = W.desc->n_cells;
    const int lane = lane_id();
    for (int l = l0; l <= kTreeLevels; ++l) {
      const int nchild = level_count(C, l - 1);
      const int nnode = (nchild + 63) >> 6;
      const double* clo = W.tree.lo[l - 1];
      const double* chi = W.tree.hi[l - 1];
      const int cs = W.tree.cap[l - 1];
      double* plo = const_cast<double*>(W.tree.lo[l]);
      double* phi = const_cast<double*>(W.tree.hi[l]);
      float* pflo = const_cast<float*>(W.tree.flo[l]);
      float* pfhi = const_cast<float*>(W.tree.fhi[l]);
      const int ps = W.tree.cap[l];
      double top_lo[D], top_hi[D];  // the box of node 0 (wave 0, lane 0)
      for (int j = threadIdx.x / kWave; j < nnode; j += kWavesPerBlock) {
        const int ch = j * 64 + lane;
        const bool v = ch < nchild;
#pragma unroll
        for (int k = 0; k < D; ++k) {
          const double a = wave_min(v ? clo[(size_t)k * cs + ch] : __builtin_inf());
          const double b = wave_max(v ? chi[(size_t)k * cs + ch] : -__builtin_inf());
          top_lo[k] = a;
          top_hi[k] = b;
          if (lane == 0) {
            plo[(size_t)k * ps + j] = a;
            phi[(size_t)k * ps + j] = b;
            pflo[(size_t)k * ps + j] = __double2float_rd(a);
            pfhi[(size_t)k * ps + j] = __double2float_ru(b);
          }
        }
      }
      if (nnode == 1) {
        // every level above holds this one node with the same box: written directly,
        // without a round of loads and reductions per level
        if (threadIdx.x == 0) {
          for (int u = l + 1; u <= kTreeLevels; ++u) {
            const int us = W.tree.cap[u];
#pragma unroll
            for (int k = 0; k < D; ++k) {
              const_cast<double*>(W.tree.lo[u])[(size_t)k * us] = top_lo[k];
              const_cast<double*>(W.tree.hi[u])[(size_t)k * us] = top_hi[k];
              const_cast<float*>(W.tree.flo[u])[(size_t)k * us] = __double2float_rd(top_lo[k]);
              const_cast<float*>(W.tree.fhi[u])[(size_t)k * us] = __double2float_ru(top_hi[k]);
            }
          }
        }
        return;
      }
      __threadfence_block();
      __syncthreads();
    }
  });
}

}  // namespace db
