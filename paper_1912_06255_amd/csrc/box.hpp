// The box method for the cells in two dimensions (section "Box Computation"):
// instead of grid cells, disjoint boxes of side at most eps / sqrt(2).  The points
// are sorted by x and cut into strips: a strip starts with the first point farther
// than eps / sqrt(2) in x from the start of the one before.  Each strip, sorted by
// y, is cut into boxes the same way.  Both cuts run as the paper parallelises them:
// every point finds, by binary search, the first point beyond its own coordinate
// plus eps / sqrt(2) (its parent), and pointer jumping from the first point marks
// the chain of parents, which are exactly the starts the sequential scan would take.
//
// The boxes then stand where the grid cells stood: the box ids are the sorted keys
// that k_cells cuts into cells, and the rest of the pipeline (cell boxes, the
// float64 diameter guard, the box tree, MarkCore, ClusterCore, ClusterBorder) runs
// unchanged.  The result is the same DBSCAN result as with grid cells; only the
// cells differ.  Neighbouring boxes are found by the box tree's walks, not by the
// paper's merging of strips s - 2 .. s + 2.
//
// Temporaries (all free while the grid is built; the clustering stages set them
// again): the union-find parents and minIdx as the two pointer arrays, coreCount
// as the marks, cellMin as the scan's output, cellLabel as the strip of each input
// point, sublist for the scan's block sums, and keyB for the y values of a strip.
#pragma once

#include "grid.hpp"

namespace db {

constexpr int kBoxScanItems = kBlock * 16;

// Order-preserving map of a finite double to an unsigned key (a < b gives
// key(a) < key(b); -0.0 sorts just before +0.0), and its inverse.
DB_DEV uint64_t box_key(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | (1ull << 63));
}
DB_DEV double box_val(uint64_t k) {
  const uint64_t b = (k >> 63) ? (k & ~(1ull << 63)) : ~k;
  return __longlong_as_double((long long)b);
}

// Histograms of the first `passes` 8-bit digits of key, added to the global ones.
DB_DEV void box_hist_add(uint32_t (*s_hist)[256], uint64_t key, int passes) {
  for (int p = 0; p < passes; ++p) atomicAdd(&s_hist[p][(key >> (8 * p)) & 255], 1u);
}
DB_DEV void box_hist_flush(const Work& W, uint32_t (*s_hist)[256], int passes) {
  __syncthreads();
  for (int i = threadIdx.x; i < passes * 256; i += kBlock) {
    const uint32_t v = (&s_hist[0][0])[i];
    if (v) atomicAdd(&W.ghist[i], v);
  }
}
DB_DEV void box_clear_lookback(const Work& W) {
  const size_t nlb = (size_t)((W.n + kTile - 1) / kTile) * 256;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < nlb; i += (size_t)gridDim.x * kBlock)
    W.lbstate[i] = 0;
}

// Sort keys of the x coordinates (what k_keys does for grid cells: the look-back
// words cleared, the bounding box checked for non-finite coordinates, MarkCore's
// counts zeroed, the histograms of all 8 passes).
__global__ __launch_bounds__(kBlock) void k_box_xkeys(Work W, int nparts) {
  __shared__ uint32_t s_hist[8][256];
  __shared__ KeyGrid g;
  for (int i = threadIdx.x; i < 8 * 256; i += kBlock) (&s_hist[0][0])[i] = 0;
  box_clear_lookback(W);
  grid_from_partials<2>(W, nparts, g);  // ends with a barrier
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    GridDesc* d = W.desc;
    for (int k = 0; k < kMaxD; ++k) {
      d->origin[k] = k < 2 ? g.origin[k] : 0.0;
      d->bits[k] = 0;
    }
    d->side = W.side;
    d->shift = 0;
    d->fine_bits = 0;
    d->cell_key_shift = 0;
    d->total_bits = 64;
    d->passes = 8;
    if (g.bad) d->status |= 1u;
  }
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < W.n; i += gridDim.x * kBlock) {
    const uint64_t key = box_key(W.pts[(size_t)i * 2]);
    W.keyA[i] = key;
    W.idxA[i] = (uint32_t)i;
    W.cnt[i] = 0;
    box_hist_add(s_hist, key, 8);
  }
  box_hist_flush(W, s_hist, 8);
}

// Before a further sort of the same call: histograms and tile counters cleared, the
// number of passes set (one workgroup).
__global__ __launch_bounds__(kBlock) void k_box_reset(Work W, int passes) {
  for (int i = threadIdx.x; i < 8 * 256; i += kBlock) W.ghist[i] = 0;
  if (threadIdx.x < 8) W.tilectr[threadIdx.x] = 0;
  if (threadIdx.x == 0) W.desc->passes = passes;
}

// Sort keys of the y coordinates, in input order.
__global__ __launch_bounds__(kBlock) void k_box_ykeys(Work W) {
  __shared__ uint32_t s_hist[8][256];
  for (int i = threadIdx.x; i < 8 * 256; i += kBlock) (&s_hist[0][0])[i] = 0;
  box_clear_lookback(W);
  __syncthreads();
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < W.n; i += gridDim.x * kBlock) {
    const uint64_t key = box_key(W.pts[(size_t)i * 2 + 1]);
    W.keyA[i] = key;
    W.idxA[i] = (uint32_t)i;
    box_hist_add(s_hist, key, 8);
  }
  box_hist_flush(W, s_hist, 8);
}

// Sort keys of the strips, in y order: a stable sort by them leaves each strip
// sorted by y (4 passes: strip ids are below 2^31).
__global__ __launch_bounds__(kBlock) void k_box_skeys(Work W) {
  __shared__ uint32_t s_hist[8][256];
  for (int i = threadIdx.x; i < 4 * 256; i += kBlock) (&s_hist[0][0])[i] = 0;
  box_clear_lookback(W);
  __syncthreads();
  for (int k = blockIdx.x * kBlock + threadIdx.x; k < W.n; k += gridDim.x * kBlock) {
    const uint64_t key = (uint64_t)(uint32_t)W.cellLabel[W.idxA[k]];
    W.keyA[k] = key;
    box_hist_add(s_hist, key, 4);
  }
  box_hist_flush(W, s_hist, 4);
}

// The y coordinates in (strip, y) order, as doubles in keyB.
__global__ __launch_bounds__(kBlock) void k_box_ygather(Work W) {
  double* ys = reinterpret_cast<double*>(W.keyB);
  for (int k = blockIdx.x * kBlock + threadIdx.x; k < W.n; k += gridDim.x * kBlock)
    ys[k] = W.pts[(size_t)W.idxA[k] * 2 + 1];
}

// Parents and first marks.  axis 0: the points in x order (keyA holds the x keys);
// the parent of k is the first point whose x exceeds x_k + s, and the first point
// is marked.  axis 1: the points in (strip, y) order (keyA holds the strip ids,
// keyB the y values); the parent of k is the first point of its strip whose y
// exceeds y_k + s, else the first point of the next strip, and the first point of
// every strip is marked.  n stands for "no parent".
__global__ __launch_bounds__(kBlock) void k_box_parent(Work W, int axis) {
  const int n = W.n;
  const double s = W.side;
  const double* ys = reinterpret_cast<const double*>(W.keyB);
  for (int k = blockIdx.x * kBlock + threadIdx.x; k < n; k += gridDim.x * kBlock) {
    int end = n;
    double t;
    bool first;
    if (axis == 0) {
      t = box_val(W.keyA[k]) + s;
      first = k == 0;
    } else {
      const uint64_t sk = W.keyA[k];
      first = k == 0 || W.keyA[k - 1] != sk;
      // end of the strip: the first position after k with a larger strip id
      int lo = k + 1, hi = n;
      while (lo < hi) {
        const int mid = lo + (hi - lo) / 2;
        if (W.keyA[mid] > sk) hi = mid;
        else lo = mid + 1;
      }
      end = lo;
      t = ys[k] + s;
    }
    // the first position in (k, end) whose coordinate exceeds t, else end
    int lo = k + 1, hi = end;
    while (lo < hi) {
      const int mid = lo + (hi - lo) / 2;
      const double v = axis == 0 ? box_val(W.keyA[mid]) : ys[mid];
      if (v > t) hi = mid;
      else lo = mid + 1;
    }
    W.parent[k] = lo;
    W.coreCount[k] = first ? 1 : 0;
  }
}

// One round of pointer jumping: a marked point marks its pointer's target, and every
// pointer jumps to its target's pointer (the pointer arrays alternate between
// rounds).  A mark only ever reaches points on a chain from a first mark, so marks
// written while the round runs are harmless; after r rounds every point within
// 2^r - 1 steps of a first mark is marked.
__global__ __launch_bounds__(kBlock) void k_box_jump(Work W, int round) {
  const int n = W.n;
  const int32_t* jin = (round & 1) ? W.minIdx : W.parent;
  int32_t* jout = (round & 1) ? W.parent : W.minIdx;
  for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) {
    const int j = jin[v];
    if (j < n) {
      if (W.coreCount[v]) W.coreCount[j] = 1;
      jout[v] = jin[j];
    } else {
      jout[v] = n;
    }
  }
}

// Inclusive scan of the marks, minus one: the strip (or box) of every position.
// Three launches: block sums, their exclusive scan (one workgroup), and the
// scan inside each block with its offset, written out by `stage`:
//   0: the strip of each input point (cellLabel, positions in x order);
//   1: the box ids as the sorted keys for k_cells (keyA, positions in (strip, y) order).
__global__ __launch_bounds__(kBlock) void k_box_scan_sums(Work W) {
  __shared__ uint32_t s_tmp[kWavesPerBlock];
  const int n = W.n;
  const int b = blockIdx.x;
  int sum = 0;
  for (int i = b * kBoxScanItems + threadIdx.x; i < min(n, (b + 1) * kBoxScanItems); i += kBlock)
    sum += W.coreCount[i];
  const int w = threadIdx.x / kWave;
  const int ws = wave_sum(sum);
  if (lane_id() == 0) s_tmp[w] = (uint32_t)ws;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int j = 0; j < kWavesPerBlock; ++j) t += (int)s_tmp[j];
    W.sublist[b] = t;
  }
}

__global__ __launch_bounds__(kBlock) void k_box_scan_top(Work W, int nb) {
  __shared__ uint32_t s_tmp[kWavesPerBlock];
  __shared__ int s_carry;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (int base = 0; base < nb; base += kBlock) {
    const int i = base + threadIdx.x;
    const int v = i < nb ? W.sublist[i] : 0;
    const uint32_t ex = block_excl_scan_256((uint32_t)v, s_tmp);
    const int carry = s_carry;
    if (i < nb) W.sublist[i] = carry + (int)ex;
    __syncthreads();
    if (threadIdx.x == kBlock - 1) s_carry = carry + (int)ex + v;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void k_box_scan_out(Work W, int stage) {
  __shared__ uint32_t s_tmp[kWavesPerBlock];
  __shared__ int s_tot;
  const int n = W.n;
  const int b = blockIdx.x;
  int run = W.sublist[b];
  for (int base = b * kBoxScanItems; base < min(n, (b + 1) * kBoxScanItems); base += kBlock) {
    const int i = base + threadIdx.x;
    const int v = i < n ? W.coreCount[i] : 0;
    const uint32_t ex = block_excl_scan_256((uint32_t)v, s_tmp);
    if (i < n) {
      const int id = run + (int)ex + v - 1;
      if (stage == 0) W.cellLabel[W.idxA[i]] = id;
      else W.keyA[i] = (uint64_t)(uint32_t)id;
    }
    if (threadIdx.x == kBlock - 1) s_tot = (int)ex + v;
    __syncthreads();
    run += s_tot;
    __syncthreads();
  }
}

}  // namespace db
