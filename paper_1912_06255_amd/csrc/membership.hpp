// Full cluster membership (paper, section "Preliminaries"; Algorithm 4 before its
// reduction to one id): a core point belongs to its own cluster, a non-core point to
// every cluster with a core point within eps (several are possible: border points
// do not merge clusters), noise to none.  Computed after a call from the state it
// leaves in the scratch (sorted points, core flags, cell labels, box tree), as CSR
// arrays in input order.  Every decision is the float64 test D <= E2.
#pragma once

#include "cluster.hpp"

namespace db {

constexpr int kMaxMembers = 256;  // distinct clusters around one point (8D packing bound: 240)

// Collects the labels of the core cells that hold a point within eps of one query
// point p into a per-wave LDS set.  A cell whose label is already in the set is
// skipped without distance tests (all core points of a cell share one label).
template <int D>
struct MemberVisitor {
  static constexpr bool kNearestFirst = false;
  DB_DEV bool keep_node(int, int) const { return true; }
  const Work* W;
  int* set;       // [kMaxMembers] LDS
  int ns;         // set size (wave-uniform)
  int overflow;   // set when more than kMaxMembers distinct labels were seen
  double p[D];    // the query point (wave-uniform)

  DB_DEV bool in_set(int lab) const {
    bool hit = false;
    for (int b = 0; b < ns; b += kWave) {
      const int k = b + lane_id();
      hit |= k < ns && set[k] == lab;
    }
    return ballot(hit) != 0;
  }

  DB_DEV bool group(int cb, uint64_t m, double) {
    const int lane = lane_id();
    const int h = cb + lane;
    bool on = ((m >> lane) & 1ull) && W->coreCount[h] > 0;
    int lab = -1, s = 0, e = 0;
    if (on) {
      lab = W->cellLabel[h];
      s = W->cellStart[h];
      e = W->cellStart[h + 1];
    }
    uint64_t alive = ballot(on);
    while (alive) {
      const int c = __ffsll((long long)alive) - 1;
      alive &= alive - 1;
      const int lc = bcast(lab, c);
      if (in_set(lc)) continue;
      const int cs = bcast(s, c), ce = bcast(e, c);
      bool found = false;
      for (int q0 = cs; q0 < ce && !found; q0 += kWave) {
        const int q = q0 + lane;
        bool hit = false;
        if (q < ce && W->coreS[q] != 0) {
          double xq[D];
          load_point<D>(W->X, W->n, q, xq);
          hit = sqdist<D>(p, xq) <= W->E2;
        }
        found = ballot(hit) != 0;
      }
      if (!found) continue;
      if (ns < kMaxMembers) {
        wave_sync();
        if (lane == 0) set[ns] = lc;
        wave_sync();
        ++ns;
      } else {
        overflow = 1;
      }
    }
    return false;
  }
};

// phase 0: count[perm[i]] = number of clusters of sorted point i (int64);
// phase 1: the ids, ascending, at ids[offsets[perm[i]] ...].
// One wave handles 64 sorted positions at a time; core points are written by their
// lanes, each non-core point gets a walk of its own.
template <int D>
__global__ __launch_bounds__(kBlock) void k_member(Work W, int phase, int64_t* count,
                                                   const int64_t* offsets, int32_t* ids,
                                                   uint32_t* overflow) {
  __shared__ uint64_t s_m[kWavesPerBlock][kTreeLevels + 2];
  __shared__ int s_cb[kWavesPerBlock][kTreeLevels + 2];
  __shared__ int s_set[kWavesPerBlock][kMaxMembers];
  const int C = W.desc->n_cells;
  const int n = W.n;
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int nchunks = (n + kWave - 1) / kWave;
  for (int ch = blockIdx.x * kWavesPerBlock + w; ch < nchunks; ch += gridDim.x * kWavesPerBlock) {
    const int i = ch * kWave + lane;
    const bool valid = i < n;
    const bool core = valid && W.coreS[i] != 0;
    if (core) {
      const int src = W.perm[i];
      if (phase == 0) count[src] = 1;
      else ids[offsets[src]] = W.cellLabel[W.cellOf[i]];
    }
    uint64_t todo = ballot(valid && !core);
    while (todo) {
      const int t = __ffsll((long long)todo) - 1;
      todo &= todo - 1;
      const int pi = ch * kWave + t;
      MemberVisitor<D> v;
      v.W = &W;
      v.set = s_set[w];
      v.ns = 0;
      v.overflow = 0;
      load_point<D>(W.X, n, pi, v.p);
      Query<D> q;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        q.lo[d] = v.p[d];
        q.hi[d] = v.p[d];
      }
      q.E2 = W.E2;
      walk<D>(W.tree, C, q, v, WalkStack{s_m[w], s_cb[w], nullptr});
      const int src = W.perm[pi];
      if (v.overflow && lane == 0) atomicOr(overflow, 1u);
      if (phase == 0) {
        if (lane == 0) count[src] = v.ns;
      } else {
        // ascending: rank of each set entry among the entries
        wave_sync();
        for (int b = 0; b < v.ns; b += kWave) {
          const int k = b + lane;
          if (k < v.ns) {
            const int x = v.set[k];
            int r = 0;
            for (int j = 0; j < v.ns; ++j) r += v.set[j] < x ? 1 : 0;
            ids[offsets[src] + r] = x;
          }
        }
        wave_sync();
      }
    }
  }
}

// Exclusive scan of int64 counts in three launches (tile sums, one workgroup over
// the tile sums, tiles with their prefix); offsets[n] receives the total.
constexpr int kScanTile = kBlock * 16;

__global__ __launch_bounds__(kBlock) void k_scan_tiles(const int64_t* in, int64_t n,
                                                       int64_t* tile_sum) {
  __shared__ int64_t s_part[kWavesPerBlock];
  const int64_t t = blockIdx.x;
  int64_t acc = 0;
  for (int j = threadIdx.x; j < kScanTile; j += kBlock) {
    const int64_t i = t * kScanTile + j;
    if (i < n) acc += in[i];
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, kWave);
  if (lane_id() == 0) s_part[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t s = 0;
    for (int k = 0; k < kWavesPerBlock; ++k) s += s_part[k];
    tile_sum[t] = s;
  }
}

// One workgroup: exclusive scan of the tile sums in place.
__global__ __launch_bounds__(kBlock) void k_scan_top(int64_t* tile_sum, int64_t ntiles) {
  __shared__ int64_t s_tot[kBlock];
  const int64_t per = (ntiles + kBlock - 1) / kBlock;
  const int64_t b = threadIdx.x * per, e = b + per < ntiles ? b + per : ntiles;
  int64_t s = 0;
  for (int64_t k = b; k < e; ++k) s += tile_sum[k];
  s_tot[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int k = 0; k < kBlock; ++k) {
      const int64_t v = s_tot[k];
      s_tot[k] = run;
      run += v;
    }
  }
  __syncthreads();
  int64_t run = s_tot[threadIdx.x];
  for (int64_t k = b; k < e; ++k) {
    const int64_t v = tile_sum[k];
    tile_sum[k] = run;
    run += v;
  }
}

__global__ __launch_bounds__(kBlock) void k_scan_apply(const int64_t* in, int64_t n,
                                                       const int64_t* tile_prefix,
                                                       int64_t* out) {
  __shared__ int64_t s_wave[kWavesPerBlock];
  const int64_t t = blockIdx.x;
  int64_t run = tile_prefix[t];
  const int w = threadIdx.x / kWave, lane = lane_id();
  for (int j0 = 0; j0 < kScanTile; j0 += kBlock) {
    const int64_t i = t * kScanTile + j0 + threadIdx.x;
    const int64_t v = i < n ? in[i] : 0;
    int64_t incl = v;
    for (int o = 1; o < kWave; o <<= 1) {
      const int64_t u = __shfl_up(incl, o, kWave);
      if (lane >= o) incl += u;
    }
    if (lane == kWave - 1) s_wave[w] = incl;
    __syncthreads();
    int64_t before = 0, total = 0;
    for (int k = 0; k < kWavesPerBlock; ++k) {
      if (k < w) before += s_wave[k];
      total += s_wave[k];
    }
    if (i < n) out[i] = run + before + incl - v;
    if (i == n - 1) out[n] = run + before + incl;
    run += total;
    __syncthreads();
  }
}

}  // namespace db
