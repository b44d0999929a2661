// MarkCore, ClusterCore and ClusterBorder for sparse grids: few points per cell, as
// in 5 and 7 dimensions at small eps or in clouds whose eps is small against their
// spread.  There the per-cell kernels of cluster.hpp spend one wave and one tree
// walk on a cell of one or two points, with most lanes idle.  Here a wave takes an
// aligned run of 64 sorted positions (points of consecutive cells in Morton order),
// one point per lane, splits the points it has to handle into compact batches, and
// walks the tree once per batch with the batch's point box as the query: every
// cell holding a point within eps of a batch point has a box within eps of that box
// (a monotone lower bound, as for one cell), so no candidate is missed.  The
// decisions are the same as in the per-cell kernels (float64, or the float32 filter
// with float64 recheck, with the offset of each pair's two cell anchors), so the
// results are identical.
//
// Measured on MI355X these kernels are slower than the per-cell ones on every
// workload tried (2D to 7D, 1 to 4 points per cell on average): a batch's union box
// admits more candidate cells than its points' own walks, and each lane still tests
// every candidate point.  They are kept behind an option (off by default) as a
// second implementation of the three steps, checked against the oracle.
#pragma once

#include "cluster.hpp"

namespace db {

// Per-lane state of one batch point: sorted position, cell, float64 coordinates and,
// in filter mode, the cell-local float32 coordinates and the cell's anchor.
template <int D, bool F32>
struct BatchPoint {
  int pos;   // sorted position, -1 for an idle lane
  int cell;
  double p[D];
  float ap[D];
  double ag[D];

  DB_DEV void load(const Work& W, int q, int c) {
    pos = q;
    cell = c;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      p[d] = 0.0;
      ap[d] = 0.0f;
      ag[d] = 0.0;
    }
    if (q < 0) return;
    load_point<D>(W.X, W.n, q, p);
    if constexpr (F32) {
      load_local<D>(W.X32, W.n, q, ap);
      load_anchor<D>(W.tree, c, ag);
    }
  }

  // Bounding box of the active lanes' points (the walk's query).
  DB_DEV void box(bool active, Query<D>& q) const {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      q.lo[d] = wave_min(active ? p[d] : __builtin_inf());
      q.hi[d] = wave_max(active ? p[d] : -__builtin_inf());
    }
  }
};

// A batch is kept compact: consecutive cells in Morton order can lie far apart (at
// the edges of the order's blocks), and one batch spanning two of them would walk
// the whole space between.  Of the lanes in `in` (taken in lane order), the batch is
// the longest run whose points' box spans at most `lim` (the radius) in every
// dimension; it holds at least the first of them.
template <int D>
DB_DEV uint64_t compact_batch(const double (&p)[D], bool in, double lim) {
  const int lane = lane_id();
  bool bad = false;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    double mn = in ? p[d] : __builtin_inf();
    double mx = in ? p[d] : -__builtin_inf();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const double a = __shfl_up(mn, o, kWave);
      const double b = __shfl_up(mx, o, kWave);
      if (lane >= o) {
        mn = fmin(mn, a);
        mx = fmax(mx, b);
      }
    }
    bad |= in && !(mx - mn <= lim);
  }
  const uint64_t all = ballot(in);
  const uint64_t bm = ballot(bad);
  return bm ? all & ((1ull << (__ffsll((long long)bm) - 1)) - 1ull) : all;
}

// One pair decision: batch point t (broadcast from its lane) against this lane's
// candidate q (sorted position qi, cell anchor ah in filter mode).  `cand` masks the
// lanes that take part.
template <int D, bool F32>
DB_DEV bool batch_hit(const Work* W, const BatchPoint<D, F32>& B, int t, bool cand,
                      const double (&xq)[D], const float (&aq)[D], const double (&ah)[D],
                      int qi, float tin, float tout, double e2, unsigned long long& rechecks) {
  if constexpr (F32) {
    float at[D], off[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      at[d] = bcast(B.ap[d], t);
      // T = fl32(fl64(A_g - A_h)) for p's cell g and q's cell h, as anchor_offsets
      off[d] = (float)(bcast(B.ag[d], t) - ah[d]);
    }
    return filtered_hit<D>(W, cand, at, aq, off, tin, tout, bcast(B.pos, t), qi, rechecks, e2);
  } else {
    double xp[D];
#pragma unroll
    for (int d = 0; d < D; ++d) xp[d] = bcast(B.p[d], t);
    return cand && sqdist<D>(xp, xq) <= e2;
  }
}

// Loads the candidate held by flattened position k of F (its cell is cb + j).
template <int D, bool F32>
DB_DEV void load_candidate(const Work& W, const Flat& F, int cb, int k, bool valid, int& j,
                           int& q, double (&xq)[D], float (&aq)[D], double (&ah)[D]) {
  j = 0;
  q = 0;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    xq[d] = 0.0;
    aq[d] = 0.0f;
    ah[d] = 0.0;
  }
  if (!valid) return;
  locate(F, k, j, q);
  if constexpr (F32) {
    load_local<D>(W.X32, W.n, q, aq);
    load_anchor<D>(W.tree, cb + j, ah);
  } else {
    load_point<D>(W.X, W.n, q, xq);
  }
}

// ---------------------------------------------------------------------------
// MarkCore: each batch point starts from the size of its own (safe) cell and adds
// the points within eps of the other cells met by the walk, up to count_cap.
// ---------------------------------------------------------------------------
template <int D, bool F32>
struct SparseCountVisitor {
  static constexpr bool kNearestFirst = true;
  DB_DEV bool keep_node(int, int) const { return true; }
  const Work* W;
  Flat F;
  BatchPoint<D, F32> B;
  int cnt;
  uint64_t pending;  // lanes still below the cap
  float tin, tout;
  Counters ctr;

  DB_DEV bool group(int cb, uint64_t m, double) {
    const int lane = lane_id();
    const int tot = flatten(F, W->cellStart, cb, m);
    for (int base = 0; base < tot; base += kWave) {
      const int k = base + lane;
      const bool valid = k < tot;
      int j, q;
      double xq[D], ah[D];
      float aq[D];
      load_candidate<D, F32>(*W, F, cb, k, valid, j, q, xq, aq, ah);
      const int hq = cb + j;
      for (uint64_t pend = pending; pend; pend &= pend - 1) {
        const int t = __ffsll((long long)pend) - 1;
        // points of p's own cell are in its starting count
        const bool cand = valid && hq != bcast(B.cell, t);
        const bool hit =
            batch_hit<D, F32>(W, B, t, cand, xq, aq, ah, q, tin, tout, W->E2, ctr.rechecks);
        const int add = __popcll(ballot(hit));
        if (lane == t) cnt += add;
        if (bcast(cnt, t) >= W->count_cap) pending &= ~(1ull << t);
      }
      if (!pending) return true;
    }
    return false;
  }
};

template <int D, bool F32, class WS>
__global__ __launch_bounds__(kBlock) void k_markcore_sparse(WS ws) {
  ws.each_wave([&](const Work& W) {
    __shared__ int s_pref[kWavesPerBlock][kWave + 1];
    __shared__ int s_start[kWavesPerBlock][kWave];
    __shared__ uint64_t s_m[kWavesPerBlock][kTreeLevels + 2];
    __shared__ int s_cb[kWavesPerBlock][kTreeLevels + 2];
    __shared__ double s_dist[kWavesPerBlock][(kTreeLevels + 2) * 64];
    const int C = W.desc->n_cells, n = W.n;
    const int w = threadIdx.x / kWave, lane = lane_id();
    const int cap = W.count_cap;
    const double lim = sqrt(W.E2);
    Counters tot;
    const UnitRange R = xcd_units((n + kWave - 1) / kWave);
    for (long long u = R.first; u < R.end; u += R.step) {
      const int i = (int)u * kWave + lane;
      const bool exists = i < n;
      int c = 0, m = 0;
      if (exists) {
        c = W.cellOf[i];
        m = W.cellStart[c + 1] - W.cellStart[c];
      }
      // a point of a cell of at least cap points has them within eps (the cell is safe)
      if (exists && m >= cap) W.cnt[i] = m;
      SparseCountVisitor<D, F32> v;
      v.W = &W;
      v.F = Flat{s_pref[w], s_start[w]};
      v.B.load(W, exists ? i : -1, c);
      v.tin = W.desc->tin;
      v.tout = W.desc->tout;
      const bool need = exists && m < cap;
      uint64_t rest = ballot(need);
      while (rest) {
        const uint64_t batch = compact_batch<D>(v.B.p, (rest >> lane) & 1ull, lim);
        rest &= ~batch;
        const bool in = (batch >> lane) & 1ull;
        v.cnt = m;
        v.pending = batch;
        Query<D> qb;
        qb.E2 = W.E2;
        v.B.box(in, qb);
        walk<D>(W.tree, C, qb, v, WalkStack{s_m[w], s_cb[w], s_dist[w]});
        if (in) W.cnt[i] = v.cnt;
      }
      tot.add(v.ctr);
    }
    tot.wave_flush(W.desc);
  });
}

// ---------------------------------------------------------------------------
// ClusterCore: each batch core point is tested against the core points of the
// cells met by the walk; a pair within eps links the two cells.  A cold run tests
// candidate cells of lower index than the point's own (each pair of cells once); a
// warm run from the previous setting's counts takes only the core points of cells
// that gained core points, against every other cell (see k_bcp).  Candidates
// already in the point's component are skipped (roots refreshed after each link).
// ---------------------------------------------------------------------------
template <int D, bool F32>
struct SparseLinkVisitor {
  static constexpr bool kNearestFirst = false;
  DB_DEV bool keep_node(int, int) const { return true; }
  const Work* W;
  Flat F;
  BatchPoint<D, F32> B;
  int root;          // lane t: a root of the component of its cell (stale is safe)
  uint64_t active;   // lanes holding a core point
  int hmax;          // candidate cells lie below the largest batch cell (cold runs)
  bool any_other;    // warm run: every other cell is a candidate
  float tin, tout;
  Counters ctr;

  DB_DEV bool group(int cb, uint64_t m, double) {
    const int lane = lane_id();
    const int h = cb + lane;
    bool on = ((m >> lane) & 1ull) && (any_other || h < hmax);
    if (on) on = W->coreCount[h] > 0;
    const uint64_t cells = ballot(on);
    if (!cells) return false;
    const int tot = flatten(F, W->cellStart, cb, cells);
    ctr.bcp += (unsigned long long)__popcll(cells);
    for (int base = 0; base < tot; base += kWave) {
      const int k = base + lane;
      bool valid = k < tot;
      int j, q;
      double xq[D], ah[D];
      float aq[D];
      load_candidate<D, F32>(*W, F, cb, k, valid, j, q, xq, aq, ah);
      const int hq = cb + j;
      int rq = -1;
      if (valid) {
        valid = (W->coreS[q] & W->core_mask) != 0;
        rq = uf_find(W->parent, hq);
      }
      if (!ballot(valid)) continue;
      for (uint64_t act = active; act; act &= act - 1) {
        const int t = __ffsll((long long)act) - 1;
        const int ct = bcast(B.cell, t);
        const int rt = bcast(root, t);
        const bool cand = valid && (any_other ? hq != ct : hq < ct) && rq != rt;
        if (!ballot(cand)) continue;
        ctr.pairs += (unsigned long long)__popcll(ballot(cand));
        const bool hit =
            batch_hit<D, F32>(W, B, t, cand, xq, aq, ah, q, tin, tout, W->E2b, ctr.rechecks);
        uint64_t hits = ballot(hit);
        if (!hits) continue;
        while (hits) {
          const int c = __ffsll((long long)hits) - 1;
          const int hc = bcast(hq, c);
          bool linked = false;
          if (lane == 0) linked = uf_link(W->parent, ct, hc);
          ctr.links += ballot(linked) ? 1ull : 0ull;
          hits &= ~ballot(hq == hc);
        }
        // components merged: refresh the roots on both sides
        if ((active >> lane) & 1ull) root = uf_find(W->parent, B.cell);
        if (valid) rq = uf_find(W->parent, hq);
      }
    }
    return false;
  }
};

template <int D, bool F32, bool WARM, class WS>
__global__ __launch_bounds__(kBlock) void k_bcp_sparse(WS ws) {
  ws.each_wave([&](const Work& W) {
    __shared__ int s_pref[kWavesPerBlock][kWave + 1];
    __shared__ int s_start[kWavesPerBlock][kWave];
    __shared__ uint64_t s_m[kWavesPerBlock][kTreeLevels + 2];
    __shared__ int s_cb[kWavesPerBlock][kTreeLevels + 2];
    const int C = W.desc->n_cells, n = W.n;
    const int w = threadIdx.x / kWave, lane = lane_id();
    const bool gained_only = WARM && W.prev_core_count != nullptr;
    const double lim = sqrt(W.E2);
    Counters tot;
    const UnitRange R = xcd_units((n + kWave - 1) / kWave);
    for (long long u = R.first; u < R.end; u += R.step) {
      const int i = (int)u * kWave + lane;
      bool need = i < n && (W.coreS[i] & W.core_mask) != 0;
      int c = 0;
      if (need) {
        c = W.cellOf[i];
        if (gained_only) need = W.coreCount[c] > W.prev_core_count[c];
      }
      uint64_t rest = ballot(need);
      if (!rest) continue;
      SparseLinkVisitor<D, F32> v;
      v.W = &W;
      v.F = Flat{s_pref[w], s_start[w]};
      v.B.load(W, need ? i : -1, c);
      v.any_other = gained_only;
      v.tin = W.desc->tinb;
      v.tout = W.desc->toutb;
      while (rest) {
        const uint64_t batch = compact_batch<D>(v.B.p, (rest >> lane) & 1ull, lim);
        rest &= ~batch;
        const bool in = (batch >> lane) & 1ull;
        v.active = batch;
        v.root = in ? uf_find(W.parent, c) : -1;
        v.hmax = wave_max(in ? c : -1);
        Query<D> qb;
        qb.E2 = W.E2;  // candidates within eps; only the pair test uses E2b
        v.B.box(in, qb);
        walk<D>(W.tree, C, qb, v, WalkStack{s_m[w], s_cb[w], nullptr});
      }
      tot.add(v.ctr);
    }
    tot.wave_flush(W.desc);
  });
}

// ---------------------------------------------------------------------------
// ClusterBorder: each batch non-core point starts from the id of its own cell (its
// core points are all within eps of it) and takes the smallest id among core
// points within eps in the cells met by the walk.
// ---------------------------------------------------------------------------
template <int D, bool F32>
struct SparseBorderVisitor {
  static constexpr bool kNearestFirst = false;
  DB_DEV bool keep_node(int, int) const { return true; }
  const Work* W;
  Flat F;
  BatchPoint<D, F32> B;
  int best;         // lane t: smallest id so far for its point
  uint64_t active;  // lanes holding a non-core point
  float tin, tout;
  Counters ctr;

  DB_DEV bool group(int cb, uint64_t m, double) {
    const int lane = lane_id();
    const int h = cb + lane;
    const int worst = wave_max(((active >> lane) & 1ull) ? best : -1);
    bool on = ((m >> lane) & 1ull) && W->coreCount[h] > 0;
    int lab = kIntMax;
    if (on) lab = W->cellLabel[h];
    on = on && lab < worst;
    const uint64_t cells = ballot(on);
    if (!cells) return false;
    const int tot = flatten(F, W->cellStart, cb, cells);
    for (int base = 0; base < tot; base += kWave) {
      const int k = base + lane;
      bool valid = k < tot;
      int j, q;
      double xq[D], ah[D];
      float aq[D];
      load_candidate<D, F32>(*W, F, cb, k, valid, j, q, xq, aq, ah);
      int lq = kIntMax;
      if (valid) {
        valid = (W->coreS[q] & W->core_mask) != 0;
        lq = W->cellLabel[cb + j];
      }
      if (!ballot(valid)) continue;
      for (uint64_t act = active; act; act &= act - 1) {
        const int t = __ffsll((long long)act) - 1;
        const int bt = bcast(best, t);
        const bool cand = valid && lq < bt;
        if (!ballot(cand)) continue;
        const bool hit =
            batch_hit<D, F32>(W, B, t, cand, xq, aq, ah, q, tin, tout, W->E2, ctr.rechecks);
        const int mn = wave_min(hit ? lq : kIntMax);
        if (lane == t && mn < best) best = mn;
      }
    }
    return false;
  }
};

template <int D, bool F32, class WS>
__global__ __launch_bounds__(kBlock) void k_border_sparse(WS ws) {
  ws.each_wave([&](const Work& W) {
    __shared__ int s_pref[kWavesPerBlock][kWave + 1];
    __shared__ int s_start[kWavesPerBlock][kWave];
    __shared__ uint64_t s_m[kWavesPerBlock][kTreeLevels + 2];
    __shared__ int s_cb[kWavesPerBlock][kTreeLevels + 2];
    const int C = W.desc->n_cells, n = W.n;
    const int w = threadIdx.x / kWave, lane = lane_id();
    const double lim = sqrt(W.E2);
    Counters tot;
    const UnitRange R = xcd_units((n + kWave - 1) / kWave);
    for (long long u = R.first; u < R.end; u += R.step) {
      const int i = (int)u * kWave + lane;
      bool need = i < n && (W.coreS[i] & W.core_mask) == 0;
      int c = 0, own = kIntMax;
      if (need) {
        c = W.cellOf[i];
        own = W.coreCount[c] > 0 ? W.cellLabel[c] : kIntMax;
        // no neighbour outside its cell (exact count of a non-core point, |c| included)
        if (W.cnt[i] == W.cellStart[c + 1] - W.cellStart[c]) {
          W.blabel[i] = own == kIntMax ? -1 : own;
          need = false;
        }
      }
      uint64_t rest = ballot(need);
      if (!rest) continue;
      SparseBorderVisitor<D, F32> v;
      v.W = &W;
      v.F = Flat{s_pref[w], s_start[w]};
      v.B.load(W, need ? i : -1, c);
      v.tin = W.desc->tin;
      v.tout = W.desc->tout;
      while (rest) {
        const uint64_t batch = compact_batch<D>(v.B.p, (rest >> lane) & 1ull, lim);
        rest &= ~batch;
        const bool in = (batch >> lane) & 1ull;
        v.active = batch;
        v.best = own;
        Query<D> qb;
        qb.E2 = W.E2;
        v.B.box(in, qb);
        walk<D>(W.tree, C, qb, v, WalkStack{s_m[w], s_cb[w], nullptr});
        if (in) W.blabel[i] = v.best == kIntMax ? -1 : v.best;
      }
      tot.add(v.ctr);
    }
    tot.wave_flush(W.desc);
  });
}

}  // namespace db
