// MarkCore (paper, Algorithm 2), ClusterCore with BCP cell connectivity and a
// lock-free union-find (Algorithm 3, section "Cluster Core"), canonical relabelling,
// and ClusterBorder (Algorithm 4).  One wavefront owns one cell; neighbour cells
// come from a wave-wide walk of the 64-ary box tree (grid.hpp).
#pragma once

#include "grid.hpp"

namespace db {

constexpr int kIntMax = 0x7fffffff;

// ---------------------------------------------------------------------------
// Tree walk.  Every node whose box can hold a point within eps of the query box
// (box_sqdist <= E2) is entered; at level 1 the surviving cells of the node's
// 64-cell group go to the visitor as a bit mask.  A visitor returning true stops
// the walk (early exit).
// ---------------------------------------------------------------------------
template <int D>
struct Query {
  double lo[D];
  double hi[D];
  double E2;
};

template <int D, int L, class V>
DB_DEV bool visit_node(const TreeView& T, const int (&cnt)[kTreeLevels + 2], int node,
                       const Query<D>& q, V& vis) {
  const int cb = node * 64;
  const int ch = cb + lane_id();
  bool ok = false;
  if (ch < cnt[L - 1]) ok = box_sqdist<D>(q.lo, q.hi, T.lo[L - 1], T.hi[L - 1], T.cap[L - 1], ch) <= q.E2;
  uint64_t m = ballot(ok);
  if constexpr (L == 1) {
    return m ? vis.group(cb, m) : false;
  } else {
    while (m) {
      const int j = __ffsll((long long)m) - 1;
      m &= m - 1;
      if (visit_node<D, L - 1, V>(T, cnt, cb + j, q, vis)) return true;
    }
    return false;
  }
}

template <int D, class V>
DB_DEV void walk(const TreeView& T, int C, const Query<D>& q, V& vis) {
  int cnt[kTreeLevels + 2];
  cnt[0] = C;
#pragma unroll
  for (int l = 1; l < kTreeLevels + 2; ++l) cnt[l] = (cnt[l - 1] + 63) >> 6;
  // top = first node level with at most 64 nodes; the walk starts at a virtual
  // parent one level above whose only child group is that level.
  if (cnt[1] <= 64) visit_node<D, 2, V>(T, cnt, 0, q, vis);
  else if (cnt[2] <= 64) visit_node<D, 3, V>(T, cnt, 0, q, vis);
  else if (cnt[3] <= 64) visit_node<D, 4, V>(T, cnt, 0, q, vis);
  else if (cnt[4] <= 64) visit_node<D, 5, V>(T, cnt, 0, q, vis);
  else visit_node<D, 6, V>(T, cnt, 0, q, vis);
}

// The tree has kTreeLevels node levels; visit_node<.., 6> reads level 5 boxes.
static_assert(kTreeLevels == 5, "walk() dispatch assumes five node levels");

// ---------------------------------------------------------------------------
// Flattening the points of the masked cells of a 64-cell group so that the 64
// lanes cover consecutive points of several small cells at once.
// ---------------------------------------------------------------------------
struct Flat {
  int* pref;   // [65] exclusive prefix of point counts over the group's cells
  int* start;  // [64] first sorted position of each cell
};

DB_DEV int flatten(const Flat& F, const int32_t* cellStart, int cb, uint64_t m) {
  const int lane = lane_id();
  wave_sync();  // earlier reads of F by this wave are done before it is rewritten
  const bool on = (m >> lane) & 1ull;
  int s = 0, cnt = 0;
  if (on) {
    s = cellStart[cb + lane];
    cnt = cellStart[cb + lane + 1] - s;
  }
  const int incl = wave_incl_scan(cnt);
  F.pref[lane] = incl - cnt;
  F.start[lane] = s;
  if (lane == kWave - 1) F.pref[kWave] = incl;
  wave_sync();
  return __shfl(incl, kWave - 1, kWave);
}

// k-th flattened point -> (group-local cell j, sorted position q).
DB_DEV void locate(const Flat& F, int k, int& j, int& q) {
  int lo = 0, hi = kWave;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (F.pref[mid] <= k) lo = mid;
    else hi = mid;
  }
  j = lo;
  q = F.start[lo] + (k - F.pref[lo]);
}

template <int D>
DB_DEV void load_point(const double* X, int n, int q, double (&x)[D]) {
#pragma unroll
  for (int k = 0; k < D; ++k) x[k] = X[(size_t)k * n + q];
}

template <int D>
DB_DEV void load_box(const TreeView& T, int c, Query<D>& q) {
#pragma unroll
  for (int k = 0; k < D; ++k) {
    q.lo[k] = T.lo[0][(size_t)k * T.cap[0] + c];
    q.hi[k] = T.hi[0][(size_t)k * T.cap[0] + c];
  }
}

// ---------------------------------------------------------------------------
// Union-find over cells.  parent[x] <= x always: links hang the larger root under
// the smaller with a CAS on the root, and path halving only ever stores an
// ancestor, so racing finds and links stay consistent.
// ---------------------------------------------------------------------------
DB_DEV int uf_find(int32_t* parent, int x) {
  while (true) {
    const int p = ld_acq(&parent[x]);
    if (p == x) return x;
    const int gp = ld_acq(&parent[p]);
    if (gp != p) st_rel(&parent[x], gp);
    x = gp;
  }
}

DB_DEV bool uf_link(int32_t* parent, int a, int b) {
  while (true) {
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    if (a == b) return false;
    if (a < b) {
      const int t = a;
      a = b;
      b = t;
    }
    const int old = atomicCAS(&parent[a], a, b);
    if (old == a) return true;
  }
}

// ---------------------------------------------------------------------------
// MarkCore (Algorithm 2).  A cell with at least minPts points is all core (its
// points are pairwise within eps: the diameter guard holds for every cell after
// splitting).  Otherwise each point starts from |g| and adds the points within
// eps in neighbour cells; it stops as soon as minPts is reached (early exit; the
// result is the same as counting everything).
// ---------------------------------------------------------------------------
template <int D>
struct MarkCoreVisitor {
  const Work* W;
  Flat F;
  int g, ps, pm;
  int cnt;           // lane t: count of point ps + t
  uint64_t pending;  // points of the batch still below minPts
  double p[D];       // lane t: coordinates of point ps + t

  DB_DEV bool group(int cb, uint64_t m) {
    if (g >= cb && g < cb + 64) m &= ~(1ull << (g - cb));
    if (!m) return false;
    const int n = W->n;
    const int tot = flatten(F, W->cellStart, cb, m);
    const int lane = lane_id();
    for (int base = 0; base < tot; base += kWave) {
      const int k = base + lane;
      const bool valid = k < tot;
      double xq[D];
      if (valid) {
        int j, q;
        locate(F, k, j, q);
        load_point<D>(W->X, n, q, xq);
      } else {
#pragma unroll
        for (int d = 0; d < D; ++d) xq[d] = 0.0;
      }
      uint64_t pend = pending;
      while (pend) {
        const int t = __ffsll((long long)pend) - 1;
        pend &= pend - 1;
        double xp[D];
#pragma unroll
        for (int d = 0; d < D; ++d) xp[d] = __shfl(p[d], t, kWave);
        const bool hit = valid && sqdist<D>(xp, xq) <= W->E2;
        const int add = __popcll(ballot(hit));
        if (lane == t) cnt += add;
        const int ct = __shfl(cnt, t, kWave);
        if (ct >= W->minPts) pending &= ~(1ull << t);
      }
      if (!pending) return true;
    }
    return false;
  }
};

template <int D>
__global__ __launch_bounds__(kBlock) void k_markcore(Work W) {
  __shared__ int s_pref[kWavesPerBlock][kWave + 1];
  __shared__ int s_start[kWavesPerBlock][kWave];
  const int C = W.desc->n_cells;
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int n = W.n;
  for (int g = blockIdx.x * kWavesPerBlock + w; g < C; g += gridDim.x * kWavesPerBlock) {
    const int s = W.cellStart[g], e = W.cellStart[g + 1], m = e - s;
    if (m >= W.minPts) {
      for (int i = s + lane; i < e; i += kWave) W.coreS[i] = 1;
      continue;
    }
    Query<D> q;
    q.E2 = W.E2;
    load_box<D>(W.tree, g, q);
    for (int ps = s; ps < e; ps += kWave) {
      MarkCoreVisitor<D> v;
      v.W = &W;
      v.F = Flat{s_pref[w], s_start[w]};
      v.g = g;
      v.ps = ps;
      v.pm = min(kWave, e - ps);
      v.cnt = m;
      v.pending = v.pm == kWave ? ~0ull : ((1ull << v.pm) - 1ull);
      if (lane < v.pm) load_point<D>(W.X, n, ps + lane, v.p);
      else {
#pragma unroll
        for (int d = 0; d < D; ++d) v.p[d] = 0.0;
      }
      walk<D>(W.tree, C, q, v);
      if (lane < v.pm) W.coreS[ps + lane] = v.cnt >= W.minPts ? 1 : 0;
    }
  }
}

// Core points per cell, union-find and relabel initialisation.
__global__ void k_core_count(Work W) {
  const int C = W.desc->n_cells;
  int ncore = 0;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < C; c += gridDim.x * blockDim.x) {
    const int s = W.cellStart[c], e = W.cellStart[c + 1];
    int cc = e - s;
    if (cc < W.minPts) {
      cc = 0;
      for (int i = s; i < e; ++i) cc += W.coreS[i];
    }
    W.coreCount[c] = cc;
    W.parent[c] = c;
    W.minIdx[c] = kIntMax;
    ncore += cc;
  }
  ncore = wave_sum(ncore);
  if (lane_id() == 0 && ncore) atomicAdd(&W.desc->n_core, ncore);
}

// ---------------------------------------------------------------------------
// ClusterCore (Algorithm 3).  For core cell g and each core neighbour h with
// h < g whose union-find root differs from g's, test pairs of core points of g
// and h (BCP with early exit: the first pair within eps links the cells).  Points
// of g are first filtered by their box distance to the live neighbour cells
// (the paper's filter of points farther than eps from the other cell).
// ---------------------------------------------------------------------------
template <int D>
struct BcpVisitor {
  const Work* W;
  Flat F;
  int g, gs, ge;
  bool gdense;

  DB_DEV bool group(int cb, uint64_t m) {
    const int lane = lane_id();
    const int n = W->n;
    const int h = cb + lane;
    bool on = ((m >> lane) & 1ull) && h < g && W->coreCount[h] > 0;
    const int rg = uf_find(W->parent, g);
    if (on) on = uf_find(W->parent, h) != rg;
    uint64_t alive = ballot(on);
    if (!alive) return false;
    if (lane == 0) atomicAdd(&W->desc->bcp_calls, (unsigned long long)__popcll(alive));
    // union box of the live cells
    Query<D> ub;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const double a = on ? W->tree.lo[0][(size_t)d * W->tree.cap[0] + h] : __builtin_inf();
      const double b = on ? W->tree.hi[0][(size_t)d * W->tree.cap[0] + h] : -__builtin_inf();
      ub.lo[d] = wave_min(a);
      ub.hi[d] = wave_max(b);
    }
    const int tot = flatten(F, W->cellStart, cb, alive);
    for (int base = 0; base < tot && alive; base += kWave) {
      const int k = base + lane;
      bool valid = k < tot;
      int j = 0, q = 0;
      double xq[D];
      if (valid) {
        locate(F, k, j, q);
        valid = W->coreS[q] != 0 && ((alive >> j) & 1ull);
      }
      if (valid) load_point<D>(W->X, n, q, xq);
      else {
#pragma unroll
        for (int d = 0; d < D; ++d) xq[d] = 0.0;
      }
      if (!ballot(valid)) continue;
      for (int p = gs; p < ge; ++p) {
        if (!gdense && !W->coreS[p]) continue;
        double xp[D];
        load_point<D>(W->X, n, p, xp);
        if (box_sqdist<D>(xp, xp, ub.lo, ub.hi, 1, 0) > W->E2) continue;
        const bool hit = valid && sqdist<D>(xp, xq) <= W->E2;
        if (ballot(hit)) {
          const uint64_t cells = wave_or(hit ? (1ull << j) : 0ull);
          if (lane == 0) {
            unsigned long long links = 0;
            uint64_t cm = cells;
            while (cm) {
              const int b = __ffsll((long long)cm) - 1;
              cm &= cm - 1;
              links += uf_link(W->parent, g, cb + b) ? 1 : 0;
            }
            if (links) atomicAdd(&W->desc->uf_links, links);
          }
          alive &= ~cells;
          valid = valid && ((alive >> j) & 1ull);
          if (!ballot(valid)) break;
        }
      }
    }
    return false;
  }
};

template <int D>
__global__ __launch_bounds__(kBlock) void k_bcp(Work W) {
  __shared__ int s_pref[kWavesPerBlock][kWave + 1];
  __shared__ int s_start[kWavesPerBlock][kWave];
  const int C = W.desc->n_cells;
  const int w = threadIdx.x / kWave;
  for (int g = blockIdx.x * kWavesPerBlock + w; g < C; g += gridDim.x * kWavesPerBlock) {
    if (W.coreCount[g] == 0) continue;
    BcpVisitor<D> v;
    v.W = &W;
    v.F = Flat{s_pref[w], s_start[w]};
    v.g = g;
    v.gs = W.cellStart[g];
    v.ge = W.cellStart[g + 1];
    v.gdense = W.coreCount[g] == v.ge - v.gs;
    Query<D> q;
    q.E2 = W.E2;
    load_box<D>(W.tree, g, q);
    walk<D>(W.tree, C, q, v);
  }
}

// ---------------------------------------------------------------------------
// Canonical ids: the cluster id is the smallest input index of a core point in
// the component.  Each wave takes 64 cells, reduces the minimum per distinct root
// among them and issues one atomicMin per root.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_relabel_min(Work W) {
  const int C = W.desc->n_cells;
  const int lane = lane_id();
  const int nchunks = (C + kWave - 1) / kWave;
  for (int ch = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; ch < nchunks;
       ch += gridDim.x * kWavesPerBlock) {
    const int c = ch * kWave + lane;
    int root = -1, mn = kIntMax;
    if (c < C && W.coreCount[c] > 0) {
      root = uf_find(W.parent, c);
      const int s = W.cellStart[c], e = W.cellStart[c + 1];
      for (int i = s; i < e; ++i)
        if (W.coreS[i]) mn = min(mn, W.perm[i]);
    }
    uint64_t todo = ballot(root >= 0);
    while (todo) {
      const int leader = __ffsll((long long)todo) - 1;
      const int r = __shfl(root, leader, kWave);
      const bool mine = root == r;
      const int v = wave_min(mine ? mn : kIntMax);
      if (lane == leader) atomicMin(&W.minIdx[r], v);
      todo &= ~ballot(mine);
    }
  }
}

__global__ void k_cell_label(Work W) {
  const int C = W.desc->n_cells;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < C; c += gridDim.x * blockDim.x) {
    W.cellLabel[c] = W.coreCount[c] > 0 ? W.minIdx[uf_find(W.parent, c)] : -1;
  }
}

// ---------------------------------------------------------------------------
// ClusterBorder (Algorithm 4), reduced to the smallest id: a non-core point takes
// the smallest cluster id among core points within eps.  All core points of one
// cell share one id, so a neighbour cell whose id is not below the current best
// is skipped without distance tests.
// ---------------------------------------------------------------------------
template <int D>
struct BorderVisitor {
  const Work* W;
  Flat F;
  int g, pm;
  int best;          // lane t: best id so far for batch point t
  double p[D];       // lane t: coordinates of batch point t

  DB_DEV bool group(int cb, uint64_t m) {
    const int lane = lane_id();
    const int n = W->n;
    if (g >= cb && g < cb + 64) m &= ~(1ull << (g - cb));
    const int h = cb + lane;
    const int worst = wave_max(lane < pm ? best : -1);
    bool on = ((m >> lane) & 1ull) && W->coreCount[h] > 0;
    int lab = kIntMax;
    if (on) lab = W->cellLabel[h];
    on = on && lab < worst;
    const uint64_t alive = ballot(on);
    if (!alive) return false;
    const int tot = flatten(F, W->cellStart, cb, alive);
    for (int base = 0; base < tot; base += kWave) {
      const int k = base + lane;
      bool valid = k < tot;
      int j = 0, q = 0, lq = kIntMax;
      double xq[D];
      if (valid) {
        locate(F, k, j, q);
        valid = W->coreS[q] != 0;
      }
      if (valid) {
        lq = W->cellLabel[cb + j];
        load_point<D>(W->X, n, q, xq);
      } else {
#pragma unroll
        for (int d = 0; d < D; ++d) xq[d] = 0.0;
      }
      for (int t = 0; t < pm; ++t) {
        const int bt = __shfl(best, t, kWave);
        const bool cand = valid && lq < bt;
        if (!ballot(cand)) continue;
        double xp[D];
#pragma unroll
        for (int d = 0; d < D; ++d) xp[d] = __shfl(p[d], t, kWave);
        const bool hit = cand && sqdist<D>(xp, xq) <= W->E2;
        const int mn = wave_min(hit ? lq : kIntMax);
        if (lane == t && mn < best) best = mn;
      }
    }
    return false;
  }
};

template <int D>
__global__ __launch_bounds__(kBlock) void k_border(Work W) {
  __shared__ int s_pref[kWavesPerBlock][kWave + 1];
  __shared__ int s_start[kWavesPerBlock][kWave];
  __shared__ int s_pos[kWavesPerBlock][kWave];
  const int C = W.desc->n_cells;
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int n = W.n;
  for (int g = blockIdx.x * kWavesPerBlock + w; g < C; g += gridDim.x * kWavesPerBlock) {
    const int s = W.cellStart[g], e = W.cellStart[g + 1];
    if (W.coreCount[g] == e - s) continue;
    Query<D> q;
    q.E2 = W.E2;
    load_box<D>(W.tree, g, q);
    const int own = W.coreCount[g] > 0 ? W.cellLabel[g] : kIntMax;
    int i = s;
    while (i < e) {
      // compact the next (up to 64) non-core positions of g into s_pos
      int taken = 0;
      while (i < e && taken < kWave) {
        const int k = i + lane;
        const bool nc = k < e && W.coreS[k] == 0;
        const uint64_t bm = ballot(nc);
        const int rank = __popcll(bm & lanemask_lt());
        const int cnt = __popcll(bm);
        const int room = kWave - taken;
        if (nc && rank < room) s_pos[w][taken + rank] = k;
        if (cnt <= room) {
          taken += cnt;
          i += kWave;
        } else {
          const uint64_t lastm = ballot(nc && rank == room - 1);
          i += __ffsll((long long)lastm);  // one past the last lane taken
          taken = kWave;
        }
      }
      wave_sync();
      const int pos = lane < taken ? s_pos[w][lane] : -1;
      wave_sync();
      if (taken == 0) break;
      BorderVisitor<D> v;
      v.W = &W;
      v.F = Flat{s_pref[w], s_start[w]};
      v.g = g;
      v.pm = taken;
      v.best = own;
      if (lane < taken) load_point<D>(W.X, n, pos, v.p);
      else {
#pragma unroll
        for (int d = 0; d < D; ++d) v.p[d] = 0.0;
      }
      walk<D>(W.tree, C, q, v);
      if (lane < taken) W.blabel[pos] = v.best == kIntMax ? -1 : v.best;
    }
  }
}

// Results back to input order.
__global__ void k_scatter(Work W) {
  const int n = W.n;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int src = W.perm[i];
    const uint8_t c = W.coreS[i];
    W.core_out[src] = c;
    W.label_out[src] = c ? W.cellLabel[W.cellOf[i]] : W.blabel[i];
  }
}

}  // namespace db
