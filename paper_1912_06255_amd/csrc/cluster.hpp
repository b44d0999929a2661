// MarkCore (paper, Algorithm 2), ClusterCore with BCP cell connectivity and a
// lock-free union-find (Algorithm 3, section "Cluster Core"), canonical relabelling,
// and ClusterBorder (Algorithm 4).  One wavefront owns one cell; neighbour cells
// come from a wave-wide walk of the 64-ary box tree (grid.hpp).
#pragma once

#include "grid.hpp"

namespace db {

constexpr int kNodeNoCore = -2;
// Mean points per live neighbour cell from which ClusterCore handles a group cell
// by cell instead of flattening it, up to 3 dimensions (the default of
// Work::dense_group).
#ifndef DB_DENSE_GROUP
#define DB_DENSE_GROUP 8
#endif
constexpr int kDenseGroup = DB_DENSE_GROUP;
// In sub-cell order, MarkCore takes neighbour cells of at least this many points
// chunk by chunk with box tests.
#ifndef DB_LEAF_CELL
#define DB_LEAF_CELL 128
#endif
constexpr int kLeafCell = DB_LEAF_CELL;

// Cells of at least this many points are in sub-cell order (compact 64-point
// chunks): every cell from kLeafCell points on with sort-time fine bits, the
// cells k_subsort regrouped otherwise, none when both are off.
DB_DEV int leaf_min(const Work& W) {
  return W.desc->fine_bits > 0 ? kLeafCell : max(W.sub_min, kLeafCell);
}
// Waves per sparse cell in MarkCore (d <= 3; the default of Work::mark_split) ...
#ifndef DB_MARK_SPLIT
#define DB_MARK_SPLIT 4
#endif
constexpr int kMarkSplit = DB_MARK_SPLIT;
// ... when the grid holds at least this many points per cell on average.  In
// sparser grids every split wave would repeat a walk that finds little to share
// (3D clouds of 1.5 points per cell: 84 -> 17.5 ms of MarkCore with one wave).
#ifndef DB_MARK_SPLIT_MEAN
#define DB_MARK_SPLIT_MEAN 32
#endif
constexpr int kMarkSplitMean = DB_MARK_SPLIT_MEAN;
// Sparse grids (sparse.hpp): MarkCore, ClusterCore and ClusterBorder can instead batch
// the points of consecutive cells per tree walk (Work::sparse_mode 1, chosen by the
// host; the per-cell kernels below are then not launched).

// Smallest segment of a ClusterCore unit handled by a wave of its own.
#ifndef DB_BCP_SEGMENT
#define DB_BCP_SEGMENT 192
#endif
constexpr int kBcpSegment = DB_BCP_SEGMENT;
// ... and of at least kSegMean times the mean cell size: where most cells are
// large, cutting all of them only doubles the tests (each segment still meets
// every neighbour), while cutting the outsize ones shortens the kernel's tail.
constexpr int kSegMean = 1;

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

// Visitors provide:
//   static constexpr bool kNearestFirst  enter child nodes by increasing box distance
//   bool keep_node(int level, int idx)   false drops a node (level >= 1) unvisited
//   bool group(int first_cell, uint64_t mask, double dist)   dist: this lane's cell box
//                                        distance to the query (masked lanes only)
//
// The walk is iterative: one frame per tree level (the mask of children still to
// enter, their first index and, for nearest-first walks, their box distances) is
// kept in a per-wave LDS stack, so that the visitor's group() is expanded once.
struct WalkStack {
  uint64_t* m;   // [kTreeLevels + 2]
  int* cb;       // [kTreeLevels + 2]
  double* dist;  // [(kTreeLevels + 2) * 64], nearest-first walks only
};

// Number of nodes at level l for C cells (level 0 = cells).
DB_DEV int nodes_at(int C, int l) {
  return (int)(((long long)C + (1ll << (6 * l)) - 1) >> (6 * l));
}

// Children (at level L - 1) of node N at level L that can hold a point within eps
// of the query box.  dist: this lane's child box distance, +inf if dropped.
template <int D, class V>
DB_DEV uint64_t test_children(const TreeView& T, int C, int L, int N, const Query<D>& q, V& vis,
                              double& dist) {
  const int ch = N * 64 + lane_id();
  dist = __builtin_inf();
  if (ch < nodes_at(C, L - 1)) {
    const double bd = box_sqdist<D>(q.lo, q.hi, T.flo[L - 1], T.fhi[L - 1], T.cap[L - 1], ch);
    if (bd <= q.E2) dist = bd;
  }
  bool ok = dist <= q.E2;
  if (L >= 2 && ok) ok = vis.keep_node(L - 1, ch);
  if (!ok) dist = __builtin_inf();
  return ballot(ok);
}

// Walk the subtree of node `node` at level `level` (Leaf .. top + 1).  The visitor's
// group() gets the children (at level Leaf - 1) of each entered node of level Leaf:
// cells for Leaf = 1.
template <int D, class V, int Leaf = 1>
DB_DEV void walk_subtree(const TreeView& T, int C, int level, int node, const Query<D>& q, V& vis,
                         const WalkStack& S) {
  const int lane = lane_id();
  double dist;
  const uint64_t m0 = test_children<D>(T, C, level, node, q, vis, dist);
  if (level == Leaf) {
    if (m0) vis.group(node * 64, m0, dist);
    return;
  }
  int lvl = level;
  wave_sync();
  S.m[lvl] = m0;
  S.cb[lvl] = node * 64;
  if constexpr (V::kNearestFirst) S.dist[lvl * 64 + lane] = dist;
  wave_sync();
  while (true) {
    const uint64_t fm = S.m[lvl];
    if (!fm) {
      if (++lvl > level) break;
      continue;
    }
    int j;
    if constexpr (V::kNearestFirst) {
      const double dv = ((fm >> lane) & 1ull) ? S.dist[lvl * 64 + lane] : __builtin_inf();
      const double mind = wave_min(dv);
      j = __ffsll((long long)(ballot(dv == mind) & fm)) - 1;
    } else {
      j = __ffsll((long long)fm) - 1;
    }
    const int child = S.cb[lvl] + j;  // a node at level lvl - 1
    wave_sync();
    S.m[lvl] = fm & ~(1ull << j);
    wave_sync();
    double d2;
    const uint64_t m2 = test_children<D>(T, C, lvl - 1, child, q, vis, d2);
    if (!m2) continue;
    if (lvl - 1 == Leaf) {
      if (vis.group(child * 64, m2, d2)) return;
    } else {
      --lvl;
      wave_sync();
      S.m[lvl] = m2;
      S.cb[lvl] = child * 64;
      if constexpr (V::kNearestFirst) S.dist[lvl * 64 + lane] = d2;
      wave_sync();
    }
  }
}

DB_DEV void level_counts(int C, int (&cnt)[kTreeLevels + 2]) {
  cnt[0] = C;
#pragma unroll
  for (int l = 1; l < kTreeLevels + 2; ++l) cnt[l] = (cnt[l - 1] + 63) >> 6;
}

// Top node level: the first with at most 64 nodes.  The whole tree is the subtree
// of a virtual node (index 0) one level above it.
DB_DEV int top_level(const int (&cnt)[kTreeLevels + 2]) {
  int top = 1;
  while (top < kTreeLevels && cnt[top] > 64) ++top;
  return top;
}

template <int D, class V>
DB_DEV void walk(const TreeView& T, int C, const Query<D>& q, V& vis, const WalkStack& S) {
  int cnt[kTreeLevels + 2];
  level_counts(C, cnt);
  walk_subtree<D, V>(T, C, top_level(cnt) + 1, 0, q, vis, S);
}

// ---------------------------------------------------------------------------
// Node lists.  For each level-1 node (64 consecutive cells) the level-1 nodes whose
// box is within reach of its box, from one walk per node that stops at level 1.  A
// cell's box lies inside its node's box, so every node a walk from the cell would
// enter is in that list, and a walk from a cell can start from it instead of the
// root (one round of box tests for the whole list instead of one per tree level).
// Lists longer than kNodeList are marked -1; walks from their cells start at the
// root.  Built for d <= 3 only: in higher dimensions most lists overflow (node boxes
// are loose there) and building them cost more than it saved.
// ---------------------------------------------------------------------------
constexpr int kNodeList = 64;
constexpr int kNodeListMaxD = 3;

struct ListVisitor {
  static constexpr bool kNearestFirst = false;
  DB_DEV bool keep_node(int, int) const { return true; }
  int32_t* list;
  int len;
  // m: the level-1 nodes cb .. cb + 63 within reach
  DB_DEV bool group(int cb, uint64_t m, double) {
    const int lane = lane_id();
    const int pos = len + __popcll(m & lanemask_lt());
    if (((m >> lane) & 1ull) && pos < kNodeList) list[pos] = cb + lane;
    len += __popcll(m);
    return len > kNodeList;
  }
};

// (workgroup bid of the nwg doing this job)
template <int D>
DB_DEV void node_lists_part(const Work& W, int nwg, int bid) {
  __shared__ uint64_t s_m[kWavesPerBlock][kTreeLevels + 2];
  __shared__ int s_cb[kWavesPerBlock][kTreeLevels + 2];
  const int C = W.desc->n_cells;
  const int w = threadIdx.x / kWave;
  const UnitRange R = xcd_units_of(nodes_at(C, 1), nwg, bid);
  for (long long u = R.first; u < R.end; u += R.step) {
    const int G = (int)u;
    Query<D> q;
    q.E2 = W.E2;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      q.lo[d] = W.tree.lo[1][(size_t)d * W.tree.cap[1] + G];
      q.hi[d] = W.tree.hi[1][(size_t)d * W.tree.cap[1] + G];
    }
    ListVisitor v{W.nlist + (size_t)G * kNodeList, 0};
    int cnt[kTreeLevels + 2];
    level_counts(C, cnt);
    walk_subtree<D, ListVisitor, 2>(W.tree, C, top_level(cnt) + 1, 0, q, v,
                                    WalkStack{s_m[w], s_cb[w], nullptr});
    if (lane_id() == 0) W.nlen[G] = v.len > kNodeList ? -1 : v.len;
  }
}

template <int D, class WS>
__global__ __launch_bounds__(kBlock) void k_node_lists(WS ws) {
  ws.each_wave([&](const Work& W) {
    node_lists_part<D>(W, (int)gridDim.x, (int)blockIdx.x);
  });
}

// Node lists and the float32 coordinates in one launch (independent jobs): the
// first nbl workgroups build the lists, the others convert the coordinates.
template <int D, class WS>
__global__ __launch_bounds__(kBlock) void k_lists_local32(WS ws, int nbl) {
  ws.each_wave([&](const Work& W) {
    if ((int)blockIdx.x < nbl) node_lists_part<D>(W, nbl, (int)blockIdx.x);
    else local32_part<D>(W, W.eps, (int)gridDim.x - nbl, (int)blockIdx.x - nbl);
  });
}

// The walk of cell g from its node's list (or from the root if the list overflowed).
// It enters the same level-1 nodes as walk(): each listed node's box is tested
// against the query (one lane per node), then the passing nodes are entered in list
// order, or nearest first for visitors that ask for it.
template <int D, class V>
DB_DEV void walk_from_list(const Work& W, int C, int g, const Query<D>& q, V& vis,
                           const WalkStack& S) {
  if constexpr (D > kNodeListMaxD) {
    walk<D>(W.tree, C, q, vis, S);
    return;
  }
  const int G = g >> 6;
  const int len = W.nlen[G];
  if (len < 0) {
    walk<D>(W.tree, C, q, vis, S);
    return;
  }
  const int lane = lane_id();
  int node = 0;
  double dist = __builtin_inf();
  if (lane < len) {
    node = W.nlist[(size_t)G * kNodeList + lane];
    const double bd = box_sqdist<D>(q.lo, q.hi, W.tree.flo[1], W.tree.fhi[1], W.tree.cap[1], node);
    if (bd <= q.E2 && vis.keep_node(1, node)) dist = bd;
  }
  uint64_t todo = ballot(dist <= q.E2);
  while (todo) {
    int j;
    if constexpr (V::kNearestFirst) {
      const double dv = ((todo >> lane) & 1ull) ? dist : __builtin_inf();
      const double mind = wave_min(dv);
      j = __ffsll((long long)(ballot(dv == mind) & todo)) - 1;
    } else {
      j = __ffsll((long long)todo) - 1;
    }
    todo &= ~(1ull << j);
    const int N = __shfl(node, j, kWave);
    double d2;
    const uint64_t m2 = test_children<D>(W.tree, C, 1, N, q, vis, d2);
    if (m2 && vis.group(N * 64, m2, d2)) return;
  }
}


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

// Same, from per-lane (start, count) already loaded (count 0 for masked lanes).
DB_DEV int flatten_ranges(const Flat& F, int s, int cnt) {
  const int lane = lane_id();
  wave_sync();
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
// Reads are plain (cacheable) loads: a stale parent is still an ancestor, so a
// find may return a former root.  That only weakens pruning; links are decided by
// the CAS in uf_link, which continues from the value it reads.
DB_DEV int uf_find(int32_t* parent, int x) {
  while (true) {
    const int p = parent[x];
    if (p == x) return x;
    const int gp = parent[p];
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
    a = old;  // a was linked meanwhile: continue from its new parent
  }
}

// ---------------------------------------------------------------------------
// Pair decisions.  Float64 mode: D(p, q) <= E2 directly.  Float32 filter mode:
// decide32 on cell-local float32 coordinates; pairs in the error band are decided
// again in float64 from the float64 coordinates (and counted).
// ---------------------------------------------------------------------------
template <int D>
DB_DEV void load_local(const float* X32, int n, int q, float (&a)[D]) {
#pragma unroll
  for (int k = 0; k < D; ++k) a[k] = X32[(size_t)k * n + q];
}

template <int D>
DB_DEV void load_anchor(const TreeView& T, int c, double (&a)[D]) {
#pragma unroll
  for (int k = 0; k < D; ++k) a[k] = T.lo[0][(size_t)k * T.cap[0] + c];
}

// T = fl32(fl64(A_g - A_h)) for the anchor A_g of p's cell and q's cell h.
template <int D>
DB_DEV void anchor_offsets(const TreeView& T, const double (&ag)[D], int h, float (&off)[D]) {
#pragma unroll
  for (int k = 0; k < D; ++k) off[k] = (float)(ag[k] - T.lo[0][(size_t)k * T.cap[0] + h]);
}

template <int D>
DB_DEV bool recheck64(const Work* W, int pi, int qi, double e2) {
  double a[D], b[D];
  load_point<D>(W->X, W->n, pi, a);
  load_point<D>(W->X, W->n, qi, b);
  return sqdist<D>(a, b) <= e2;
}

// One pair per lane in filter mode: p (index pi, coordinates ap) broadcast, q per
// lane.  Returns whether q is within eps of p; band lanes are rechecked in float64
// against e2 (E2; ClusterCore passes its own threshold E2b >= E2: a pair the filter
// proves within eps links either way, one it proves beyond eps never does, which
// approximate DBSCAN allows).
template <int D>
DB_DEV bool filtered_hit(const Work* W, bool valid, const float (&ap)[D], const float (&aq)[D],
                         const float (&off)[D], float tin, float tout, int pi, int qi,
                         unsigned long long& rechecks, double e2) {
  const int cls = valid ? decide32<D>(ap, aq, off, tin, tout) : 0;
  bool hit = cls == 1;
  const uint64_t bm = ballot(cls == 2);
  if (bm) {
    if (cls == 2) hit = recheck64<D>(W, pi, qi, e2);
    rechecks += (unsigned long long)__popcll(bm);
  }
  return hit;
}

// Per-wave counters of one unit of work, flushed once with stat_add.
struct Counters {
  unsigned long long bcp = 0, links = 0, rechecks = 0, pairs = 0;
  DB_DEV void add(const Counters& o) {
    bcp += o.bcp;
    links += o.links;
    rechecks += o.rechecks;
    pairs += o.pairs;
  }
  // Once per wave, at the end of a kernel: the wave's totals over all its units,
  // one atomic per counter (no workgroup barrier: waves that finish early leave).
  DB_DEV void wave_flush(GridDesc* g) const {
    if (lane_id() == 0) {
      const int slot = (int)(blockIdx.x * kWavesPerBlock + threadIdx.x / kWave);
      stat_add_slot(g, kCtrBcp, slot, bcp);
      stat_add_slot(g, kCtrLinks, slot, links);
      stat_add_slot(g, kCtrRechecks, slot, rechecks);
      stat_add_slot(g, kCtrPairs, slot, pairs);
    }
  }
};

// ---------------------------------------------------------------------------
// MarkCore (Algorithm 2).  A cell with at least minPts points is all core (its
// points are pairwise within eps: the diameter guard holds for every cell after
// splitting).  Otherwise each point starts from |g| and adds the points within
// eps in neighbour cells; it stops as soon as minPts is reached (early exit; the
// result is the same as counting everything).
// ---------------------------------------------------------------------------
// LEAF: the sub-cell (chunk-box) path is compiled in; see k_markcore_leaf.
template <int D, bool F32, bool LEAF>
struct MarkCoreVisitor {
  static constexpr bool kNearestFirst = true;
  DB_DEV bool keep_node(int, int) const { return true; }
  const Work* W;
  Flat F;
  int* order;        // [64] LDS: group-local cell of each flattened position
  int g, ps, pm;
  int cnt;           // lane t: count of point ps + t (|g| plus this wave's share)
  uint64_t pending;  // points of the batch still below minPts
  int smask, part;   // this wave tests every (smask + 1)-th candidate chunk, from part
  int chunk_no;
  int flushed;       // split waves: how much of cnt this lane has added to W->cnt so far
  double p[D];       // lane t: coordinates of point ps + t (float64 mode)
  float ap[D];       // lane t: cell-local float32 coordinates (filter mode)
  double ag[D];      // anchor of g (filter mode)
  float tin, tout;
  int lm;            // neighbour cells of at least lm points are taken by chunk boxes
  Counters ctr;

  // Split waves add their shares to the point's count as they go (one atomic per
  // pending point and chunk), so a point stops once the shares of all its waves
  // together reach the cap, not only when this wave's own share does.
  DB_DEV void publish() {
    if (!smask) return;
    const int lane = lane_id();
    const bool on = ((pending >> lane) & 1ull) && cnt > flushed;
    int total = 0;
    if (on) {
      total = atomicAdd(&W->cnt[ps + lane], cnt - flushed) + (cnt - flushed);
      flushed = cnt;
    }
    pending &= ~ballot(on && total >= W->count_cap);
  }

  // A large neighbour cell h in sub-cell order: the leaves of the paper's per-cell
  // quadtree are its aligned 64-point chunks, and above them the aligned groups of
  // 64 chunks that lie inside h (k_group_box).  A group or chunk whose box lies
  // wholly within eps of a point adds its share of h to that point's count without
  // tests, one farther than eps is skipped, and only the others are opened: a group
  // into its chunks, a chunk into point tests.
  //
  // One chunk for the lanes in `act`.
  DB_DEV void leaf_chunk(int ch, int hs, int he, const float (&off)[D], uint64_t act) {
    const int lane = lane_id();
    const int n = W->n;
    const int b0 = max(hs, ch * kWave), b1 = min(he, ch * kWave + kWave);
    bool test = false;
    if ((act >> lane) & 1ull) {
      if (box_maxdist<D>(p, W->chunkLo, W->chunkHi, W->chunkCap, ch) <= W->E2)
        cnt += b1 - b0;
      else
        test = box_sqdist<D>(p, p, W->chunkLo, W->chunkHi, W->chunkCap, ch) <= W->E2;
    }
    uint64_t tm = ballot(test);
    if (tm) {
      const int q = ch * kWave + lane;
      const bool valid = q >= b0 && q < b1;
      double xq[D];
      float aq[D];
#pragma unroll
      for (int d = 0; d < D; ++d) {
        xq[d] = 0.0;
        aq[d] = 0.0f;
      }
      if (valid) {
        if constexpr (F32) load_local<D>(W->X32, n, q, aq);
        else load_point<D>(W->X, n, q, xq);
      }
      while (tm) {
        const int t = __ffsll((long long)tm) - 1;
        tm &= tm - 1;
        bool hit;
        if constexpr (F32) {
          float at[D];
#pragma unroll
          for (int d = 0; d < D; ++d) at[d] = bcast(ap[d], t);
          hit = filtered_hit<D>(W, valid, at, aq, off, tin, tout, ps + t, q, ctr.rechecks,
                                W->E2);
        } else {
          double xp[D];
#pragma unroll
          for (int d = 0; d < D; ++d) xp[d] = bcast(p[d], t);
          hit = valid && sqdist<D>(xp, xq) <= W->E2;
        }
        const int add = __popcll(ballot(hit));
        if (lane == t) cnt += add;
      }
    }
  }

  // After a step of the walk through h: points at the cap stop, the split waves'
  // shares are published; true when every point of the wave is done.
  DB_DEV bool leaf_step_done() {
    pending &= ~ballot(cnt >= W->count_cap);
    publish();
    return !pending;
  }

  DB_DEV bool leaf_cell(int h, int hs, int he) {
    const int lane = lane_id();
    float off[D];
#pragma unroll
    for (int d = 0; d < D; ++d) off[d] = 0.0f;
    if constexpr (F32) anchor_offsets<D>(W->tree, ag, h, off);
    // One pass over h's chunks.  A group wholly inside h is one share of a split:
    // the wave that owns it tests its box and opens its chunks if it must (gact: the
    // lanes that take them); the other waves skip it.  Chunks outside such groups
    // are shares one by one.
    uint64_t gact = ~0ull;
    int gend = 0;  // end of the group being opened
    const int c_last = (he - 1) / kWave;
    for (int ch = hs / kWave; ch <= c_last;) {
      const bool whole = ch % kGroupChunks == 0 && ch * kWave >= hs &&
                         (ch + kGroupChunks) * kWave <= he;
      if (whole) {
        if ((chunk_no++ & smask) != part) {
          ch += kGroupChunks;
          continue;
        }
        bool open = false;
        if ((pending >> lane) & 1ull) {
          const int g = ch / kGroupChunks;
          if (box_maxdist<D>(p, W->groupLo, W->groupHi, W->groupCap, g) <= W->E2)
            cnt += kGroupPts;
          else
            open = box_sqdist<D>(p, p, W->groupLo, W->groupHi, W->groupCap, g) <= W->E2;
        }
        gact = ballot(open);
        gend = ch + kGroupChunks;
        if (leaf_step_done()) return true;
        if (!gact) {
          ch = gend;
          continue;
        }
      } else if (ch >= gend) {
        gact = ~0ull;
        if ((chunk_no++ & smask) != part) {
          ++ch;
          continue;
        }
      }
      leaf_chunk(ch, hs, he, off, pending & gact);
      if (leaf_step_done()) return true;
      ++ch;
    }
    return false;
  }

  DB_DEV bool group(int cb, uint64_t m, double dist) {
    if (g >= cb && g < cb + 64) m &= ~(1ull << (g - cb));
    if (!m) return false;
    const int n = W->n;
    const int lane = lane_id();
    // In low dimensions the group's cells are taken nearest first (by box distance
    // to g), so that the counts reach count_cap after as few chunks as possible;
    // in high dimensions the ranking costs more than it saves.
    const bool on = (m >> lane) & 1ull;
    int cs = 0, cn = 0;
    if (on) {
      cs = W->cellStart[cb + lane];
      cn = W->cellStart[cb + lane + 1] - cs;
    }
    int rank = lane;  // identity order when everything fits one chunk
    if (D <= 3 && wave_sum(cn) > kWave) {
      // masked cells by (distance, lane), then the others by lane
      const double dv = on ? dist : 0.0;
      int r = 0;
      for (uint64_t mm = m; mm; mm &= mm - 1) {
        const int l = __ffsll((long long)mm) - 1;
        const double dl = bcast(dv, l);
        r += (dl < dv || (dl == dv && l < lane)) ? 1 : 0;
      }
      rank = on ? r : __popcll(m) + __popcll(~m & lanemask_lt());
    }
    wave_sync();
    order[rank] = lane;
    wave_sync();
    const int src = order[lane];
    wave_sync();
    const int rcs = __shfl(cs, src, kWave), rcn = __shfl(cn, src, kWave);
    bool big = false;
    if constexpr (LEAF) {
      big = rcn >= lm;
      for (uint64_t bm = ballot(big); bm; bm &= bm - 1) {
        const int r = __ffsll((long long)bm) - 1;
        const int hs = bcast(rcs, r);
        if (leaf_cell(cb + bcast(src, r), hs, hs + bcast(rcn, r))) return true;
      }
    }
    const int tot = flatten_ranges(F, rcs, big ? 0 : rcn);
    for (int base = 0; base < tot; base += kWave) {
      if ((chunk_no++ & smask) != part) continue;
      const int k = base + lane;
      const bool valid = k < tot;
      int j = 0, q = 0;
      double xq[D];
      float aq[D], off[D];
#pragma unroll
      for (int d = 0; d < D; ++d) {
        xq[d] = 0.0;
        aq[d] = 0.0f;
        off[d] = 0.0f;
      }
      if (valid) {
        locate(F, k, j, q);
        if constexpr (F32) {
          load_local<D>(W->X32, n, q, aq);
          anchor_offsets<D>(W->tree, ag, cb + order[j], off);
        } else {
          load_point<D>(W->X, n, q, xq);
        }
      }
      uint64_t pend = pending;
      while (pend) {
        const int t = __ffsll((long long)pend) - 1;
        pend &= pend - 1;
        bool hit;
        if constexpr (F32) {
          float at[D];
#pragma unroll
          for (int d = 0; d < D; ++d) at[d] = bcast(ap[d], t);
          hit = filtered_hit<D>(W, valid, at, aq, off, tin, tout, ps + t, q, ctr.rechecks,
                                  W->E2);
        } else {
          double xp[D];
#pragma unroll
          for (int d = 0; d < D; ++d) xp[d] = bcast(p[d], t);
          hit = valid && sqdist<D>(xp, xq) <= W->E2;
        }
        const int add = __popcll(ballot(hit));
        if (lane == t) cnt += add;
        const int ct = bcast(cnt, t);
        if (ct >= W->count_cap) pending &= ~(1ull << t);
      }
      publish();
      if (!pending) return true;
    }
    return false;
  }
};

// Neighbour counts, capped at count_cap (the largest minPts run with this eps, so
// that one count serves every minPts).  A cell with at least count_cap points
// needs no test: all its points are pairwise within eps.
template <int D, bool F32, bool LEAF, class WS>
DB_DEV void markcore_body(const WS& ws) {
  ws.each_wave([&](const Work& W) {
    __shared__ int s_pref[kWavesPerBlock][kWave + 1];
    __shared__ int s_start[kWavesPerBlock][kWave];
    __shared__ uint64_t s_m[kWavesPerBlock][kTreeLevels + 2];
    __shared__ int s_cb[kWavesPerBlock][kTreeLevels + 2];
    __shared__ double s_dist[kWavesPerBlock][(kTreeLevels + 2) * 64];
    __shared__ int s_order[kWavesPerBlock][kWave];
    const int C = W.desc->n_cells;
    const int w = threadIdx.x / kWave, lane = lane_id();
    const int n = W.n;
    const int cap = W.count_cap;
    // Waves per cell: the candidate chunks of a cell's walk are dealt out to split
    // waves, which add their counts (cnt is zeroed by k_keys) as they go; a wave stops
    // with a point when its own share, or the sum added so far by all of them,
    // reaches the cap, so every count is exact or at least the cap.
    static_assert((kMarkSplit & (kMarkSplit - 1)) == 0, "split must be a power of two");
    const int sh = (D <= 3 && (long long)n >= (long long)kMarkSplitMean * C)
                       ? __builtin_ctz((unsigned)W.mark_split)
                       : 0;
    const int split = 1 << sh;
    Counters tot;
    const UnitRange R = xcd_units((long long)C << sh);
    for (long long u = R.first; u < R.end; u += R.step) {
      const int g = (int)(u >> sh);
      const int part = (int)(u & (split - 1));
      const int s = W.cellStart[g], e = W.cellStart[g + 1], m = e - s;
      if (m >= cap) {
        if (part == 0)
          for (int i = s + lane; i < e; i += kWave) W.cnt[i] = m;
        continue;
      }
      Query<D> q;
      q.E2 = W.E2;
      load_box<D>(W.tree, g, q);
      for (int ps = s; ps < e; ps += kWave) {
        MarkCoreVisitor<D, F32, LEAF> v;
        v.W = &W;
        v.F = Flat{s_pref[w], s_start[w]};
        v.order = s_order[w];
        v.g = g;
        v.ps = ps;
        v.pm = min(kWave, e - ps);
        v.cnt = m;
        v.pending = v.pm == kWave ? ~0ull : ((1ull << v.pm) - 1ull);
        v.smask = split - 1;
        v.part = part;
        v.chunk_no = 0;
        v.flushed = part == 0 ? 0 : m;  // (every wave's cnt starts at |g|; part 0 adds it)
        v.tin = W.desc->tin;
        v.tout = W.desc->tout;
#pragma unroll
        for (int d = 0; d < D; ++d) {
          v.p[d] = 0.0;
          v.ap[d] = 0.0f;
        }
        v.lm = LEAF ? leaf_min(W) : kIntMax;
        if (lane < v.pm) {
          if constexpr (F32) load_local<D>(W.X32, n, ps + lane, v.ap);
          if (!F32 || v.lm != kIntMax) load_point<D>(W.X, n, ps + lane, v.p);
        }
        if constexpr (F32) load_anchor<D>(W.tree, g, v.ag);
        walk_from_list<D>(W, C, g, q, v, WalkStack{s_m[w], s_cb[w], s_dist[w]});
        if (lane < v.pm) {
          if (split == 1) W.cnt[ps + lane] = v.cnt;
          else if (v.cnt > v.flushed) atomicAdd(&W.cnt[ps + lane], v.cnt - v.flushed);
        }
        tot.add(v.ctr);
      }
    }
    tot.wave_flush(W.desc);
  });
}

// Up to 3 dimensions with the sub-cell path; four waves per SIMD there (without the
// bound the float32 instantiation settles one register above that limit).
template <int D, bool F32, class WS>
__global__ __launch_bounds__(kBlock, D <= 3 ? 4 : 1) void k_markcore(WS ws) {
  markcore_body<D, F32, D <= 3>(ws);
}

// Above 3 dimensions, for grids with sub-cell order: a separate kernel, so that the
// usual one (cells of few points) keeps its register budget.
template <int D, bool F32, class WS>
__global__ __launch_bounds__(kBlock, 1) void k_markcore_leaf(WS ws) {
  markcore_body<D, F32, true>(ws);
}

// Core flags of one minPts from the counts (Algorithm 2's test), the number of
// core points and the smallest input index among them per cell, and the
// union-find initialisation.
template <class WS>
__global__ __launch_bounds__(kBlock) void k_core_from_count(WS ws) {
  ws.each_wave([&](const Work& W) {
    const int C = W.desc->n_cells;
    const int w = threadIdx.x / kWave, lane = lane_id();
    for (int g = blockIdx.x * kWavesPerBlock + w; g < C; g += gridDim.x * kWavesPerBlock) {
      const int s = W.cellStart[g], e = W.cellStart[g + 1];
      int cc = 0, mn = kIntMax;
      // 8 x 64 points per step, all loads issued before any is used: a large cell
      // costs a few load latencies instead of one per 64 points
      for (int i0 = s; i0 < e; i0 += 8 * kWave) {
        int c[8], pm[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int i = i0 + u * kWave + lane;
          c[u] = i < e ? W.cnt[i] : -1;
          pm[u] = i < e ? W.perm[i] : kIntMax;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int i = i0 + u * kWave + lane;
          const bool core = c[u] >= W.minPts;
          if (i < e) W.coreS[i] = core ? 1 : 0;
          if (core) {
            ++cc;
            mn = min(mn, pm[u]);
          }
        }
      }
      cc = wave_sum(cc);
      mn = wave_min(mn);
      if (lane == 0) {
        W.coreCount[g] = cc;
        W.cellMin[g] = mn;
        W.parent[g] = g;
        W.minIdx[g] = kIntMax;
      }
    }
  });
}

// The settings of one eps (up to kMultiMax, by decreasing minPts) from the one
// neighbour count: bit s of coreS is the core flag under minPts[s], and each
// setting gets its own per-cell core count, smallest core input index and root
// minimum.  The union-find starts at the identity unless `warm` (a further group
// of the same eps continues from the previous group's links).
constexpr int kMultiMax = 8;
struct MultiCore {
  int k, warm;
  int minPts[kMultiMax];
  int32_t* coreCount[kMultiMax];
  int32_t* cellMin[kMultiMax];
  int32_t* minIdx[kMultiMax];
};

// Per-cell starting values of k_core_multi (one thread per cell).
__global__ void k_core_multi_init(Work W, MultiCore M) {
  const int C = W.desc->n_cells;
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < C; g += gridDim.x * blockDim.x) {
#pragma unroll
    for (int t = 0; t < kMultiMax; ++t) {
      if (t >= M.k) break;
      M.coreCount[t][g] = 0;
      M.cellMin[t][g] = kIntMax;
      M.minIdx[t][g] = kIntMax;
    }
    if (!M.warm) W.parent[g] = g;
  }
}

// One thread per sorted position: each wave takes a run of kCoreRun consecutive
// 64-position chunks, so a large cell is spread over many waves instead of one.
// Per setting, the core count and smallest core input index of each cell are
// reduced over the wave's positions (kept across its chunks while the cell
// continues) and added to the cell with one atomic each.
constexpr int kCoreRun = 16;

__global__ __launch_bounds__(kBlock) void k_core_multi(Work W, MultiCore M) {
  const int n = W.n;
  const int lane = lane_id();
  const int nchunks = (n + kWave - 1) / kWave;
  const int nruns = (nchunks + kCoreRun - 1) / kCoreRun;
  for (int run = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; run < nruns;
       run += gridDim.x * kWavesPerBlock) {
    int cur = -1;  // cell of the running partials (wave-uniform)
    int sum[kMultiMax], mn[kMultiMax];
    auto flush = [&]() {
      if (cur < 0 || lane != 0) return;
#pragma unroll
      for (int t = 0; t < kMultiMax; ++t) {
        if (t >= M.k) break;
        if (sum[t] > 0) {
          atomicAdd(&M.coreCount[t][cur], sum[t]);
          atomicMin(&M.cellMin[t][cur], mn[t]);
        }
      }
    };
    const int ch_end = min(nchunks, (run + 1) * kCoreRun);
    for (int ch = run * kCoreRun; ch < ch_end; ++ch) {
      const int i = ch * kWave + lane;
      const bool valid = i < n;
      const int c = valid ? W.cellOf[i] : -1;
      const int cn = valid ? W.cnt[i] : -1;
      const int pm = valid ? W.perm[i] : kIntMax;
      uint32_t bits = 0;
#pragma unroll
      for (int t = 0; t < kMultiMax; ++t)
        bits |= (t < M.k && cn >= M.minPts[t]) ? (1u << t) : 0u;
      if (valid) {
        W.coreS[i] = (uint8_t)bits;
        W.pk[i] = ((uint64_t)c << 8) | bits;
      }
      // the cells of this chunk, in order (usually one or two)
      for (uint64_t todo = ballot(valid); todo;) {
        const int leader = __ffsll((long long)todo) - 1;
        const int cc = __shfl(c, leader, kWave);
        const bool mine = valid && c == cc;
        if (cc != cur) {
          flush();
          cur = cc;
#pragma unroll
          for (int t = 0; t < kMultiMax; ++t) {
            sum[t] = 0;
            mn[t] = kIntMax;
          }
        }
#pragma unroll
        for (int t = 0; t < kMultiMax; ++t) {
          if (t >= M.k) break;
          const bool core = mine && ((bits >> t) & 1u);
          sum[t] += wave_sum(core ? 1 : 0);
          mn[t] = min(mn[t], wave_min(core ? pm : kIntMax));
        }
        todo &= ~ballot(mine);
      }
    }
    flush();
  }
}

// Outputs of the settings of one eps in input order: position j of every output
// array is written by one thread (coalesced stores), which gathers its sorted
// position's cell and core bits (one word, through the inverse permutation) and
// then the setting's cell label (core points) or border label.
struct MultiOut {
  int k;
  uint8_t* core[kMultiMax];
  int32_t* label[kMultiMax];
  const int32_t* cellLabel[kMultiMax];
  const int32_t* blabel[kMultiMax];
};

__global__ void k_output_multi(Work W, MultiOut O) {
  const int n = W.n;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    int i = W.inv[j];
    if ((unsigned)i >= (unsigned)n) i = 0;  // only if the sort failed (its status says so)
    const uint64_t v = W.pk[i];
    const int c = (int)(v >> 8);
    const uint32_t bits = (uint32_t)(v & 255u);
#pragma unroll
    for (int t = 0; t < kMultiMax; ++t) {
      if (t >= O.k) break;
      const bool core = (bits >> t) & 1u;
      O.core[t][j] = core ? 1 : 0;
      O.label[t][j] = core ? O.cellLabel[t][c] : O.blabel[t][i];
    }
  }
}

// Number of core points of the last setting, for the statistics (not on the hot
// path: run when they are read).  One workgroup sums the per-cell core counts.
__global__ __launch_bounds__(kBlock) void k_core_total(Work W) {
  __shared__ unsigned long long s_sum[kWavesPerBlock];
  const int C = W.desc->n_cells;
  unsigned long long t = 0;
  for (int c = threadIdx.x; c < C; c += blockDim.x) t += (unsigned long long)W.coreCount[c];
  for (int o = 32; o > 0; o >>= 1) t += __shfl_down(t, o, kWave);
  if (lane_id() == 0) s_sum[threadIdx.x / kWave] = t;
  __syncthreads();
  for (int i = threadIdx.x; i < kCtrSlots; i += blockDim.x) {
    unsigned long long v = 0;
    if (i == 0)
      for (int k = 0; k < kWavesPerBlock; ++k) v += s_sum[k];
    W.desc->ctr[kCtrCore][i] = v;
  }
}


// ---------------------------------------------------------------------------
// ClusterCore (Algorithm 3).  A unit (a core cell, or a tree node whose core
// cells already form one component) is tested against each core neighbour cell h
// of lower index whose union-find root differs: pairs of core points are scanned
// until the first pair within eps, which links the two (BCP with early exit).
// Points farther than eps from the other side's box drop out first (the paper's
// filter), and 64 x 64 tiles whose chunk boxes are farther than eps apart are
// skipped whole.
// ---------------------------------------------------------------------------
// LEAF: the cell-by-cell and sub-cell paths are compiled in; see k_bcp_leaf.
template <int D, bool F32, bool LEAF>
struct BcpVisitor {
  static constexpr bool kNearestFirst = false;
  float tin, tout;
  const Work* W;
  Flat F;
  int ps, pe;      // sorted point range of the unit (its core points take part)
  int c0, nchk;    // first aligned chunk of the unit and number of chunks
  int hmax;        // candidate cells are those with index < hmax
  int ucell;       // a core cell of the unit; links are made from it
  bool one_cell;   // the unit is one cell (its anchor is uq.lo): float32 offsets need no loads
  int rg;          // a root of the unit's component (refreshed per group; stale is safe)
  Query<D> uq;     // box of the unit
  double* ub;      // [2 D][64] LDS: the unit's chunk boxes (lo, then hi), when it has <= 64
  bool ub_ready;
  int excl_level;  // node already covered by an earlier round (level, index), or -1
  int excl_idx;
  bool prune;      // node roots of the previous round are valid
  Counters ctr;

  DB_DEV void load_chunk(int c, double (&x)[D], float (&a)[D], int& cell, bool& v) const {
    const int i = (c0 + c) * kWave + lane_id();
    v = i >= ps && i < pe;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      x[d] = 0.0;
      a[d] = 0.0f;
    }
    cell = -1;
    if (v) {
      const uint8_t core = W->coreS[i];
      load_point<D>(W->X, W->n, i, x);
      if constexpr (F32) {
        load_local<D>(W->X32, W->n, i, a);
        if (!one_cell) cell = W->cellOf[i];
      }
      v = (core & W->core_mask) != 0;
    }
  }

  // A node is skipped when an earlier round already handled it, when it has no
  // core cell, or when all its core cells were in one component that the unit has
  // joined since (components only merge, so this stays true).
  DB_DEV bool keep_node(int level, int idx) const {
    if (level == excl_level && idx == excl_idx) return false;
    if (!prune) return true;
    const int r = W->nroot[level][idx];
    if (r == kNodeNoCore) return false;
    if (r < 0) return true;
    return uf_find(W->parent, r) != rg;
  }

  // One 64 x 64 tile: the wave's q points of cell h (one per lane) against the
  // unit's chunk cidx.  Unit points farther than eps from the box [blo, bhi], which
  // holds every valid q, drop out first.  Links the unit to h at the first pair
  // within eps and returns true.
  // Approximate DBSCAN takes a small box whole, as the paper's approximate range
  // count takes a quadtree cell of side at most eps rho / sqrt(d): when the box's
  // diameter is at most eps rho / 2 and a unit core point lies within eps of it,
  // that point is within eps (1 + rho / 2) of every valid q, so the unit and h are
  // linked without pair tests (the margin of rho / 2 keeps rounding far from R).
  // hoff: T = fl32(A_unit - A_h) when the unit is one cell (else unused).
  DB_DEV bool tile(int cidx, int h, const double (&xq)[D], const float (&aq)[D], bool valid,
                   int q, const double (&blo)[D], const double (&bhi)[D], const float (&hoff)[D]) {
    const int lane = lane_id();
    const int chunk = c0 + cidx;
    double xp[D];
    float ap[D];
    int pcell = -1;
    bool pv = false;
    load_chunk(cidx, xp, ap, pcell, pv);
    pv = pv && box_sqdist<D>(xp, xp, blo, bhi, 1, 0) <= W->E2;
    uint64_t pm = ballot(pv);
    if (pm && W->E2leaf > 0.0 && ballot(valid) && sqdist<D>(blo, bhi) <= W->E2leaf) {
      bool linked = false;
      if (lane == 0) linked = uf_link(W->parent, ucell, h);
      ctr.links += ballot(linked) ? 1ull : 0ull;
      return true;
    }
    int curcell = -1;
    float off[D];
#pragma unroll
    for (int d = 0; d < D; ++d) off[d] = hoff[d];
    while (pm) {
      const int t = __ffsll((long long)pm) - 1;
      pm &= pm - 1;
      bool hit;
      ctr.pairs += (unsigned long long)__popcll(ballot(valid));
      if constexpr (F32) {
        const int pc = one_cell ? -1 : bcast(pcell, t);
        if (pc != curcell) {
          curcell = pc;
          double apc[D];
          load_anchor<D>(W->tree, pc, apc);
          anchor_offsets<D>(W->tree, apc, h, off);
        }
        float at[D];
#pragma unroll
        for (int d = 0; d < D; ++d) at[d] = bcast(ap[d], t);
        hit = filtered_hit<D>(W, valid, at, aq, off, tin, tout, chunk * kWave + t, q,
                              ctr.rechecks, W->E2b);
      } else {
        double xt[D];
#pragma unroll
        for (int d = 0; d < D; ++d) xt[d] = bcast(xp[d], t);
        hit = valid && sqdist<D>(xt, xq) <= W->E2b;
      }
      if (ballot(hit)) {
        bool linked = false;
        if (lane == 0) linked = uf_link(W->parent, ucell, h);
        ctr.links += ballot(linked) ? 1ull : 0ull;
        return true;
      }
    }
    return false;
  }

  // Loads the q points of h held by sorted positions [qb, qb + 64) (lane = one
  // position); a q takes part when it lies in [hs, he), is core and lies within
  // eps of the unit's box.
  DB_DEV bool load_q(int qb, int hs, int he, double (&xq)[D], float (&aq)[D], int& q) const {
    q = qb + lane_id();
    bool valid = q >= hs && q < he;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      xq[d] = 0.0;
      aq[d] = 0.0f;
    }
    if (valid) {
      const uint8_t core = W->coreS[q];
      load_point<D>(W->X, W->n, q, xq);
      if constexpr (F32) load_local<D>(W->X32, W->n, q, aq);
      valid = (core & W->core_mask) != 0 && box_sqdist<D>(xq, xq, uq.lo, uq.hi, 1, 0) <= W->E2;
    }
    return valid;
  }

  // Sub-cell order: the points of large cells follow a Morton curve inside the
  // cell, so every aligned 64-point chunk covers a compact part of it, like a leaf
  // of the paper's per-cell quadtree.  Chunks of h farther than eps from the
  // unit's box are skipped unloaded, and each remaining q chunk is tested only
  // against the unit chunks within eps of the box of its taking-part points: far
  // corners of two large cells cost box tests, not tiles.  The unit's chunk boxes
  // sit in LDS when it has at most 64.
  // The unit's chunk boxes into LDS, once per unit (units of at most 64 chunks).
  DB_DEV void ensure_ub() {
    if (nchk > kWave || ub_ready) return;
    const int lane = lane_id();
    if (lane < nchk) {
#pragma unroll
      for (int k = 0; k < D; ++k) {
        ub[k * kWave + lane] = W->chunkLo[(size_t)k * W->chunkCap + c0 + lane];
        ub[(D + k) * kWave + lane] = W->chunkHi[(size_t)k * W->chunkCap + c0 + lane];
      }
    }
    wave_sync();
    ub_ready = true;
  }

  // Unit chunks pc0 .. pc0 + 63 whose box lies within eps of [blo, bhi] (one per lane).
  DB_DEV uint64_t unit_mask(int pc0, const double (&blo)[D], const double (&bhi)[D]) const {
    const int pcl = pc0 + lane_id();
    bool sv = false;
    if (pcl < nchk)
      sv = (nchk <= kWave ? box_sqdist<D>(blo, bhi, ub, ub + D * kWave, kWave, pcl)
                          : box_sqdist<D>(blo, bhi, W->chunkLo, W->chunkHi, W->chunkCap, c0 + pcl)) <=
           W->E2;
    return ballot(sv);
  }

  // T = fl32(A_unit - A_h) for a one-cell unit (the same arithmetic as anchor_offsets)
  DB_DEV void unit_offsets(const double (&ah)[D], float (&hoff)[D]) const {
#pragma unroll
    for (int d = 0; d < D; ++d) hoff[d] = F32 && one_cell ? (float)(uq.lo[d] - ah[d]) : 0.0f;
  }

  DB_DEV bool dense_leaves(int h, int hs, int he) {
    const int lane = lane_id();
    const int cap = W->chunkCap;
    ensure_ub();
    float hoff[D];
    {
      double ah[D];
#pragma unroll
      for (int d = 0; d < D; ++d) ah[d] = 0.0;
      if (F32 && one_cell) load_anchor<D>(W->tree, h, ah);
      unit_offsets(ah, hoff);
    }
    const int hc0 = hs / kWave, hc1 = (he - 1) / kWave;
    // windows of 64 chunks aligned to the groups of k_group_box: a group wholly inside
    // h whose box is farther than eps from the unit's box is skipped unloaded
    for (int hw = hc0 / kGroupChunks * kGroupChunks; hw <= hc1; hw += kGroupChunks) {
      const int g = hw / kGroupChunks;
      if (hw * kWave >= hs && (hw + kGroupChunks) * kWave <= he &&
          !(box_sqdist<D>(uq.lo, uq.hi, W->groupLo, W->groupHi, W->groupCap, g) <= W->E2))
        continue;
      const int hcl = hw + lane;
      double hd = hcl >= hc0 && hcl <= hc1
                      ? box_sqdist<D>(uq.lo, uq.hi, W->chunkLo, W->chunkHi, cap, hcl)
                      : __builtin_inf();
      for (uint64_t hm = ballot(hd <= W->E2); hm; hm &= hm - 1) {
        const int j = __ffsll((long long)hm) - 1;
        double xq[D];
        float aq[D];
        int q;
        const bool valid = load_q((hw + j) * kWave, hs, he, xq, aq, q);
        if (!ballot(valid)) continue;
        // the box of the q points that take part (core, within eps of the unit):
        // much tighter than the chunk's box, so far fewer unit chunks pass
        double qlo[D], qhi[D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
          qlo[k] = wave_min(valid ? xq[k] : __builtin_inf());
          qhi[k] = wave_max(valid ? xq[k] : -__builtin_inf());
        }
        for (int pc0 = 0; pc0 < nchk; pc0 += kWave)
          for (uint64_t sm = unit_mask(pc0, qlo, qhi); sm; sm &= sm - 1)
            if (tile(pc0 + __ffsll((long long)sm) - 1, h, xq, aq, valid, q, qlo, qhi, hoff))
              return true;
      }
    }
    return false;
  }

  // Dense groups: the live neighbour cells are taken one at a time; the q side is
  // a contiguous run of the cell's points and the cell's box stands in for the box
  // of each q chunk, so no chunk search or box reduction is needed.  Without
  // sub-cell order the points of a cell are in input order: every 64-point run
  // spreads over its whole cell, so the first tiles tried usually hold a pair
  // within eps when one exists, and chunk boxes would prune nothing.
  DB_DEV void dense_cells(int cb, uint64_t alive, int hr, int s0, int s1) {
    const int lane = lane_id();
    const int lm = leaf_min(*W);
    bool fresh = true;  // the roots were just taken by group()
    while (alive) {
      // Components merge while this wave works (other waves link concurrently):
      // roots are refreshed before each further test and cells already joined
      // drop out.
      if (!fresh) {
        const int ru = uf_find(W->parent, ucell);
        const bool on = (alive >> lane) & 1ull;
        if (on) hr = uf_find(W->parent, cb + lane);
        alive &= ballot(on && hr != ru);
        if (!alive) break;
      }
      fresh = false;
      const int c = __ffsll((long long)alive) - 1;
      const int h = cb + c;
      const int hs = bcast(s0, c), he = bcast(s1, c);
      bool linked_h = false;
      // Either side in sub-cell order: chunk boxes prune; both in input order:
      // every tile samples the whole of both cells.
      if (he - hs >= lm || pe - ps >= lm) {
        linked_h = dense_leaves(h, hs, he);
      } else {
        Query<D> hb;
        load_box<D>(W->tree, h, hb);
        float hoff[D];
        unit_offsets(hb.lo, hoff);
        for (int qb = hs; qb < he && !linked_h; qb += kWave) {
          double xq[D];
          float aq[D];
          int q;
          const bool valid = load_q(qb, hs, he, xq, aq, q);
          if (!ballot(valid)) continue;
          for (int cidx = 0; cidx < nchk && !linked_h; ++cidx)
            linked_h = tile(cidx, h, xq, aq, valid, q, hb.lo, hb.hi, hoff);
        }
      }
      if (linked_h) {
        const int rc = bcast(hr, c);
        alive &= ~ballot(hr == rc);  // that whole component has joined
      }
      alive &= ~(1ull << c);
    }
  }

  DB_DEV bool group(int cb, uint64_t m, double) {
    const int lane = lane_id();
    const int n = W->n;
    const int h = cb + lane;
    const bool inm = ((m >> lane) & 1ull) && h < hmax;
    // every per-cell load of the group at once
    int cc = 0, s0 = 0, s1 = 0, par = -1;
    if (inm) {
      cc = W->coreCount[h];
      s0 = W->cellStart[h];
      s1 = W->cellStart[h + 1];
      par = W->parent[h];
    }
    rg = uf_find(W->parent, ucell);
    bool on = inm && cc > 0;
    int hr = -1;
    if (on) {
      hr = par == h ? h : uf_find(W->parent, par);
      on = hr != rg;
    }
    uint64_t alive = ballot(on);
    if (!alive) return false;
    ctr.bcp += (unsigned long long)__popcll(alive);
    // Cell by cell: dense groups up to 3 dimensions; above, where cells mostly hold
    // few points, only groups with a cell in sub-cell order.
    if constexpr (LEAF) {
      bool dense;
      if constexpr (D <= 3) {
        const int tot_pts = wave_sum(on ? s1 - s0 : 0);
        dense = tot_pts >= W->dense_group * __popcll(alive);
      } else {
        dense = ballot(on && s1 - s0 >= leaf_min(*W)) != 0;
      }
      if (dense) {
        dense_cells(cb, alive, hr, on ? s0 : 0, on ? s1 : 0);
        return false;
      }
    }
    const int tot = flatten_ranges(F, on ? s0 : 0, on ? s1 - s0 : 0);
    for (int base = 0; base < tot && alive; base += kWave) {
      const int k = base + lane;
      bool valid = k < tot;
      int j = 0, q = 0;
      double xq[D];
      float aq[D], qoff[D];
#pragma unroll
      for (int d = 0; d < D; ++d) {
        xq[d] = 0.0;
        aq[d] = 0.0f;
        qoff[d] = 0.0f;
      }
      if (valid) {
        locate(F, k, j, q);
        const uint8_t core = W->coreS[q];
        load_point<D>(W->X, n, q, xq);
        if constexpr (F32) {
          load_local<D>(W->X32, n, q, aq);
          // a one-cell unit: T of this lane's cell, once for every unit chunk
          if (one_cell) anchor_offsets<D>(W->tree, uq.lo, cb + j, qoff);
        }
        // points of h farther than eps from the unit's box drop out
        valid = (core & W->core_mask) != 0 && ((alive >> j) & 1ull) &&
                box_sqdist<D>(xq, xq, uq.lo, uq.hi, 1, 0) <= W->E2;
      }
      if (!ballot(valid)) continue;
      double qlo[D], qhi[D];
#pragma unroll
      for (int d = 0; d < D; ++d) {
        qlo[d] = wave_min(valid ? xq[d] : __builtin_inf());
        qhi[d] = wave_max(valid ? xq[d] : -__builtin_inf());
      }
      bool stop = false;
      // 64 x 64 tiles: unit chunks whose box is farther than eps from this chunk's
      // box are skipped whole (the lanes test 64 chunk boxes at once)
      for (int pc0 = 0; pc0 < nchk && !stop; pc0 += kWave) {
        const int pcl = pc0 + lane;
        bool sv = false;
        if (pcl < nchk)
          sv = box_sqdist<D>(qlo, qhi, W->chunkLo, W->chunkHi, W->chunkCap, c0 + pcl) <= W->E2;
        uint64_t sm = ballot(sv);
        while (sm && !stop) {
          const int b = __ffsll((long long)sm) - 1;
          sm &= sm - 1;
          const int cidx = pc0 + b;
          const int chunk = c0 + cidx;
          double xp[D];
          float ap[D];
          int pcell = -1;
          bool pv = false;
          load_chunk(cidx, xp, ap, pcell, pv);
          // points of the unit farther than eps from this chunk's box drop out
          pv = pv && box_sqdist<D>(xp, xp, qlo, qhi, 1, 0) <= W->E2;
          uint64_t pm = ballot(pv);
          int curcell = -1;
          float off[D];
#pragma unroll
          for (int d = 0; d < D; ++d) off[d] = qoff[d];
          while (pm) {
            const int t = __ffsll((long long)pm) - 1;
            pm &= pm - 1;
            bool hit;
            ctr.pairs += (unsigned long long)__popcll(ballot(valid));
            if constexpr (F32) {
              const int pc = one_cell ? -1 : bcast(pcell, t);
              if (pc != curcell) {
                curcell = pc;
                double apc[D];
                load_anchor<D>(W->tree, pc, apc);
                anchor_offsets<D>(W->tree, apc, cb + j, off);
              }
              float at[D];
#pragma unroll
              for (int d = 0; d < D; ++d) at[d] = bcast(ap[d], t);
              hit = filtered_hit<D>(W, valid, at, aq, off, tin, tout, chunk * kWave + t, q,
                                    ctr.rechecks, W->E2b);
            } else {
              double xt[D];
#pragma unroll
              for (int d = 0; d < D; ++d) xt[d] = bcast(xp[d], t);
              hit = valid && sqdist<D>(xt, xq) <= W->E2b;
            }
            if (!ballot(hit)) continue;
            uint64_t cells = wave_or(hit ? (1ull << j) : 0ull);
            while (cells) {
              const int c = __ffsll((long long)cells) - 1;
              cells &= cells - 1;
              if (!((alive >> c) & 1ull)) continue;
              const int rc = bcast(hr, c);
              bool linked = false;
              if (lane == 0) linked = uf_link(W->parent, ucell, cb + c);
              ctr.links += ballot(linked) ? 1ull : 0ull;
              alive &= ~ballot(hr == rc);  // that whole component has joined
            }
            valid = valid && ((alive >> j) & 1ull);
            if (!ballot(valid)) {
              stop = true;
              break;
            }
          }
        }
      }
    }
    return false;
  }
};

// Round r (0 .. top) connects cells whose lowest common tree ancestor is at level
// r + 1: each unit walks its level-(r+1) ancestor, leaving out its level-r
// ancestor handled by earlier rounds (the paper's bucketing: early, local rounds
// link most cells, so that later rounds skip whole subtrees already in one
// component).  From round 1 on, a node whose core cells all lie in one component
// acts as a single unit (its first cell's wave runs it), instead of each of its
// cells repeating the same links.
// round = -1: a single pass in which every core cell walks the whole tree.
// WARM: the union-find starts from the previous setting's (see Work::warm); a
// separate instantiation, so that the cold kernel keeps its register budget.
template <int D, bool F32, bool WARM, bool LEAF, class WS>
DB_DEV void bcp_body(const WS& ws, int round) {
  ws.each_wave([&](const Work& W) {
    __shared__ int s_pref[kWavesPerBlock][kWave + 1];
    __shared__ int s_start[kWavesPerBlock][kWave];
    __shared__ uint64_t s_m[kWavesPerBlock][kTreeLevels + 2];
    __shared__ int s_cb[kWavesPerBlock][kTreeLevels + 2];
    __shared__ double s_ub[kWavesPerBlock][LEAF ? 2 * D * kWave : 1];
    const int C = W.desc->n_cells;
    int cnt[kTreeLevels + 2];
    level_counts(C, cnt);
    const int top = top_level(cnt);
    if (round > top) return;
    const int w = threadIdx.x / kWave;
    // Up to W.bcp_split waves share one unit: its points are cut into that many
    // segments of at least seg_min points, and each wave tests its segment
    // against every neighbour, so a large cell no longer sets the kernel's length
    // alone.  Links are made from the same cell, and a segment that finds its
    // neighbour already joined (by another segment) skips it.
    const int split = W.bcp_split;
    const int seg_min = max(kBcpSegment, (int)((long long)kSegMean * W.n / max(C, 1)));
    Counters tot;
    const UnitRange R = xcd_units((long long)C * split);
    for (long long u = R.first; u < R.end; u += R.step) {
      const int g = (int)(u / split);
      const int part = (int)(u % split);
      const int umax = round < 0 ? 0 : min(round, W.unit_max_level);
      int ulevel = -1;
      if (W.coreCount[g] > 0 && (umax == 0 || W.nroot[1][g >> 6] < 0)) ulevel = 0;
      for (int l = 1; l <= umax && ulevel < 0; ++l) {
        const int idx = g >> (6 * l);
        if ((idx << (6 * l)) != g) break;
        if (W.nroot[l][idx] >= 0 && (l == umax || W.nroot[l + 1][g >> (6 * (l + 1))] < 0)) ulevel = l;
      }
      if (ulevel < 0) continue;
      // Warm start with the previous setting's core counts: a link the union-find lacks
      // needs a pair within eps with a point that was not core before (pairs of earlier
      // core points were all linked), so only cells that gained core points act, and
      // they test every neighbour cell, not only those of lower index.
      const bool gained_only = WARM && W.prev_core_count != nullptr;
      if (gained_only && W.coreCount[g] <= W.prev_core_count[g]) continue;
      BcpVisitor<D, F32, LEAF> v;
      v.W = &W;
      v.F = Flat{s_pref[w], s_start[w]};
      v.ub = s_ub[w];
      v.ub_ready = false;
      // The walk, the point filters and the chunk masks work at eps: every pair within
      // eps is met.  Only the pair test works at E2b (eps (1 + rho) when approximate),
      // so an approximate run meets the same candidates and stops sooner.
      v.uq.E2 = W.E2;
      v.tin = W.desc->tinb;
      v.tout = W.desc->toutb;
      v.one_cell = ulevel == 0;
      if (ulevel == 0) {
        v.ps = W.cellStart[g];
        v.pe = W.cellStart[g + 1];
        v.hmax = gained_only ? C : g;
        v.ucell = g;
        load_box<D>(W.tree, g, v.uq);
      } else {
        const int idx = g >> (6 * ulevel);
        const int first = idx << (6 * ulevel);
        const int last = min(C, (idx + 1) << (6 * ulevel)) - 1;
        v.ps = W.cellStart[first];
        v.pe = W.cellStart[last + 1];
        v.hmax = first;
        v.ucell = W.nroot[ulevel][idx];
#pragma unroll
        for (int d = 0; d < D; ++d) {
          v.uq.lo[d] = W.tree.lo[ulevel][(size_t)d * W.tree.cap[ulevel] + idx];
          v.uq.hi[d] = W.tree.hi[ulevel][(size_t)d * W.tree.cap[ulevel] + idx];
        }
      }
      {
        const int m = v.pe - v.ps;
        const int nseg = max(1, min(split, m / seg_min));
        if (part >= nseg) continue;
        const int len = (m + nseg - 1) / nseg;
        v.ps += part * len;
        v.pe = min(v.pe, v.ps + len);
      }
      v.c0 = v.ps >> 6;
      v.nchk = ((v.pe - 1) >> 6) - v.c0 + 1;
      // a warm start prunes by the node roots taken before the launch from the start:
      // the cell's parent is its root after most links (a full find here made the
      // compiler spill the kernel's registers; the walk's groups refresh the root)
      v.rg = WARM ? W.parent[v.ucell] : v.ucell;
      v.excl_level = round >= 1 ? round : -1;
      v.excl_idx = round >= 1 ? (g >> (6 * round)) : 0;
      // (a warm start with known previous counts takes no node roots: see stage_cluster)
      v.prune = (WARM && !gained_only) || round >= 1;
      const int anc_level = round < 0 ? top + 1 : round + 1;
      const int anc = (round < 0 || round == top) ? 0 : (g >> (6 * anc_level));
      if (round < 0 && ulevel == 0)
        walk_from_list<D>(W, C, g, v.uq, v, WalkStack{s_m[w], s_cb[w], nullptr});
      else
        walk_subtree<D>(W.tree, C, anc_level, anc, v.uq, v, WalkStack{s_m[w], s_cb[w], nullptr});
      tot.add(v.ctr);
    }
    tot.wave_flush(W.desc);
  });
}

// Up to 3 dimensions with the cell-by-cell and sub-cell paths.  Four waves per SIMD
// where that fits without spilling (float64, d <= 4); the other instantiations need
// more registers and would spill to scratch.
template <int D, bool F32, bool WARM, class WS>
__global__ __launch_bounds__(kBlock, (F32 || D > 4) ? 1 : 4) void k_bcp(WS ws, int round) {
  bcp_body<D, F32, WARM, D <= 3>(ws, round);
}

// Above 3 dimensions, for grids with sub-cell order: a separate kernel, so that the
// usual one (cells of few points) keeps its register budget.
template <int D, bool F32, bool WARM, class WS>
__global__ __launch_bounds__(kBlock, 1) void k_bcp_leaf(WS ws, int round) {
  bcp_body<D, F32, WARM, true>(ws, round);
}

// Node roots for pruning: per node, the common root of its core cells, -1 when
// they are in several components, kNodeNoCore when it has no core cell.
template <class WS>
__global__ __launch_bounds__(kBlock) void k_node_roots(WS ws, int level) {
  ws.each_wave([&](const Work& W) {
    const int C = W.desc->n_cells;
    int cnt[kTreeLevels + 2];
    level_counts(C, cnt);
    const int lane = lane_id();
    for (int j = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; j < cnt[level];
         j += gridDim.x * kWavesPerBlock) {
      const int ch = j * 64 + lane;
      int v = kNodeNoCore;
      if (ch < cnt[level - 1]) {
        if (level == 1) v = W.coreCount[ch] > 0 ? uf_find(W.parent, ch) : kNodeNoCore;
        else v = W.nroot[level - 1][ch];
      }
      const bool mixed = ballot(v == -1) != 0;
      const int hi = wave_max(v);
      const int lo = wave_min(v == kNodeNoCore ? kIntMax : v);
      int r;
      if (mixed) r = -1;
      else if (hi == kNodeNoCore) r = kNodeNoCore;
      else r = (lo == hi) ? hi : -1;
      if (lane == 0) W.nroot[level][j] = r;
    }
  });
}

// ---------------------------------------------------------------------------
// Canonical ids: the cluster id is the smallest input index of a core point in
// the component.  Each wave takes 64 cells, reduces the minimum per distinct root
// among them and issues one atomicMin per root.
// ---------------------------------------------------------------------------
template <class WS>
__global__ __launch_bounds__(kBlock) void k_relabel_min(WS ws) {
  ws.each_wave([&](const Work& W) {
    const int C = W.desc->n_cells;
    const int lane = lane_id();
    const int nchunks = (C + kWave - 1) / kWave;
    for (int ch = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; ch < nchunks;
         ch += gridDim.x * kWavesPerBlock) {
      const int c = ch * kWave + lane;
      int root = -1, mn = kIntMax;
      if (c < C && W.coreCount[c] > 0) {
        root = uf_find(W.parent, c);
        mn = W.cellMin[c];
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
  });
}

template <class WS>
__global__ void k_cell_label(WS ws) {
  ws.each_wave([&](const Work& W) {
    const int C = W.desc->n_cells;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < C; c += gridDim.x * blockDim.x) {
      W.cellLabel[c] = W.coreCount[c] > 0 ? W.minIdx[uf_find(W.parent, c)] : -1;
    }
  });
}

// ---------------------------------------------------------------------------
// ClusterBorder (Algorithm 4), reduced to the smallest id: a non-core point takes
// the smallest cluster id among core points within eps.  All core points of one
// cell share one id, so a neighbour cell whose id is not below the current best
// is skipped without distance tests.
// ---------------------------------------------------------------------------
template <int D, bool F32>
struct BorderVisitor {
  static constexpr bool kNearestFirst = false;
  // Only core points can give a label: with the node roots of this setting taken
  // (core_nodes), a node without a core cell is not entered.
  DB_DEV bool keep_node(int level, int idx) const {
    return !core_nodes || W->nroot[level][idx] != kNodeNoCore;
  }
  bool core_nodes;
  const Work* W;
  Flat F;
  int g, pm;
  int best;          // lane t: best id so far for batch point t
  int pidx;          // lane t: sorted position of batch point t
  double p[D];       // lane t: coordinates of batch point t (float64 mode)
  float ap[D];       // lane t: cell-local float32 coordinates (filter mode)
  double ag[D];      // anchor of g (filter mode)
  float tin, tout;
  Counters ctr;

  DB_DEV bool group(int cb, uint64_t m, double) {
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
      float aq[D], off[D];
#pragma unroll
      for (int d = 0; d < D; ++d) {
        xq[d] = 0.0;
        aq[d] = 0.0f;
        off[d] = 0.0f;
      }
      if (valid) {
        locate(F, k, j, q);
        valid = (W->coreS[q] & W->core_mask) != 0;
      }
      if (valid) {
        lq = W->cellLabel[cb + j];
        if constexpr (F32) {
          load_local<D>(W->X32, n, q, aq);
          anchor_offsets<D>(W->tree, ag, cb + j, off);
        } else {
          load_point<D>(W->X, n, q, xq);
        }
      }
      for (int t = 0; t < pm; ++t) {
        const int bt = bcast(best, t);
        const bool cand = valid && lq < bt;
        if (!ballot(cand)) continue;
        bool hit;
        if constexpr (F32) {
          float at[D];
#pragma unroll
          for (int d = 0; d < D; ++d) at[d] = bcast(ap[d], t);
          hit = filtered_hit<D>(W, cand, at, aq, off, tin, tout, bcast(pidx, t), q, ctr.rechecks,
                              W->E2);
        } else {
          double xp[D];
#pragma unroll
          for (int d = 0; d < D; ++d) xp[d] = bcast(p[d], t);
          hit = cand && sqdist<D>(xp, xq) <= W->E2;
        }
        const int mn = wave_min(hit ? lq : kIntMax);
        if (lane == t && mn < best) best = mn;
      }
    }
    return false;
  }
};

template <int D, bool F32, class WS>
__global__ __launch_bounds__(kBlock) void k_border(WS ws, int core_nodes) {
  ws.each_wave([&](const Work& W) {
    __shared__ int s_pref[kWavesPerBlock][kWave + 1];
    __shared__ int s_start[kWavesPerBlock][kWave];
    __shared__ uint64_t s_m[kWavesPerBlock][kTreeLevels + 2];
    __shared__ int s_cb[kWavesPerBlock][kTreeLevels + 2];
    __shared__ int s_pos[kWavesPerBlock][kWave];
    const int C = W.desc->n_cells;
    const int w = threadIdx.x / kWave, lane = lane_id();
    const int n = W.n;
    Counters tot;
    const UnitRange R = xcd_units(C);
    for (long long u = R.first; u < R.end; u += R.step) {
      const int g = (int)u;
      const int s = W.cellStart[g], e = W.cellStart[g + 1];
      if (W.coreCount[g] == e - s) continue;
      Query<D> q;
      q.E2 = W.E2;
      load_box<D>(W.tree, g, q);
      const int own = W.coreCount[g] > 0 ? W.cellLabel[g] : kIntMax;
      int i = s;
      while (i < e) {
        // compact the next (up to 64) non-core positions of g that have neighbours
        // outside g into s_pos.  A non-core point's count is exact (below every cap)
        // and includes the |g| points of its own cell, all within eps of it; a count
        // of |g| means no neighbour elsewhere, so its label is g's cluster or noise.
        int taken = 0;
        while (i < e && taken < kWave) {
          const int k = i + lane;
          bool nc = k < e && (W.coreS[k] & W.core_mask) == 0;
          if (nc && W.cnt[k] == e - s) {
            W.blabel[k] = own == kIntMax ? -1 : own;
            nc = false;
          }
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
        BorderVisitor<D, F32> v;
        v.core_nodes = core_nodes != 0;
        v.W = &W;
        v.F = Flat{s_pref[w], s_start[w]};
        v.g = g;
        v.pm = taken;
        v.best = own;
        v.pidx = pos;
        v.tin = W.desc->tin;
        v.tout = W.desc->tout;
#pragma unroll
        for (int d = 0; d < D; ++d) {
          v.p[d] = 0.0;
          v.ap[d] = 0.0f;
        }
        if (lane < taken) {
          if constexpr (F32) load_local<D>(W.X32, n, pos, v.ap);
          else load_point<D>(W.X, n, pos, v.p);
        }
        if constexpr (F32) load_anchor<D>(W.tree, g, v.ag);
        walk_from_list<D>(W, C, g, q, v, WalkStack{s_m[w], s_cb[w], nullptr});
        if (lane < taken) W.blabel[pos] = v.best == kIntMax ? -1 : v.best;
        tot.add(v.ctr);
      }
    }
    tot.wave_flush(W.desc);
  });
}

// Results back to input order.
template <class WS>
__global__ void k_scatter(WS ws) {
  ws.each_wave([&](const Work& W) {
    const int n = W.n;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
      const int src = W.perm[i];
      const uint8_t c = (W.coreS[i] & W.core_mask) ? 1 : 0;
      W.core_out[src] = c;
      W.label_out[src] = c ? W.cellLabel[W.cellOf[i]] : W.blabel[i];
    }
  });
}

}  // namespace db
