// Host side of the C ABI declared in include/dbscan.h: context, scratch layout,
// the launch sequence of one exact DBSCAN (paper, Algorithm 1), and batches of
// clouds and settings captured into one HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <utility>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/dbscan.h"
#include "cluster.hpp"
#include "membership.hpp"
#include "sparse.hpp"
#include "box.hpp"

using namespace db;

namespace {

// Effective tuning options of one call (after automatic choices and the tuned table).
struct Resolved {
  int rounds;      // 0: one ClusterCore pass, 1: rounds over the tree levels
  int unit_level;  // largest tree level acting as one unit in rounds
  int split;       // most waves per ClusterCore unit
  int fine;        // sub-cell Morton bits per dimension
  int sub;         // cells of at least this many points get sub-cell order (k_subsort); 0: none
  int mark_split;  // MarkCore waves per cell (d <= 3, grids of kMarkSplitMean+ points per cell)
  int dense;       // ClusterCore takes a group cell by cell from this many points per live cell
};

// One tuned choice: instances of dimension d, mode and n in [2^lg, 2^(lg+1)).
struct TunedEntry {
  int d, mode, lg;
  Resolved r;
  float ms;
};

}  // namespace

struct dbscan_ctx {
  int device = 0;
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  GridDesc* desc = nullptr;  // lives at the start of scratch, survives growth
  size_t desc_bytes = 0;
  int64_t last_n = 0;
  // the last dbscan() call, for dbscan_membership()
  bool last_valid = false;
  int last_d = 0;
  Work last_work;
  // the last setting enqueued (its per-cell core counts give n_core in the stats)
  bool stats_valid = false;
  Work stats_work;
  // tuning options
  int bcp_rounds = -1;  // -1: automatic (one pass for d <= 3, rounds above)
  int unit_level = -1;  // -1: automatic (1)
  int fine_bits = -1;   // -1: automatic (0)
  int force_recheck = 0;
  int batch_graph = 1;
  int bcp_split = -1;   // -1: automatic (1)
  int filter_max_d = -1;  // -1: automatic (3)
  int subcell_min = -1;   // -1: automatic (sub_auto), 0: never
  int sparse = -1;        // -1: automatic (never: slower on every workload measured),
                          // 0: never, 1: always
  int group_clouds = -1;  // -1: automatic (groups of at least two), 0: never, 1: always
  int mark_split = -1;    // -1: automatic (kMarkSplit)
  int dense_group = -1;   // -1: automatic (kDenseGroup)
  int cells = 0;          // 0: grid cells; 1: the box method in 2 dimensions
  // grouped batches: the scratch offset of the group area (0: none laid out), the
  // layout its descriptors were set up for, and the epoch base for the next layout
  size_t group_area_off = 0;
  std::vector<unsigned char> group_key;
  uint32_t group_seed = 0;
  std::vector<Work> group_table_host;
  // autotuner: choices per (d, mode, size class), used where an option is automatic
  std::vector<TunedEntry> tuned;
  uint32_t tune_gen = 0;
  // profiling: one event per phase boundary of the last call, in order, with the
  // boundary's index (a pool reused from call to call)
  bool profile = false;
  bool events_recorded = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_mark;
  bool ev_error = false;
  // captured batch
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph = nullptr;
  std::vector<unsigned char> graph_key;
};

// The box method's cells: asked for, and only in 2 dimensions.
bool box_cells(const dbscan_ctx* ctx, int d) { return ctx->cells == 1 && d == 2; }

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Bump layout of the per-call arrays inside the scratch block.  The same function
// sizes the allocation (base = nullptr) and carves the pointers.
struct Carver {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(int64_t count) {
    T* p = reinterpret_cast<T*>(base + off);
    off = align_up(off + sizeof(T) * (size_t)(count > 0 ? count : 1));
    return p;
  }
};

// slots: settings whose per-setting arrays coexist (several settings of one eps,
// computed together); 1 for a single setting.
// keep_keys: a copy of the sorted keys for grids derived from a finer one.
size_t layout(char* base, int64_t n, int d, Work* W, int slots = 1, bool keep_keys = false) {
  Work tmp;
  Work& w = W ? *W : tmp;
  Carver c{base};
  const int64_t tiles = ceil_div(n, kTile);
  w.bbox_part = c.take<double>((int64_t)kBBoxBlocks * 2 * kMaxD);
  w.bbox_flag = c.take<uint32_t>(kBBoxBlocks);
  w.ghist = c.take<uint32_t>(8 * 256);
  w.tilectr = c.take<uint32_t>(16);
  w.lbstate = c.take<uint64_t>(tiles * 256);
  w.keyA = c.take<uint64_t>(n);
  w.keyB = c.take<uint64_t>(n);
  w.idxA = c.take<uint32_t>(n);
  w.idxB = c.take<uint32_t>(n);
  w.X = c.take<double>(n * d);
  w.X32 = c.take<float>(n * d);
  w.chunkCap = (int)ceil_div(n, 64);
  w.chunkLo = c.take<double>((int64_t)w.chunkCap * d);
  w.chunkHi = c.take<double>((int64_t)w.chunkCap * d);
  w.runBox = c.take<double>((int64_t)w.chunkCap * d * 4);
  // the boxes of the groups of 64 chunks live in the run boxes' room, which is free
  // once the cell boxes are built (see k_group_box)
  w.groupCap = (int)ceil_div(w.chunkCap, kGroupChunks);
  w.groupLo = w.runBox;
  w.groupHi = w.runBox + (size_t)w.groupCap * d;
  w.perm = c.take<int32_t>(n);
  w.cellOf = c.take<int32_t>(n);
  w.cellStart = c.take<int32_t>(n + 1);
  w.cellOf2 = c.take<int32_t>(n);
  w.cellStart2 = c.take<int32_t>(n + 1);
  w.unsafe = c.take<uint8_t>(n);
  w.sublist = c.take<int32_t>(n / 2 + 1);
  int64_t cap = n;
  for (int l = 0; l <= kTreeLevels; ++l) {
    if (l > 0) cap = ceil_div(cap, 64);
    w.tree.cap[l] = (int)cap;
    w.tree.lo[l] = c.take<double>(cap * d);
    w.tree.hi[l] = c.take<double>(cap * d);
    w.tree.flo[l] = c.take<float>(cap * d);
    w.tree.fhi[l] = c.take<float>(cap * d);
    w.nroot[l] = l > 0 ? c.take<int32_t>(cap) : nullptr;
  }
  w.nlist = c.take<int32_t>((int64_t)w.tree.cap[1] * 64);
  w.nlen = c.take<int32_t>(w.tree.cap[1]);
  w.coreS = c.take<uint8_t>(n);
  w.cnt = c.take<int32_t>(n);
  w.parent = c.take<int32_t>(n);
  const int64_t ns = n * (int64_t)std::max(1, slots);
  w.coreCount = c.take<int32_t>(ns);
  w.minIdx = c.take<int32_t>(ns);
  w.cellLabel = c.take<int32_t>(ns);
  w.cellMin = c.take<int32_t>(ns);
  w.blabel = c.take<int32_t>(ns);
  w.inv = slots > 1 ? c.take<int32_t>(n) : nullptr;
  w.pk = slots > 1 ? c.take<uint64_t>(n) : nullptr;
  w.skey = keep_keys ? c.take<uint64_t>(n) : nullptr;
  return c.off;
}

void drop_graph(dbscan_ctx* ctx) {
  if (ctx->graph) (void)hipGraphExecDestroy(ctx->graph);
  ctx->graph = nullptr;
  ctx->graph_key.clear();
}

int grow(dbscan_ctx* ctx, int64_t n, int d, int slots = 1, bool keep_keys = false,
         size_t extra = 0) {
  const size_t need = ctx->desc_bytes + layout(nullptr, n, d, nullptr, slots, keep_keys) + extra;
  if (need <= ctx->scratch_bytes) return DBSCAN_OK;
  if (hipSetDevice(ctx->device) != hipSuccess) return DBSCAN_EHIP;
  if (hipDeviceSynchronize() != hipSuccess) return DBSCAN_EHIP;
  void* p = nullptr;
  if (hipMalloc(&p, need) != hipSuccess) return DBSCAN_ENOMEM;
  // keep the descriptor (and its epoch counter) across growth
  if (ctx->scratch) {
    if (hipMemcpy(p, ctx->scratch, ctx->desc_bytes, hipMemcpyDeviceToDevice) != hipSuccess) {
      (void)hipFree(p);
      return DBSCAN_EHIP;
    }
    (void)hipFree(ctx->scratch);
  }
  drop_graph(ctx);  // a captured batch refers to the old scratch
  ctx->group_area_off = 0;
  ctx->group_key.clear();
  ctx->last_valid = false;
  ctx->stats_valid = false;
  ctx->scratch = p;
  ctx->scratch_bytes = need;
  ctx->desc = reinterpret_cast<GridDesc*>(p);
  return DBSCAN_OK;
}

unsigned grid_for(int64_t items, int per_block, unsigned cap) {
  int64_t b = ceil_div(items, per_block);
  if (b < 1) b = 1;
  return (unsigned)(b > cap ? cap : b);
}

const char* const kPhaseNames[DBSCAN_NUM_PHASES] = {
    "bbox", "keys", "radix_sort", "cells", "cell_boxes", "tree", "markcore", "core_flags",
    "cluster_core", "relabel", "border", "scatter", "cluster_core_warm"};
// ClusterCore of a warm-started setting is timed as a phase of its own.
constexpr int kPhaseClusterWarm = 12;

// Phase boundaries: mark(i) ends phase i - 1 (and starts phase i).  With profiling
// on, each boundary records an event; the time between two consecutive events is
// charged to the phase the later one ends, so a batch, which repeats phases (the
// setting stages once per setting), sums every occurrence.
struct Marks {
  dbscan_ctx* ctx;  // null when profiling is off
  hipStream_t s;
  void operator()(int i) const {
    if (!ctx) return;
    const size_t k = ctx->ev_mark.size();
    if (k == ctx->ev_pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) {
        ctx->ev_error = true;
        return;
      }
      ctx->ev_pool.push_back(e);
    }
    if (hipEventRecord(ctx->ev_pool[k], s) != hipSuccess) ctx->ev_error = true;
    ctx->ev_mark.push_back(i);
  }
};

void reset_marks(dbscan_ctx* ctx) {
  ctx->ev_mark.clear();
  ctx->ev_error = false;
  ctx->events_recorded = ctx->profile;
}

// ---------------------------------------------------------------------------
// Launch stages.  grid: cells, boxes, guard, tree (and the float32 coordinates
// and thresholds); count: MarkCore neighbour counts up to count_cap; setting:
// core flags of one minPts, ClusterCore, relabel, ClusterBorder, scatter.
// ---------------------------------------------------------------------------
// The grid after the cell runs: boxes, guard and split, sub-cell order (`subsort`),
// box tree, node lists and float32 coordinates.
// Every stage launches its kernels on a work source `ws`: OneWork{W} for one grid,
// or a ManyWork table for a group of grids that share each launch.  W is the host
// view used to size the launches (for a group: its largest grid) and to choose the
// kernels (the same for every grid of a group).
template <int D, bool F32, class WS>
void stage_grid_back(const Work& W, const WS& ws, hipStream_t s, const Marks& mark, bool subsort);

// A grid cut from the previous (finer) grid of the same cloud: eps = 2^j times its eps.
template <int D, bool F32>
void stage_grid_derived(const Work& W, hipStream_t s, const Marks& mark, int j) {
  const OneWork ws{W};
  const unsigned tiles = (unsigned)ceil_div(W.n, kTile);
  mark(0);
  k_derive<D><<<1, kBlock, 0, s>>>(W, j);
  mark(1);
  mark(2);
  mark(3);
  k_cells<D><<<tiles, kBlock, 0, s>>>(ws, 2);
  mark(4);
  // no sub-cell regrouping: the points keep the finer grid's order, in which the
  // large cells' chunks are already compact (each lies in one finer cell, itself in
  // sub-cell order when large); measured faster on the 10M-point sweep (12.8 against
  // 14.9 ms per batched step, identical outputs)
  stage_grid_back<D, F32>(W, ws, s, mark, false);
}

// The box method's cells in 2 dimensions, for a grid built alone (see box.hpp):
// strips by x, boxes by y inside each strip, each cut by binary search and pointer
// jumping; the box ids are the sorted keys that k_cells cuts.  Profiling counts the
// whole construction as the keys phase.
template <bool F32>
void stage_grid_box(const Work& W, const OneWork& ws, hipStream_t s, const Marks& mark, bool first) {
  const int64_t n = W.n;
  const unsigned nb = grid_for(n, kBlock, kBBoxBlocks);
  const unsigned tiles = (unsigned)ceil_div(n, kTile);
  const unsigned gp = grid_for(n, kBlock, 2048);
  const unsigned gk = grid_for(n, kBlock, 512);
  const unsigned nsb = (unsigned)ceil_div(n, kBoxScanItems);
  int rounds = 1;  // 2^rounds > n: longer than any chain of parents
  while ((int64_t{1} << rounds) <= n) ++rounds;
  auto sort = [&]() {
    for (int pass = 0; pass < 8; ++pass) k_sort_pass<<<tiles, kBlock, 0, s>>>(ws, pass);
  };
  auto cut = [&](int axis) {
    k_box_parent<<<gp, kBlock, 0, s>>>(W, axis);
    for (int r = 0; r < rounds; ++r) k_box_jump<<<gp, kBlock, 0, s>>>(W, r);
    k_box_scan_sums<<<nsb, kBlock, 0, s>>>(W);
    k_box_scan_top<<<1, kBlock, 0, s>>>(W, (int)nsb);
    k_box_scan_out<<<nsb, kBlock, 0, s>>>(W, axis);
  };
  mark(0);
  k_bbox_partial<2><<<nb, kBlock, 0, s>>>(ws, first ? 1 : 0);
  mark(1);
  k_box_xkeys<<<gk, kBlock, 0, s>>>(W, (int)nb);  // strips: sorted by x, then cut
  sort();
  cut(0);
  k_box_reset<<<1, kBlock, 0, s>>>(W, 8);  // boxes: sorted by y, then stably by strip
  k_box_ykeys<<<gk, kBlock, 0, s>>>(W);
  sort();
  k_box_reset<<<1, kBlock, 0, s>>>(W, 4);
  k_box_skeys<<<gk, kBlock, 0, s>>>(W);
  sort();
  k_box_ygather<<<gp, kBlock, 0, s>>>(W);
  cut(1);
  mark(2);
  mark(3);
  k_cells<2><<<tiles, kBlock, 0, s>>>(ws, 0);
  mark(4);
  stage_grid_back<2, F32>(W, ws, s, mark, true);
}

template <int D, bool F32, class WS>
void stage_grid(const Work& W, const WS& ws, hipStream_t s, const Marks& mark, bool first) {
  if constexpr (D == 2 && std::is_same<WS, OneWork>::value) {
    if (W.box_cells) {
      stage_grid_box<F32>(W, ws, s, mark, first);
      return;
    }
  }
  const int64_t n = W.n;
  const unsigned nb = grid_for(n, kBlock, kBBoxBlocks);
  const unsigned tiles = (unsigned)ceil_div(n, kTile);
  mark(0);
  k_bbox_partial<D><<<nb, kBlock, 0, s>>>(ws, first ? 1 : 0);
  mark(1);
  // 512 workgroups: each merges its digit histograms into the global ones with
  // one atomic per bin, so fewer, fuller workgroups contend less
  k_keys<D><<<grid_for(n, kBlock, 512), kBlock, 0, s>>>(ws, (int)nb);
  mark(2);
  for (int pass = 0; pass < 8; ++pass) k_sort_pass<<<tiles, kBlock, 0, s>>>(ws, pass);
  mark(3);
  k_cells<D><<<tiles, kBlock, 0, s>>>(ws, 0);
  mark(4);
  stage_grid_back<D, F32>(W, ws, s, mark, true);
}

template <int D, bool F32, class WS>
void stage_grid_back(const Work& W, const WS& ws, hipStream_t s, const Marks& mark, bool subsort) {
  const int64_t n = W.n;
  const unsigned gp = grid_for(n, kBlock, 2048);
  const unsigned gc = grid_for(ceil_div(n, kWave), kWavesPerBlock, 4096);
  const unsigned tiles = (unsigned)ceil_div(n, kTile);
  k_cell_box<D><<<gc, kBlock, 0, s>>>(ws, 0);
  k_cell_span<D><<<gc, kBlock, 0, s>>>(ws, 0);
  k_cell_safe<D><<<gp, kBlock, 0, s>>>(ws);
  // cells that fail the float64 diameter guard become singletons
  k_cells<D><<<tiles, kBlock, 0, s>>>(ws, 1);
  k_cell_box<D><<<gc, kBlock, 0, s>>>(ws, 1);
  k_cell_span<D><<<gc, kBlock, 0, s>>>(ws, 1);
  if (subsort && W.sub_min != kIntMax) k_subsort<D><<<kSubBlocks, kSubThreads, 0, s>>>(ws);
  if (W.sub_min != kIntMax)
    k_group_box<D><<<grid_for(ceil_div(n, kGroupPts), kWavesPerBlock, 1024), kBlock, 0, s>>>(ws);
  mark(5);
  for (int l = 1; l <= 2; ++l) {
    const int64_t nodes = W.tree.cap[l];
    k_tree_level<D><<<grid_for(nodes, kWavesPerBlock, 4096), kBlock, 0, s>>>(ws, l);
  }
  k_tree_tail<D><<<1, kBlock, 0, s>>>(ws, 3);
  const unsigned gl = grid_for(W.tree.cap[1], kWavesPerBlock, 4096);
  if (D <= kNodeListMaxD && F32)
    k_lists_local32<D><<<gl + gp, kBlock, 0, s>>>(ws, (int)gl);
  else if (D <= kNodeListMaxD)
    k_node_lists<D><<<gl, kBlock, 0, s>>>(ws);
  else if (F32)
    k_local32<D><<<gp, kBlock, 0, s>>>(ws);
  mark(6);
}

template <int D, bool F32, class WS>
void stage_count(const Work& W, const WS& ws, hipStream_t s, const Marks& mark) {
  if (W.sparse_mode != 1) {
    const unsigned gm = grid_for((int64_t)W.n * (D <= 3 ? W.mark_split : 1), kWavesPerBlock, 8192);
    // above 3 dimensions the sub-cell path has a kernel of its own (see k_markcore_leaf)
    bool leaf = false;
    if constexpr (D > 3) {
      leaf = W.sub_min != kIntMax;
      if (leaf) k_markcore_leaf<D, F32><<<gm, kBlock, 0, s>>>(ws);
    }
    if (!leaf) k_markcore<D, F32><<<gm, kBlock, 0, s>>>(ws);
  }
  if (W.sparse_mode != 0)
    k_markcore_sparse<D, F32><<<grid_for(ceil_div(W.n, kWave), kWavesPerBlock, 4096), kBlock, 0, s>>>(ws);
  mark(7);
}

// ClusterCore, cluster ids and ClusterBorder of one setting whose core flags are
// set.  A warm start (W.warm) first takes the node roots of the union-find the
// previous setting left, so that ClusterCore prunes subtrees already joined.
template <int D, bool F32, class WS>
void stage_cluster(const Work& W, const WS& ws, hipStream_t s, const Marks& mark, bool rounds) {
  const int64_t n = W.n;
  const unsigned gp = grid_for(n, kBlock, 2048);
  const unsigned gw = grid_for(n, kWavesPerBlock, 4096);
  const unsigned gb = grid_for(n * W.bcp_split, kWavesPerBlock, 8192);
  const unsigned gc = grid_for(ceil_div(n, kWave), kWavesPerBlock, 4096);
  // whether this setting's node roots were taken (ClusterBorder then skips nodes
  // without a core cell: which nodes have one does not change during ClusterCore)
  bool roots_taken = false;
  auto node_roots = [&]() {
    for (int l = 1; l <= kTreeLevels; ++l)
      k_node_roots<<<grid_for(W.tree.cap[l], kWavesPerBlock, 4096), kBlock, 0, s>>>(ws, l);
    roots_taken = true;
  };
  // a warm start that knows the previous core counts runs one pass in any dimension:
  // only cells that gained core points act (see k_bcp)
  auto bcp = [&](int round) {
    if constexpr (D > 3) {
      if (W.sub_min != kIntMax) {  // the sub-cell path's own kernel (see k_bcp_leaf)
        if (W.warm) k_bcp_leaf<D, F32, true><<<gb, kBlock, 0, s>>>(ws, round);
        else k_bcp_leaf<D, F32, false><<<gb, kBlock, 0, s>>>(ws, round);
        return;
      }
    }
    if (W.warm) k_bcp<D, F32, true><<<gb, kBlock, 0, s>>>(ws, round);
    else k_bcp<D, F32, false><<<gb, kBlock, 0, s>>>(ws, round);
  };
  if (W.sparse_mode == 1) {
    // batched sparse kernel only
  } else if (!rounds || (W.warm && W.prev_core_count)) {
    // (with the previous counts only cells that gained core points act, and they
    // need no subtree pruning: the node roots are not taken)
    if (W.warm && !W.prev_core_count) node_roots();
    bcp(-1);
  } else {
    for (int round = 0; round < kTreeLevels; ++round) {
      if (round > 0 || W.warm) node_roots();
      bcp(round);
    }
  }
  if (W.sparse_mode != 0) {
    const unsigned gn = grid_for(ceil_div(n, kWave), kWavesPerBlock, 4096);
    if (W.warm) k_bcp_sparse<D, F32, true><<<gn, kBlock, 0, s>>>(ws);
    else k_bcp_sparse<D, F32, false><<<gn, kBlock, 0, s>>>(ws);
  }
  mark(W.warm ? kPhaseClusterWarm + 1 : 9);
  k_relabel_min<<<gc, kBlock, 0, s>>>(ws);
  k_cell_label<<<gp, kBlock, 0, s>>>(ws);
  mark(10);
  if (W.sparse_mode != 1) k_border<D, F32><<<gw, kBlock, 0, s>>>(ws, roots_taken ? 1 : 0);
  if (W.sparse_mode != 0)
    k_border_sparse<D, F32><<<grid_for(ceil_div(n, kWave), kWavesPerBlock, 4096), kBlock, 0, s>>>(ws);
  mark(11);
}

template <int D, bool F32, class WS>
void stage_setting(const Work& W, const WS& ws, hipStream_t s, const Marks& mark, bool rounds) {
  const int64_t n = W.n;
  const unsigned gp = grid_for(n, kBlock, 2048);
  const unsigned gw = grid_for(n, kWavesPerBlock, 4096);
  k_core_from_count<<<gw, kBlock, 0, s>>>(ws);
  mark(8);
  stage_cluster<D, F32>(W, ws, s, mark, rounds);
  k_scatter<<<gp, kBlock, 0, s>>>(ws);
  mark(12);
}

// One grid per launch.
template <int D, bool F32>
void one_grid(const Work& W, hipStream_t s, const Marks& m, bool first) {
  stage_grid<D, F32>(W, OneWork{W}, s, m, first);
}
template <int D, bool F32>
void one_count(const Work& W, hipStream_t s, const Marks& m) {
  stage_count<D, F32>(W, OneWork{W}, s, m);
}
template <int D, bool F32>
void one_setting(const Work& W, hipStream_t s, const Marks& m, bool rounds) {
  stage_setting<D, F32>(W, OneWork{W}, s, m, rounds);
}
template <int D, bool F32>
void one_cluster(const Work& W, hipStream_t s, const Marks& m, bool rounds) {
  stage_cluster<D, F32>(W, OneWork{W}, s, m, rounds);
}

// A group of single-setting grids sharing every launch: grid, count and setting.
template <int D, bool F32>
void group_run(const Work& W, const ManyWork& ws, hipStream_t s, const Marks& m, bool rounds) {
  stage_grid<D, F32>(W, ws, s, m, true);  // (each grid clears its own descriptor)
  stage_count<D, F32>(W, ws, s, m);
  stage_setting<D, F32>(W, ws, s, m, rounds);
}

struct Stages {
  void (*grid)(const Work&, hipStream_t, const Marks&, bool);
  void (*derived)(const Work&, hipStream_t, const Marks&, int);
  void (*count)(const Work&, hipStream_t, const Marks&);
  void (*setting)(const Work&, hipStream_t, const Marks&, bool);
  void (*cluster)(const Work&, hipStream_t, const Marks&, bool);
  void (*group)(const Work&, const ManyWork&, hipStream_t, const Marks&, bool);
};

template <int D, bool F32>
Stages stages_of() {
  return Stages{&one_grid<D, F32>,    &stage_grid_derived<D, F32>, &one_count<D, F32>,
                &one_setting<D, F32>, &one_cluster<D, F32>,        &group_run<D, F32>};
}

Stages stages_for(int d, bool f32) {
  switch (d) {
#define DB_STAGES(DD) \
  case DD:            \
    return f32 ? stages_of<DD, true>() : stages_of<DD, false>();
    DB_STAGES(1)
    DB_STAGES(2)
    DB_STAGES(3)
    DB_STAGES(4)
    DB_STAGES(5)
    DB_STAGES(6)
    DB_STAGES(7)
    DB_STAGES(8)
#undef DB_STAGES
  }
  return Stages{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
}

// Whether a call in `mode` takes its pair decisions through the float32 filter:
// only up to filter_max_d dimensions (on this GPU unpacked float32 runs at the
// float64 rate, and in higher dimensions the per-cell anchors cost more loads
// than the float32 coordinates save, so there float64 decides directly).
bool use_filter(const dbscan_ctx* ctx, int mode, int d) {
  const int maxd = ctx->filter_max_d >= 0 ? ctx->filter_max_d : 3;
  return mode == DBSCAN_FP32_FILTER && d <= maxd;
}

int size_class(int64_t n) {
  int lg = 0;
  while (lg < 62 && (int64_t(1) << (lg + 1)) <= n) ++lg;
  return lg;
}

const TunedEntry* find_tuned(const dbscan_ctx* ctx, int64_t n, int d, int mode) {
  const int lg = size_class(n);
  for (const TunedEntry& e : ctx->tuned)
    if (e.d == d && e.mode == mode && e.lg == lg) return &e;
  return nullptr;
}

// The automatic sub-cell threshold: above 3 dimensions sub-cell order is only taken
// when asked for (an option or a tuned entry), since cells there mostly hold few
// points and its kernels need more registers.
int sub_auto(int d) { return d <= 3 ? kSubMinAuto : 0; }

// Explicit options win; automatic ones come from the tuned table, else from fixed
// rules (one pass for d <= 3, rounds above; one wave per unit).
Resolved resolve(const dbscan_ctx* ctx, int64_t n, int d, int mode) {
  Resolved r{d > 3 ? 1 : 0, 1, 0, 0, sub_auto(d), kMarkSplit, kDenseGroup};
  if (const TunedEntry* e = find_tuned(ctx, n, d, mode)) r = e->r;
  if (ctx->subcell_min >= 0) r.sub = ctx->subcell_min;
  if (ctx->bcp_rounds >= 0) r.rounds = ctx->bcp_rounds;
  if (ctx->unit_level >= 0) r.unit_level = ctx->unit_level;
  if (ctx->fine_bits >= 0) r.fine = ctx->fine_bits;
  if (ctx->bcp_split > 0) r.split = ctx->bcp_split;
  if (r.split <= 0) r.split = 1;
  if (ctx->mark_split > 0) r.mark_split = ctx->mark_split;
  if (ctx->dense_group > 0) r.dense = ctx->dense_group;
  return r;
}

// Fields of Work shared by every stage of one grid.
// base/desc: the arrays and descriptor of one grid of a group (default: the single-grid
// region after the context's descriptor).
void fill_work(dbscan_ctx* ctx, Work& W, const double* points, int64_t n, int d, double eps,
               const Resolved& R, int slots = 1, bool keep_keys = false, char* base = nullptr,
               GridDesc* desc = nullptr) {
  std::memset(static_cast<void*>(&W), 0, sizeof(W));
  if (!base && ctx->group_area_off &&
      ctx->desc_bytes + layout(nullptr, n, d, nullptr, slots, keep_keys) > ctx->group_area_off) {
    // this grid overwrites the group area: a later grouped batch lays it out again
    ctx->group_area_off = 0;
    ctx->group_key.clear();
    drop_graph(ctx);
  }
  W.n = (int)n;
  W.eps = eps;
  W.E2 = eps * eps;
  W.E2b = W.E2;
  W.E2leaf = 0.0;
  W.side = eps / std::sqrt((double)d);
  W.pts = points;
  W.desc = desc ? desc : ctx->desc;
  W.fine_max = R.fine;
  // sub-cell order after the grid is built, only without sort-time fine bits
  W.sub_min = (R.fine == 0 && R.sub > 0) ? R.sub : kIntMax;
  W.box_cells = box_cells(ctx, d) ? 1 : 0;
  W.unit_max_level = R.unit_level;
  W.force_recheck = ctx->force_recheck;
  W.bcp_split = R.split;
  W.mark_split = R.mark_split;
  W.dense_group = R.dense;
  W.warm = 0;
  W.prev_core_count = nullptr;
  W.core_mask = 1u;
  W.sparse_mode = ctx->sparse == 1 ? 1 : 0;
  layout(base ? base : static_cast<char*>(ctx->scratch) + ctx->desc_bytes, n, d, &W, slots,
         keep_keys);
}

int check_args(int64_t n, int32_t d, double eps, int32_t min_pts) {
  if (n < 0 || n > DBSCAN_MAX_N || d < 1 || d > DBSCAN_MAX_D) return DBSCAN_EINVAL;
  if (!(eps > 0.0) || !std::isfinite(eps) || min_pts < 1) return DBSCAN_EINVAL;
  return DBSCAN_OK;
}

// Most settings of one eps in a batch (kMultiMax per group of per-setting arrays).
int batch_slots(const dbscan_instance* inst, int32_t count) {
  int slots = 1;
  for (int32_t i = 0; i < count; ++i) {
    const dbscan_instance& I = inst[i];
    for (int32_t a = 0; a < I.n_settings; ++a) {
      int same = 0;
      for (int32_t b = 0; b < I.n_settings; ++b) same += I.eps[b] == I.eps[a];
      slots = std::max(slots, std::min(same, kMultiMax));
    }
  }
  return slots;
}

// The grids of one cloud, one per distinct eps.  Eps values that differ by a power
// of two (equal binary mantissas) form a chain, taken in increasing order: the
// first grid of a chain is sorted and keeps its sorted keys, each further one is
// cut from the one before (derive_j levels coarser) without sorting again.
struct EpsStep {
  double eps;
  int derive_j;    // 0: a sorted grid; j > 0: cut from the previous grid (eps / 2^j)
  bool keep_keys;  // a later grid of the chain is cut from this one
};

// chains: false for grids that cannot be cut from a finer one (the box method)
std::vector<EpsStep> eps_plan(const dbscan_instance& I, bool chains = true) {
  std::vector<double> es;
  for (int32_t a = 0; a < I.n_settings; ++a)
    if (std::find(es.begin(), es.end(), I.eps[a]) == es.end()) es.push_back(I.eps[a]);
  std::vector<EpsStep> plan;
  std::vector<char> used(es.size(), 0);
  for (size_t a = 0; a < es.size(); ++a) {
    if (used[a]) continue;
    int ea;
    const double ma = std::frexp(es[a], &ea);
    std::vector<std::pair<int, double>> chain;  // (exponent, eps)
    for (size_t b = a; b < es.size(); ++b) {
      int eb;
      if (!used[b] && (b == a || chains) && std::frexp(es[b], &eb) == ma) {
        used[b] = 1;
        chain.push_back({eb, es[b]});
      }
    }
    std::sort(chain.begin(), chain.end());
    for (size_t c = 0; c < chain.size(); ++c)
      plan.push_back(EpsStep{chain[c].second, c == 0 ? 0 : chain[c].first - chain[c - 1].first,
                             c + 1 < chain.size()});
  }
  return plan;
}

bool plan_keeps_keys(const dbscan_ctx* ctx, const dbscan_instance* inst, int32_t count) {
  for (int32_t i = 0; i < count; ++i)
    for (const EpsStep& P : eps_plan(inst[i], !box_cells(ctx, inst[i].d)))
      if (P.keep_keys) return true;
  return false;
}


template <class T>
void put(std::vector<unsigned char>& k, const T& v) {
  const unsigned char* p = reinterpret_cast<const unsigned char*>(&v);
  k.insert(k.end(), p, p + sizeof(T));
}

// The status bits and counters of a group's grids, added to the context's
// descriptor (one workgroup of kCtrSlots threads); its cell counts become the last
// grid's.  clear: the descriptor starts from zero (no single grid ran before).
__global__ void k_group_merge(ConstWork* Ws, int k, GridDesc* main, int clear) {
  const int t = threadIdx.x;
  for (int w = 0; w < 5; ++w) {
    unsigned long long v = clear ? 0ull : main->ctr[w][t];
    for (int c = 0; c < k; ++c) v += Ws[c].desc->ctr[w][t];
    main->ctr[w][t] = v;
  }
  if (t == 0) {
    uint32_t st = clear ? 0u : main->status;
    for (int c = 0; c < k; ++c) st |= Ws[c].desc->status;
    main->status = st;
    main->n_cells = Ws[k - 1].desc->n_cells;
    main->n_unsafe = Ws[k - 1].desc->n_unsafe;
  }
}

// Grouped clouds: instances with one setting, of the same dimension and options,
// run as one group whose grids share every launch (OneWork / ManyWork), instead of
// a chain of launches per cloud.  Each grid keeps its own descriptor and arrays, in
// a region of its own after the single-grid region, and the group's Work table sits
// in front of its regions.
struct GroupPlan {
  std::vector<int32_t> members;  // instance indices, in batch order
  int d = 0;
  bool f32 = false;
  Resolved R{};
  size_t table_off = 0;            // from the start of the scratch
  std::vector<size_t> region_off;  // each member's descriptor, then its arrays
  Work host{};                     // launch sizes (largest grid) and options of the group
  Work last{};                     // the last member's grid (for the stats)
};

struct BatchPlan {
  std::vector<GroupPlan> groups;
  std::vector<char> grouped;  // per instance
  int64_t nmax = 0;           // largest instance of the single-grid path
  int32_t dmax = 1;
  size_t area_off = 0;        // group area: after the single-grid region
  size_t area_bytes = 0;
};

bool same_resolved(const Resolved& a, const Resolved& b) {
  return a.rounds == b.rounds && a.unit_level == b.unit_level && a.split == b.split &&
         a.fine == b.fine && a.sub == b.sub && a.mark_split == b.mark_split &&
         a.dense == b.dense;
}

#ifndef DB_GROUP_MAX_N
#define DB_GROUP_MAX_N (1 << 17)
#endif
// Automatic grouping in more than 3 dimensions takes clouds of at most this many
// points.  There the tree walks of a large cloud read much more than the caches
// hold, and grouped large clouds ran slower than alone (their waves spread over many
// clouds at once): on the 5-dimensional clouds of the 256-cloud batch, 906 ms
// grouped whole against 700 ms with this limit and 723 ms ungrouped.  Up to 3
// dimensions every size gains from grouping (2D: 19.7 -> 8.8 ms, 3D: 81 -> 53 ms).
constexpr int64_t kGroupMaxN = DB_GROUP_MAX_N;

BatchPlan plan_batch(const dbscan_ctx* ctx, const dbscan_instance* inst, int32_t count,
                     int32_t mode, int slots, bool keep_keys) {
  BatchPlan P;
  P.grouped.assign((size_t)std::max(count, 0), 0);
  if (ctx->group_clouds != 0) {
    for (int32_t i = 0; i < count; ++i) {
      const dbscan_instance& I = inst[i];
      if (I.n == 0 || I.n_settings != 1 || box_cells(ctx, I.d)) continue;
      if (ctx->group_clouds < 0 && I.d > 3 && I.n > kGroupMaxN) continue;
      const bool f32 = use_filter(ctx, mode, I.d);
      const Resolved R = resolve(ctx, I.n, I.d, mode);
      GroupPlan* g = nullptr;
      for (GroupPlan& G : P.groups)
        if (G.d == I.d && G.f32 == f32 && same_resolved(G.R, R)) g = &G;
      if (!g) {
        P.groups.emplace_back();
        g = &P.groups.back();
        g->d = I.d;
        g->f32 = f32;
        g->R = R;
      }
      g->members.push_back(i);
    }
    const size_t min_size = ctx->group_clouds == 1 ? 1 : 2;
    std::vector<GroupPlan> keep;
    for (GroupPlan& G : P.groups)
      if (G.members.size() >= min_size) keep.push_back(std::move(G));
    P.groups.swap(keep);
  }
  for (const GroupPlan& G : P.groups)
    for (int32_t i : G.members) P.grouped[i] = 1;
  for (int32_t i = 0; i < count; ++i)
    if (!P.grouped[i]) {
      P.nmax = std::max(P.nmax, inst[i].n);
      P.dmax = std::max(P.dmax, inst[i].d);
    }
  P.area_off = ctx->desc_bytes + layout(nullptr, P.nmax, P.dmax, nullptr, slots, keep_keys);
  size_t off = P.area_off;
  for (GroupPlan& G : P.groups) {
    G.table_off = off;
    off += align_up(sizeof(Work) * G.members.size());
    for (int32_t i : G.members) {
      G.region_off.push_back(off);
      off += ctx->desc_bytes + layout(nullptr, inst[i].n, G.d, nullptr);
    }
  }
  P.area_bytes = off - P.area_off;
  return P;
}

// Everything the group descriptors were set up for: a different layout gets fresh
// descriptors.
std::vector<unsigned char> group_layout_key(const dbscan_ctx* ctx, const BatchPlan& P,
                                            const dbscan_instance* inst) {
  std::vector<unsigned char> k;
  put(k, ctx->scratch);
  put(k, ctx->scratch_bytes);
  put(k, P.area_off);
  for (const GroupPlan& G : P.groups)
    for (size_t m = 0; m < G.members.size(); ++m) {
      put(k, G.region_off[m]);
      put(k, inst[G.members[m]].n);
      put(k, G.d);
    }
  return k;
}

// Fills each group's Work table (host copies kept in the context) and writes it to
// the device on stream s (never under capture).  A new layout first gives every
// grid's descriptor a fresh epoch base: look-back words left in the region by
// another layout then carry epochs the new grid does not reach.
int prepare_groups(dbscan_ctx* ctx, BatchPlan& P, const dbscan_instance* inst, int32_t mode,
                   hipStream_t s) {
  if (P.groups.empty()) return DBSCAN_OK;
  char* base = static_cast<char*>(ctx->scratch);
  std::vector<unsigned char> key = group_layout_key(ctx, P, inst);
  const bool fresh = key != ctx->group_key;
  if (fresh) {
    ctx->group_seed += 1u << 16;
    GridDesc d0;
    std::memset(static_cast<void*>(&d0), 0, sizeof(d0));
    d0.epoch = ctx->group_seed;
    for (const GroupPlan& G : P.groups)
      for (size_t off : G.region_off)
        if (hipMemcpyAsync(base + off, &d0, sizeof(d0), hipMemcpyHostToDevice, s) != hipSuccess)
          return DBSCAN_EHIP;
  }
  std::vector<Work>& T = ctx->group_table_host;
  for (GroupPlan& G : P.groups) {
    T.assign(G.members.size(), Work{});
    for (size_t m = 0; m < G.members.size(); ++m) {
      const dbscan_instance& I = inst[G.members[m]];
      Work& W = T[m];
      char* rb = base + G.region_off[m];
      fill_work(ctx, W, I.points, I.n, I.d, I.eps[0], G.R, 1, false, rb + ctx->desc_bytes,
                reinterpret_cast<GridDesc*>(rb));
      W.count_cap = I.min_pts[0];
      W.minPts = I.min_pts[0];
      W.core_out = I.core_flags;
      W.label_out = I.cluster_id;
    }
    // launch sizes of the largest grid; every grid of the group takes the same
    // kernels (same dimension, mode and options)
    G.host = T[0];
    for (const Work& W : T) {
      G.host.n = std::max(G.host.n, W.n);
      for (int l = 0; l <= kTreeLevels; ++l) G.host.tree.cap[l] = std::max(G.host.tree.cap[l], W.tree.cap[l]);
      G.host.chunkCap = std::max(G.host.chunkCap, W.chunkCap);
    }
    G.last = T.back();
    if (hipMemcpyAsync(base + G.table_off, T.data(), sizeof(Work) * T.size(),
                       hipMemcpyHostToDevice, s) != hipSuccess)
      return DBSCAN_EHIP;
  }
  // the copies read host memory that is rewritten by the next call
  if (hipStreamSynchronize(s) != hipSuccess) return DBSCAN_EHIP;
  ctx->group_area_off = P.area_off;
  ctx->group_key.swap(key);
  return DBSCAN_OK;
}

// Enqueue a whole batch on stream s (eagerly or under capture).  Settings of one
// instance with equal eps share the grid and one neighbour count, taken up to the
// largest of their minPts.  They are taken by decreasing minPts: the core points of
// a smaller minPts include those of a larger one, so every link the larger one made
// is a link of the smaller one too, and ClusterCore starts from the union-find the
// previous setting left (it then only tests cells not yet joined).  Their core
// flags are set together (one bit per setting) and their outputs are written
// together, in input order, after the last of them.
int enqueue_batch(dbscan_ctx* ctx, const dbscan_instance* inst, int32_t count, bool f32,
                  hipStream_t s, const Marks& marks, int slots, bool keep_keys,
                  const BatchPlan& plan) {
  bool first = true;
  for (int32_t i = 0; i < count; ++i) {
    const dbscan_instance& I = inst[i];
    if (I.n == 0 || plan.grouped[i]) continue;
    const int mode = f32 ? DBSCAN_FP32_FILTER : DBSCAN_PLAIN_FP64;
    const Stages st = stages_for(I.d, use_filter(ctx, mode, I.d));
    const Resolved R = resolve(ctx, I.n, I.d, mode);
    const bool rounds = R.rounds != 0;
    const int64_t n = I.n;
    const std::vector<EpsStep> plan = eps_plan(I, !box_cells(ctx, I.d));
    for (size_t pi = 0; pi < plan.size(); ++pi) {
      const EpsStep& P = plan[pi];
      const double eps = P.eps;
      std::vector<int> grp;
      for (int32_t b = 0; b < I.n_settings; ++b)
        if (I.eps[b] == eps) grp.push_back(b);
      std::stable_sort(grp.begin(), grp.end(),
                       [&](int x, int y) { return I.min_pts[x] > I.min_pts[y]; });
      Work W;
      fill_work(ctx, W, I.points, n, I.d, eps, R, slots, keep_keys);
      W.count_cap = I.min_pts[grp[0]];
      // (the inverse permutation, when kept, follows every grid of the batch: a later
      // grid of the same chain keeps this one's order)
      if (!P.keep_keys && P.derive_j == 0) W.skey = nullptr;  // a cut grid reads the kept keys
      if (P.derive_j > 0) st.derived(W, s, marks, P.derive_j);
      else st.grid(W, s, marks, first);
      first = false;
      st.count(W, s, marks);
      if (grp.size() == 1) {
        Work Ws = W;
        Ws.minPts = I.min_pts[grp[0]];
        Ws.core_out = I.core_flags + (size_t)grp[0] * (size_t)n;
        Ws.label_out = I.cluster_id + (size_t)grp[0] * (size_t)n;
        st.setting(Ws, s, marks, rounds);
        ctx->stats_valid = true;
        ctx->stats_work = Ws;
        continue;
      }
      const unsigned gp = grid_for(n, kBlock, 2048);
      for (size_t c0 = 0; c0 < grp.size(); c0 += kMultiMax) {
        const int k = (int)std::min<size_t>(kMultiMax, grp.size() - c0);
        MultiCore M{};
        MultiOut O{};
        M.k = O.k = k;
        M.warm = c0 > 0;
        for (int t = 0; t < k; ++t) {
          M.minPts[t] = I.min_pts[grp[c0 + t]];
          M.coreCount[t] = W.coreCount + (size_t)t * n;
          M.cellMin[t] = W.cellMin + (size_t)t * n;
          M.minIdx[t] = W.minIdx + (size_t)t * n;
        }
        k_core_multi_init<<<grid_for(n, kBlock, 2048), kBlock, 0, s>>>(W, M);
        k_core_multi<<<grid_for(ceil_div(n, kWave * kCoreRun), kWavesPerBlock, 4096), kBlock, 0,
                       s>>>(W, M);
        marks(8);
        for (int t = 0; t < k; ++t) {
          const int b = grp[c0 + t];
          Work Ws = W;
          Ws.minPts = I.min_pts[b];
          Ws.core_mask = 1u << t;
          Ws.warm = (c0 + t) > 0;
          Ws.prev_core_count = t > 0 ? M.coreCount[t - 1] : nullptr;
          Ws.coreCount = M.coreCount[t];
          Ws.cellMin = M.cellMin[t];
          Ws.minIdx = M.minIdx[t];
          Ws.cellLabel = W.cellLabel + (size_t)t * n;
          Ws.blabel = W.blabel + (size_t)t * n;
          Ws.core_out = I.core_flags + (size_t)b * (size_t)n;
          Ws.label_out = I.cluster_id + (size_t)b * (size_t)n;
          st.cluster(Ws, s, marks, rounds);
          O.core[t] = Ws.core_out;
          O.label[t] = Ws.label_out;
          O.cellLabel[t] = Ws.cellLabel;
          O.blabel[t] = Ws.blabel;
          ctx->stats_valid = true;
          ctx->stats_work = Ws;
        }
        k_output_multi<<<gp, kBlock, 0, s>>>(W, O);
        marks(12);
      }
    }
  }
  char* base = static_cast<char*>(ctx->scratch);
  for (const GroupPlan& G : plan.groups) {
    const Stages st = stages_for(G.d, G.f32);
    const ManyWork ws{(ConstWork*)(base + G.table_off), (int)G.members.size()};
    st.group(G.host, ws, s, marks, G.R.rounds != 0);
    // status bits and counters of the group's grids into the context's descriptor
    // (cleared first when no single grid ran before)
    k_group_merge<<<1, kCtrSlots, 0, s>>>(ws.Ws, ws.k, ctx->desc, first ? 1 : 0);
    first = false;
    // n_core in the stats: the last grid's core points, counted into the context's
    // descriptor
    ctx->stats_valid = true;
    ctx->stats_work = G.last;
    ctx->stats_work.desc = ctx->desc;
  }
  return hipGetLastError() == hipSuccess ? DBSCAN_OK : DBSCAN_EHIP;
}

// Everything a captured batch depends on.
std::vector<unsigned char> batch_key(const dbscan_ctx* ctx, const dbscan_instance* inst,
                                     int32_t count, int32_t mode) {
  std::vector<unsigned char> k;
  put(k, ctx->scratch);
  put(k, ctx->scratch_bytes);
  put(k, mode);
  put(k, ctx->bcp_rounds);
  put(k, ctx->unit_level);
  put(k, ctx->fine_bits);
  put(k, ctx->force_recheck);
  put(k, ctx->bcp_split);
  put(k, ctx->tune_gen);
  put(k, ctx->filter_max_d);
  put(k, ctx->subcell_min);
  put(k, ctx->sparse);
  put(k, ctx->group_clouds);
  put(k, ctx->mark_split);
  put(k, ctx->dense_group);
  put(k, count);
  for (int32_t i = 0; i < count; ++i) {
    const dbscan_instance& I = inst[i];
    put(k, I.points);
    put(k, I.n);
    put(k, I.d);
    put(k, I.n_settings);
    put(k, I.core_flags);
    put(k, I.cluster_id);
    for (int32_t a = 0; a < I.n_settings; ++a) {
      put(k, I.eps[a]);
      put(k, I.min_pts[a]);
    }
  }
  return k;
}

}  // namespace

namespace {

template <int D>
void member_pass(const Work& W, hipStream_t s, int phase, int64_t* count, const int64_t* offsets,
                 int32_t* ids, uint32_t* overflow) {
  k_member<D><<<grid_for(ceil_div(W.n, kWave), kWavesPerBlock, 4096), kBlock, 0, s>>>(
      W, phase, count, offsets, ids, overflow);
}

void member_dispatch(int d, const Work& W, hipStream_t s, int phase, int64_t* count,
                     const int64_t* offsets, int32_t* ids, uint32_t* overflow) {
  switch (d) {
#define DB_MEMBER(DD) \
  case DD:            \
    member_pass<DD>(W, s, phase, count, offsets, ids, overflow); \
    break;
    DB_MEMBER(1)
    DB_MEMBER(2)
    DB_MEMBER(3)
    DB_MEMBER(4)
    DB_MEMBER(5)
    DB_MEMBER(6)
    DB_MEMBER(7)
    DB_MEMBER(8)
#undef DB_MEMBER
  }
}

}  // namespace

extern "C" {

int dbscan_ctx_create(dbscan_ctx** out, int device) {
  if (!out) return DBSCAN_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess) return DBSCAN_EHIP;
  if (device < 0 || device >= count) return DBSCAN_EINVAL;
  dbscan_ctx* c = new (std::nothrow) dbscan_ctx();
  if (!c) return DBSCAN_ENOMEM;
  c->device = device;
  c->desc_bytes = align_up(sizeof(GridDesc));
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return DBSCAN_EHIP;
  }
  void* p = nullptr;
  if (hipMalloc(&p, c->desc_bytes) != hipSuccess) {
    delete c;
    return DBSCAN_ENOMEM;
  }
  if (hipMemset(p, 0, c->desc_bytes) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    (void)hipFree(p);
    delete c;
    return DBSCAN_EHIP;
  }
  c->scratch = p;
  c->scratch_bytes = c->desc_bytes;
  c->desc = reinterpret_cast<GridDesc*>(p);
  *out = c;
  return DBSCAN_OK;
}

int dbscan_ctx_destroy(dbscan_ctx* ctx) {
  if (!ctx) return DBSCAN_EINVAL;
  int rc = DBSCAN_OK;
  if (hipSetDevice(ctx->device) != hipSuccess) rc = DBSCAN_EHIP;
  if (hipDeviceSynchronize() != hipSuccess) rc = DBSCAN_EHIP;
  drop_graph(ctx);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  if (ctx->scratch && hipFree(ctx->scratch) != hipSuccess) rc = DBSCAN_EHIP;
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  delete ctx;
  return rc;
}

int dbscan_reserve(dbscan_ctx* ctx, int64_t n, int32_t d) {
  if (!ctx || n < 0 || n > DBSCAN_MAX_N || d < 1 || d > DBSCAN_MAX_D) return DBSCAN_EINVAL;
  return grow(ctx, n, d);
}

namespace {

// One exact DBSCAN with the given options (arguments already checked, n > 0).
int run_one(dbscan_ctx* ctx, const double* points, int64_t n, int32_t d, double eps,
            int32_t min_pts, int32_t mode, uint8_t* core_flags, int32_t* cluster_id,
            hipStream_t s, const Resolved& R, double rho = 0.0) {
  if (hipSetDevice(ctx->device) != hipSuccess) return DBSCAN_EHIP;
  int rc = grow(ctx, n, d);
  if (rc != DBSCAN_OK) return rc;
  Work W;
  fill_work(ctx, W, points, n, d, eps, R);
  if (rho > 0.0) {
    // approximate DBSCAN: ClusterCore links core points up to R = eps (1 + rho), and
    // takes a leaf of diameter at most eps rho / 2 whole (see BcpVisitor::tile)
    const double r = eps * (1.0 + rho);
    W.E2b = r * r;
    // (not for rho below 1e-6, where the margin of rho / 2 nears the rounding of the
    // tests; such leaves would hold next to nothing anyway)
    const double l = 0.5 * eps * rho;
    if (rho >= 1e-6) W.E2leaf = l * l;
  }
  W.count_cap = min_pts;
  W.minPts = min_pts;
  W.core_out = core_flags;
  W.label_out = cluster_id;
  ctx->last_n = n;
  ctx->last_valid = true;
  ctx->last_d = d;
  ctx->last_work = W;
  ctx->stats_valid = true;
  ctx->stats_work = W;
  reset_marks(ctx);
  const Marks mark{ctx->profile ? ctx : nullptr, s};
  const Stages st = stages_for(d, use_filter(ctx, mode, d));
  st.grid(W, s, mark, true);
  st.count(W, s, mark);
  st.setting(W, s, mark, R.rounds != 0);
  return hipGetLastError() == hipSuccess ? DBSCAN_OK : DBSCAN_EHIP;
}

int check_call(const dbscan_ctx* ctx, const double* points, int64_t n, int32_t d, double eps,
               int32_t min_pts, int32_t mode, const uint8_t* core_flags,
               const int32_t* cluster_id) {
  if (!ctx) return DBSCAN_EINVAL;
  const int rc = check_args(n, d, eps, min_pts);
  if (rc != DBSCAN_OK) return rc;
  if (mode != DBSCAN_PLAIN_FP64 && mode != DBSCAN_FP32_FILTER) return DBSCAN_EINVAL;
  if (n > 0 && (!points || !core_flags || !cluster_id)) return DBSCAN_EINVAL;
  return DBSCAN_OK;
}

}  // namespace

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free calls (dbscan_noalloc): the scratch of one call lives in a
// file-scope device array of fixed size instead of a context's allocation.  Each
// GPU holds its own copy of the array for the life of the process; host code
// never uses the array's name (a host-side stand-in), only the device address
// hipGetSymbolAddress returns, looked up once per device.  The array starts
// zeroed (the code object's zero-filled segment), so the call descriptor at its
// start begins with epoch 0 and no look-back word of an earlier call can match a
// later call's epoch.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[DBSCAN_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kNoAllocDevices = 64;

struct NoAllocSlot {
  bool ready = false;
  void* ptr = nullptr;  // device address of `scratch` on this device
  dbscan_ctx ctx;       // default options, scratch = ptr (never grown)
};

NoAllocSlot g_noalloc[kNoAllocDevices];
std::mutex g_noalloc_mu;

// The call's status bits (0 for a call with no points: g == nullptr).
__global__ void k_status_out(const GridDesc* g, uint32_t* out) {
  if (threadIdx.x == 0) *out = g ? g->status : 0u;
}

// The slot of device dev, set up on its first use (dev current).
int noalloc_slot(int dev, NoAllocSlot** out) {
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  NoAllocSlot& S = g_noalloc[dev];
  if (!S.ready) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return DBSCAN_EHIP;
    // the lookup may leave an error recorded for code objects it searched before
    // finding the symbol; it succeeded, so that record is dropped
    (void)hipGetLastError();
    S.ptr = p;
    S.ctx.device = dev;
    S.ctx.desc_bytes = align_up(sizeof(GridDesc));
    S.ctx.scratch = p;
    S.ctx.scratch_bytes = DBSCAN_NOALLOC_SCRATCH_BYTES;
    S.ctx.desc = reinterpret_cast<GridDesc*>(p);
    S.ready = true;
  }
  *out = &S;
  return DBSCAN_OK;
}

}  // namespace

extern "C" {

int dbscan_noalloc(const double* points, int64_t n, int32_t d, double eps, int32_t min_pts,
                   int32_t mode, uint8_t* core_flags, int32_t* cluster_id, uint32_t* status,
                   void* stream) {
  int rc = check_args(n, d, eps, min_pts);
  if (rc != DBSCAN_OK) return rc;
  if (mode != DBSCAN_PLAIN_FP64 && mode != DBSCAN_FP32_FILTER) return DBSCAN_EINVAL;
  if (n > 0 && (!points || !core_flags || !cluster_id)) return DBSCAN_EINVAL;
  if (align_up(sizeof(GridDesc)) + layout(nullptr, n, d, nullptr) > DBSCAN_NOALLOC_SCRATCH_BYTES)
    return DBSCAN_ETOOLARGE;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return DBSCAN_EHIP;
  if (dev < 0 || dev >= kNoAllocDevices) return DBSCAN_EINVAL;
  NoAllocSlot* S = nullptr;
  rc = noalloc_slot(dev, &S);
  if (rc != DBSCAN_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (n > 0) {
    // the size check above keeps run_one's scratch growth a no-op: nothing is allocated
    rc = run_one(&S->ctx, points, n, d, eps, min_pts, mode, core_flags, cluster_id, s,
                 resolve(&S->ctx, n, d, mode));
    if (rc != DBSCAN_OK) return rc;
  }
  if (status) {
    if (n > 0) k_status_out<<<1, 64, 0, s>>>(S->ctx.desc, status);
    else k_status_out<<<1, 64, 0, s>>>(nullptr, status);
  }
  return hipGetLastError() == hipSuccess ? DBSCAN_OK : DBSCAN_EHIP;
}

int dbscan(dbscan_ctx* ctx, const double* points, int64_t n, int32_t d, double eps,
           int32_t min_pts, int32_t mode, uint8_t* core_flags, int32_t* cluster_id,
           void* stream) {
  const int rc = check_call(ctx, points, n, d, eps, min_pts, mode, core_flags, cluster_id);
  if (rc != DBSCAN_OK) return rc;
  if (n == 0) {
    ctx->last_n = 0;
    ctx->last_valid = true;
    return DBSCAN_OK;
  }
  return run_one(ctx, points, n, d, eps, min_pts, mode, core_flags, cluster_id,
                 static_cast<hipStream_t>(stream), resolve(ctx, n, d, mode));
}

int dbscan_approx(dbscan_ctx* ctx, const double* points, int64_t n, int32_t d, double eps,
                  int32_t min_pts, double rho, int32_t mode, uint8_t* core_flags,
                  int32_t* cluster_id, void* stream) {
  const int rc = check_call(ctx, points, n, d, eps, min_pts, mode, core_flags, cluster_id);
  if (rc != DBSCAN_OK) return rc;
  if (!(rho >= 0.0) || !std::isfinite(rho) || !std::isfinite(eps * (1.0 + rho) * eps * (1.0 + rho)))
    return DBSCAN_EINVAL;
  if (n == 0) {
    ctx->last_n = 0;
    ctx->last_valid = true;
    return DBSCAN_OK;
  }
  return run_one(ctx, points, n, d, eps, min_pts, mode, core_flags, cluster_id,
                 static_cast<hipStream_t>(stream), resolve(ctx, n, d, mode), rho);
}

namespace {

// Median of three timed runs of one option set (ms), or a negative error code.
float time_options(dbscan_ctx* ctx, const double* points, int64_t n, int32_t d, double eps,
                   int32_t min_pts, int32_t mode, uint8_t* core, int32_t* label, hipStream_t s,
                   const Resolved& R, hipEvent_t e0, hipEvent_t e1, int* err) {
  float t[3];
  for (int k = 0; k < 3; ++k) {
    if (hipEventRecord(e0, s) != hipSuccess) *err = DBSCAN_EHIP;
    const int rc = run_one(ctx, points, n, d, eps, min_pts, mode, core, label, s, R);
    if (rc != DBSCAN_OK) *err = rc;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
      *err = DBSCAN_EHIP;
    if (*err != DBSCAN_OK) return -1.0f;
    if (hipEventElapsedTime(&t[k], e0, e1) != hipSuccess) *err = DBSCAN_EHIP;
  }
  std::sort(t, t + 3);
  return t[1];
}

}  // namespace

int dbscan_tune(dbscan_ctx* ctx, const double* points, int64_t n, int32_t d, double eps,
                int32_t min_pts, int32_t mode, uint8_t* core_flags, int32_t* cluster_id,
                void* stream, dbscan_tuned* out) {
  int rc = check_call(ctx, points, n, d, eps, min_pts, mode, core_flags, cluster_id);
  if (rc != DBSCAN_OK) return rc;
  if (n == 0) return DBSCAN_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (hipSetDevice(ctx->device) != hipSuccess) return DBSCAN_EHIP;
  const bool prof = ctx->profile;
  ctx->profile = false;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return DBSCAN_EHIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return DBSCAN_EHIP;
  }
  // start from the fixed rules (the tuned table of this class is ignored)
  Resolved best{d > 3 ? 1 : 0, 1, 1, 0, sub_auto(d), kMarkSplit, kDenseGroup};
  int err = DBSCAN_OK;
  // first run pays one-time costs (scratch growth, code loading); not timed
  rc = run_one(ctx, points, n, d, eps, min_pts, mode, core_flags, cluster_id, s, best);
  if (rc != DBSCAN_OK) err = rc;
  int trials = 0;
  float t_best = err == DBSCAN_OK ? time_options(ctx, points, n, d, eps, min_pts, mode, core_flags,
                                                 cluster_id, s, best, e0, e1, &err)
                                  : -1.0f;
  const float t_default = t_best;
  ++trials;
  // coordinate descent over the options, two sweeps; a change must win by 2%
  for (int sweep = 0; sweep < 2 && err == DBSCAN_OK; ++sweep) {
    bool changed = false;
    for (int opt = 0; opt < 7 && err == DBSCAN_OK; ++opt) {
      static const int kVals[7][3] = {{0, 1, -1}, {1, 2, 4},    {0, 2, -1},      {0, 1, 2},
                                      {kSubMinAuto, 512, 0}, {1, 2, 8}, {4, 16, 24}};
      for (int k = 0; k < 3 && err == DBSCAN_OK; ++k) {
        const int v = kVals[opt][k];
        if (v < 0) continue;
        Resolved c = best;
        int* field = opt == 0 ? &c.rounds
                     : opt == 1 ? &c.split
                     : opt == 2 ? &c.fine
                     : opt == 3 ? &c.unit_level
                     : opt == 4 ? &c.sub
                     : opt == 5 ? &c.mark_split
                                : &c.dense;
        if (*field == v) continue;
        if (opt == 3 && !c.rounds) continue;  // the unit level only acts in rounds
        if (opt == 4 && c.fine > 0) continue;  // sub-cell order: only without fine bits
        if (opt >= 5 && d > 3) continue;  // MarkCore's split and the cell-by-cell path: d <= 3
        *field = v;
        const float t = time_options(ctx, points, n, d, eps, min_pts, mode, core_flags, cluster_id,
                                     s, c, e0, e1, &err);
        ++trials;
        if (err == DBSCAN_OK && t < 0.98f * t_best) {
          t_best = t;
          best = c;
          changed = true;
        }
      }
    }
    if (!changed) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ctx->profile = prof;
  if (err != DBSCAN_OK) return err;
  const int lg = size_class(n);
  bool found = false;
  for (TunedEntry& e : ctx->tuned)
    if (e.d == d && e.mode == mode && e.lg == lg) {
      e.r = best;
      e.ms = t_best;
      found = true;
    }
  if (!found) ctx->tuned.push_back(TunedEntry{d, mode, lg, best, t_best});
  ++ctx->tune_gen;
  if (out) {
    out->bcp_rounds = best.rounds;
    out->unit_level = best.unit_level;
    out->bcp_split = best.split;
    out->fine_bits = best.fine;
    out->subcell_min = best.sub;
    out->mark_split = best.mark_split;
    out->dense_group = best.dense;
    out->ms = t_best;
    out->ms_default = t_default;
    out->trials = trials;
    out->size_class = lg;
  }
  return DBSCAN_OK;
}

int dbscan_tune_save(dbscan_ctx* ctx, const char* path) {
  if (!ctx || !path) return DBSCAN_EINVAL;
  FILE* f = std::fopen(path, "w");
  if (!f) return DBSCAN_EINVAL;
  std::fprintf(f, "dbscan-tune 4\n");
  for (const TunedEntry& e : ctx->tuned)
    std::fprintf(f, "%d %d %d %d %d %d %d %d %d %d %.6g\n", e.d, e.mode, e.lg, e.r.rounds,
                 e.r.unit_level, e.r.split, e.r.fine, e.r.sub, e.r.mark_split, e.r.dense,
                 (double)e.ms);
  return std::fclose(f) == 0 ? DBSCAN_OK : DBSCAN_EINVAL;
}

int dbscan_tune_load(dbscan_ctx* ctx, const char* path) {
  if (!ctx || !path) return DBSCAN_EINVAL;
  FILE* f = std::fopen(path, "r");
  if (!f) return DBSCAN_EINVAL;
  int version = 0;
  std::vector<TunedEntry> got;
  // version 1 has no sub-cell threshold, versions 1 and 2 no MarkCore split or
  // cell-by-cell threshold (they read as automatic); up to version 3 the sub-cell
  // threshold of d > 3 was not used (it reads as automatic too); version 4 has the
  // fields of version 3
  int rc = std::fscanf(f, "dbscan-tune %d", &version) == 1 && version >= 1 && version <= 4
               ? DBSCAN_OK
               : DBSCAN_EINVAL;
  while (rc == DBSCAN_OK) {
    TunedEntry e{};
    e.r.sub = kSubMinAuto;
    e.r.mark_split = kMarkSplit;
    e.r.dense = kDenseGroup;
    double ms = 0.0;
    const int want = version == 1 ? 8 : version == 2 ? 9 : 11;
    const int k = version == 1
                      ? std::fscanf(f, "%d %d %d %d %d %d %d %lf", &e.d, &e.mode, &e.lg,
                                    &e.r.rounds, &e.r.unit_level, &e.r.split, &e.r.fine, &ms)
                  : version == 2
                      ? std::fscanf(f, "%d %d %d %d %d %d %d %d %lf", &e.d, &e.mode, &e.lg,
                                    &e.r.rounds, &e.r.unit_level, &e.r.split, &e.r.fine,
                                    &e.r.sub, &ms)
                      : std::fscanf(f, "%d %d %d %d %d %d %d %d %d %d %lf", &e.d, &e.mode,
                                    &e.lg, &e.r.rounds, &e.r.unit_level, &e.r.split, &e.r.fine,
                                    &e.r.sub, &e.r.mark_split, &e.r.dense, &ms);
    if (k == EOF) break;
    if (version == 1 || (version <= 3 && e.d > 3)) e.r.sub = sub_auto(e.d);
    const bool ok = k == want && e.d >= 1 && e.d <= DBSCAN_MAX_D &&
                    (e.mode == DBSCAN_PLAIN_FP64 || e.mode == DBSCAN_FP32_FILTER) &&
                    e.lg >= 0 && e.lg <= 62 && (e.r.rounds == 0 || e.r.rounds == 1) &&
                    e.r.unit_level >= 0 && e.r.unit_level <= kTreeLevels && e.r.split >= 1 &&
                    e.r.split <= 64 && e.r.fine >= 0 && e.r.fine <= 8 && e.r.sub >= 0 &&
                    e.r.sub != 1 && (e.r.mark_split == 1 || e.r.mark_split == 2 ||
                                     e.r.mark_split == 4 || e.r.mark_split == 8) &&
                    e.r.dense >= 1 && e.r.dense <= 64;
    if (!ok) {
      rc = DBSCAN_EINVAL;
      break;
    }
    e.ms = (float)ms;
    got.push_back(e);
  }
  std::fclose(f);
  if (rc != DBSCAN_OK) return rc;  // the table is left as it was
  for (const TunedEntry& g : got) {
    bool found = false;
    for (TunedEntry& e : ctx->tuned)
      if (e.d == g.d && e.mode == g.mode && e.lg == g.lg) {
        e = g;
        found = true;
      }
    if (!found) ctx->tuned.push_back(g);
  }
  ++ctx->tune_gen;
  return DBSCAN_OK;
}

int dbscan_tune_clear(dbscan_ctx* ctx) {
  if (!ctx) return DBSCAN_EINVAL;
  ctx->tuned.clear();
  ++ctx->tune_gen;
  return DBSCAN_OK;
}


int dbscan_membership(dbscan_ctx* ctx, int64_t* offsets, int32_t* ids, int64_t ids_cap,
                      int64_t* total, void* stream) {
  if (!ctx || !offsets || !total || ids_cap < 0) return DBSCAN_EINVAL;
  if (!ctx->last_valid) return DBSCAN_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (hipSetDevice(ctx->device) != hipSuccess) return DBSCAN_EHIP;
  const int64_t n = ctx->last_n;
  if (n == 0) {
    *total = 0;
    if (hipMemsetAsync(offsets, 0, sizeof(int64_t), s) != hipSuccess) return DBSCAN_EHIP;
    return hipStreamSynchronize(s) == hipSuccess ? DBSCAN_OK : DBSCAN_EHIP;
  }
  const Work& W = ctx->last_work;
  // the sort buffers are free once the cells are built
  int64_t* count = reinterpret_cast<int64_t*>(W.keyA);
  int64_t* tiles = reinterpret_cast<int64_t*>(W.keyB);
  uint32_t* overflow = W.tilectr + 15;
  if (hipMemsetAsync(overflow, 0, sizeof(uint32_t), s) != hipSuccess) return DBSCAN_EHIP;
  member_dispatch(ctx->last_d, W, s, 0, count, nullptr, nullptr, overflow);
  const int64_t ntiles = ceil_div(n, kScanTile);
  k_scan_tiles<<<(unsigned)ntiles, kBlock, 0, s>>>(count, n, tiles);
  k_scan_top<<<1, kBlock, 0, s>>>(tiles, ntiles);
  k_scan_apply<<<(unsigned)ntiles, kBlock, 0, s>>>(count, n, tiles, offsets);
  uint32_t ovf = 0;
  if (hipMemcpyAsync(total, offsets + n, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(&ovf, overflow, sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return DBSCAN_EHIP;
  if (ovf) return DBSCAN_EINTERNAL;
  if (!ids) return hipGetLastError() == hipSuccess ? DBSCAN_OK : DBSCAN_EHIP;
  if (ids_cap < *total) return DBSCAN_EINVAL;
  member_dispatch(ctx->last_d, W, s, 1, count, offsets, ids, overflow);
  if (hipStreamSynchronize(s) != hipSuccess) return DBSCAN_EHIP;
  return hipGetLastError() == hipSuccess ? DBSCAN_OK : DBSCAN_EHIP;
}

int dbscan_batch(dbscan_ctx* ctx, const dbscan_instance* inst, int32_t count, int32_t mode,
                 void* stream) {
  if (!ctx || count < 0 || (count > 0 && !inst)) return DBSCAN_EINVAL;
  ctx->last_valid = false;
  if (mode != DBSCAN_PLAIN_FP64 && mode != DBSCAN_FP32_FILTER) return DBSCAN_EINVAL;
  int64_t nmax = 0;
  int32_t dmax = 1;
  for (int32_t i = 0; i < count; ++i) {
    const dbscan_instance& I = inst[i];
    if (I.n_settings < 1 || !I.eps || !I.min_pts) return DBSCAN_EINVAL;
    for (int32_t a = 0; a < I.n_settings; ++a) {
      const int rc = check_args(I.n, I.d, I.eps[a], I.min_pts[a]);
      if (rc != DBSCAN_OK) return rc;
    }
    if (I.n > 0 && (!I.points || !I.core_flags || !I.cluster_id)) return DBSCAN_EINVAL;
    nmax = std::max(nmax, I.n);
    dmax = std::max(dmax, I.d);
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return DBSCAN_EHIP;
  const int slots = batch_slots(inst, count);
  const bool keep_keys = plan_keeps_keys(ctx, inst, count);
  BatchPlan plan = plan_batch(ctx, inst, count, mode, slots, keep_keys);
  (void)nmax;
  (void)dmax;
  int rc = grow(ctx, plan.nmax, plan.dmax, slots, keep_keys, plan.area_bytes);
  if (rc != DBSCAN_OK) return rc;
  ctx->last_n = 0;
  for (int32_t i = 0; i < count; ++i) ctx->last_n += inst[i].n * inst[i].n_settings;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool f32 = mode == DBSCAN_FP32_FILTER;
  reset_marks(ctx);
  // profiled batches run eagerly, with an event at every phase boundary
  if (ctx->profile || !ctx->batch_graph) {
    rc = prepare_groups(ctx, plan, inst, mode, s);
    if (rc != DBSCAN_OK) return rc;
    return enqueue_batch(ctx, inst, count, f32, s, Marks{ctx->profile ? ctx : nullptr, s}, slots,
                         keep_keys, plan);
  }

  std::vector<unsigned char> key = batch_key(ctx, inst, count, mode);
  if (!ctx->graph || key != ctx->graph_key) {
    drop_graph(ctx);
    // the group tables are written before capture, on the stream the graph runs on
    rc = prepare_groups(ctx, plan, inst, mode, s);
    if (rc != DBSCAN_OK) return rc;
    if (!ctx->cap_stream &&
        hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess)
      return DBSCAN_EHIP;
    if (hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return DBSCAN_EHIP;
    rc = enqueue_batch(ctx, inst, count, f32, ctx->cap_stream, Marks{nullptr, ctx->cap_stream},
                       slots, keep_keys, plan);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(ctx->cap_stream, &g);
    if (rc != DBSCAN_OK || e != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      return rc != DBSCAN_OK ? rc : DBSCAN_EHIP;
    }
    const hipError_t ie = hipGraphInstantiate(&ctx->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
      ctx->graph = nullptr;
      return DBSCAN_EHIP;
    }
    ctx->graph_key.swap(key);
  }
  return hipGraphLaunch(ctx->graph, s) == hipSuccess ? DBSCAN_OK : DBSCAN_EHIP;
}

int dbscan_get_stats(dbscan_ctx* ctx, void* stream, dbscan_stats* out) {
  if (!ctx || !out) return DBSCAN_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return DBSCAN_EHIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (ctx->stats_valid && ctx->last_n > 0) k_core_total<<<1, kBlock, 0, st>>>(ctx->stats_work);
  if (hipStreamSynchronize(st) != hipSuccess) return DBSCAN_EHIP;
  GridDesc g;
  if (hipMemcpy(&g, ctx->desc, sizeof(g), hipMemcpyDeviceToHost) != hipSuccess) return DBSCAN_EHIP;
  std::memset(out, 0, sizeof(*out));
  out->n_points = ctx->last_n;
  out->n_cells = g.n_cells;
  out->n_unsafe = g.n_unsafe;
  int64_t sum[5] = {0, 0, 0, 0, 0};
  for (int w = 0; w < 5; ++w)
    for (int i = 0; i < kCtrSlots; ++i) sum[w] += (int64_t)g.ctr[w][i];
  out->n_core = sum[kCtrCore];
  out->bcp_calls = sum[kCtrBcp];
  out->uf_links = sum[kCtrLinks];
  out->fp64_rechecks = sum[kCtrRechecks];
  out->pair_tests = sum[kCtrPairs];
  out->key_bits = g.total_bits;
  out->key_shift = g.shift;
  out->status = g.status;
  out->filter_tin = g.tin;
  out->filter_tout = g.tout;
  if (g.status & DBSCAN_STATUS_NONFINITE) return DBSCAN_ENONFINITE;
  if (g.status & DBSCAN_STATUS_WAIT_EXPIRED) return DBSCAN_EINTERNAL;
  return DBSCAN_OK;
}

int dbscan_set_option(dbscan_ctx* ctx, int32_t option, int64_t value) {
  if (!ctx) return DBSCAN_EINVAL;
  switch (option) {
    case DBSCAN_OPT_BCP_ROUNDS:
      if (value < -1 || value > 1) return DBSCAN_EINVAL;
      ctx->bcp_rounds = (int)value;
      return DBSCAN_OK;
    case DBSCAN_OPT_UNIT_LEVEL:
      if (value < -1 || value > kTreeLevels) return DBSCAN_EINVAL;
      ctx->unit_level = (int)value;
      return DBSCAN_OK;
    case DBSCAN_OPT_FINE_BITS:
      if (value < -1 || value > 8) return DBSCAN_EINVAL;
      ctx->fine_bits = (int)value;
      return DBSCAN_OK;
    case DBSCAN_OPT_FORCE_RECHECK:
      if (value != 0 && value != 1) return DBSCAN_EINVAL;
      ctx->force_recheck = (int)value;
      return DBSCAN_OK;
    case DBSCAN_OPT_BATCH_GRAPH:
      if (value != 0 && value != 1) return DBSCAN_EINVAL;
      ctx->batch_graph = (int)value;
      return DBSCAN_OK;
    case DBSCAN_OPT_BCP_SPLIT:
      if (value < -1 || value == 0 || value > 64) return DBSCAN_EINVAL;
      ctx->bcp_split = (int)value;
      return DBSCAN_OK;
    case DBSCAN_OPT_FILTER_MAX_D:
      if (value < -1 || value > DBSCAN_MAX_D) return DBSCAN_EINVAL;
      ctx->filter_max_d = (int)value;
      return DBSCAN_OK;
    case DBSCAN_OPT_SUBCELL_MIN:
      if (value < -1 || value == 1 || value > kIntMax) return DBSCAN_EINVAL;
      ctx->subcell_min = (int)value;
      return DBSCAN_OK;
    case DBSCAN_OPT_SPARSE:
      if (value < -1 || value > 1) return DBSCAN_EINVAL;
      ctx->sparse = (int)value;
      return DBSCAN_OK;
    case DBSCAN_OPT_GROUP_CLOUDS:
      if (value < -1 || value > 1) return DBSCAN_EINVAL;
      ctx->group_clouds = (int)value;
      return DBSCAN_OK;
    case DBSCAN_OPT_MARK_SPLIT:
      if (value != -1 && value != 1 && value != 2 && value != 4 && value != 8) return DBSCAN_EINVAL;
      ctx->mark_split = (int)value;
      return DBSCAN_OK;
    case DBSCAN_OPT_DENSE_GROUP:
      if (value != -1 && (value < 1 || value > 64)) return DBSCAN_EINVAL;
      ctx->dense_group = (int)value;
      return DBSCAN_OK;
    case DBSCAN_OPT_CELLS:
      if (value < -1 || value > 1) return DBSCAN_EINVAL;
      ctx->cells = value == 1 ? 1 : 0;
      return DBSCAN_OK;
  }
  return DBSCAN_EINVAL;
}

int dbscan_get_option(dbscan_ctx* ctx, int32_t option, int64_t* value) {
  if (!ctx || !value) return DBSCAN_EINVAL;
  switch (option) {
    case DBSCAN_OPT_BCP_ROUNDS: *value = ctx->bcp_rounds; return DBSCAN_OK;
    case DBSCAN_OPT_UNIT_LEVEL: *value = ctx->unit_level; return DBSCAN_OK;
    case DBSCAN_OPT_FINE_BITS: *value = ctx->fine_bits; return DBSCAN_OK;
    case DBSCAN_OPT_FORCE_RECHECK: *value = ctx->force_recheck; return DBSCAN_OK;
    case DBSCAN_OPT_BATCH_GRAPH: *value = ctx->batch_graph; return DBSCAN_OK;
    case DBSCAN_OPT_BCP_SPLIT: *value = ctx->bcp_split; return DBSCAN_OK;
    case DBSCAN_OPT_FILTER_MAX_D: *value = ctx->filter_max_d; return DBSCAN_OK;
    case DBSCAN_OPT_SUBCELL_MIN: *value = ctx->subcell_min; return DBSCAN_OK;
    case DBSCAN_OPT_SPARSE: *value = ctx->sparse; return DBSCAN_OK;
    case DBSCAN_OPT_GROUP_CLOUDS: *value = ctx->group_clouds; return DBSCAN_OK;
    case DBSCAN_OPT_MARK_SPLIT: *value = ctx->mark_split; return DBSCAN_OK;
    case DBSCAN_OPT_DENSE_GROUP: *value = ctx->dense_group; return DBSCAN_OK;
    case DBSCAN_OPT_CELLS: *value = ctx->cells; return DBSCAN_OK;
  }
  return DBSCAN_EINVAL;
}

int dbscan_set_profiling(dbscan_ctx* ctx, int on) {
  if (!ctx) return DBSCAN_EINVAL;
  ctx->profile = on != 0;
  return DBSCAN_OK;
}

int dbscan_phase_times(dbscan_ctx* ctx, void* stream, float* ms, int32_t cap) {
  return dbscan_phase_stats(ctx, stream, ms, nullptr, cap);
}

int dbscan_phase_stats(dbscan_ctx* ctx, void* stream, float* ms, int32_t* occurrences,
                       int32_t cap) {
  if (!ctx || !ms || cap < 0) return DBSCAN_EINVAL;
  if (!ctx->events_recorded) return DBSCAN_EINVAL;
  if (ctx->ev_error) return DBSCAN_EHIP;
  if (hipSetDevice(ctx->device) != hipSuccess) return DBSCAN_EHIP;
  if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return DBSCAN_EHIP;
  float sum[DBSCAN_NUM_PHASES] = {};
  int32_t occ[DBSCAN_NUM_PHASES] = {};
  for (size_t k = 1; k < ctx->ev_mark.size(); ++k) {
    const int ph = ctx->ev_mark[k] - 1;  // the phase this boundary ends
    if (ph < 0 || ph >= DBSCAN_NUM_PHASES) continue;
    float t = 0.0f;
    if (hipEventElapsedTime(&t, ctx->ev_pool[k - 1], ctx->ev_pool[k]) != hipSuccess)
      return DBSCAN_EHIP;
    sum[ph] += t;
    ++occ[ph];
  }
  for (int i = 0; i < DBSCAN_NUM_PHASES && i < cap; ++i) {
    ms[i] = sum[i];
    if (occurrences) occurrences[i] = occ[i];
  }
  return DBSCAN_NUM_PHASES;
}

const char* dbscan_phase_name(int32_t phase) {
  return phase >= 0 && phase < DBSCAN_NUM_PHASES ? kPhaseNames[phase] : "";
}

const char* dbscan_strerror(int code) {
  switch (code) {
    case DBSCAN_OK: return "ok";
    case DBSCAN_EINVAL: return "invalid argument";
    case DBSCAN_ENOMEM: return "device scratch allocation failed";
    case DBSCAN_EHIP: return "HIP runtime error";
    case DBSCAN_ENONFINITE: return "non-finite coordinate";
    case DBSCAN_EINTERNAL: return "internal bounded wait expired";
    case DBSCAN_ETOOLARGE: return "input exceeds the allocation-free scratch";
  }
  return "unknown error";
}

}  // extern "C"
