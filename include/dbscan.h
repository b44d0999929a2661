/*
 * Exact Euclidean DBSCAN on one AMD Instinct MI355X (gfx950): C ABI.
 *
 * The operation is the DBSCAN problem of Wang, Gu and Shun, "Theoretically-Efficient
 * and Practical Parallel DBSCAN" (SIGMOD 2020), section "Preliminaries", computed by
 * the grid method of the paper's Algorithm 1: cells of side eps/sqrt(d) (section
 * "Grid Computation"), MarkCore (Algorithm 2), ClusterCore with bichromatic-closest-
 * pair cell connectivity and a lock-free union-find (Algorithm 3 and section
 * "Cluster Core"), and ClusterBorder (Algorithm 4).
 *
 * Output contract (exact; identical on every call for the same input):
 *   - core_flags[i] = 1 iff at least min_pts points p_j (p_i included) satisfy
 *     D(p_i, p_j) <= E2, else 0;
 *   - cluster_id[i] for a core point = the smallest index of a core point in its
 *     cluster; for a non-core point = the smallest cluster id among core points
 *     within eps (the paper lets such a point belong to several clusters), or -1
 *     (noise) when there is none;
 *   where D(p, q) = (((0 + t_0*t_0) + t_1*t_1) + ...), t_k = p_k - q_k, every step a
 *   float64 operation rounded to nearest-even, summed in dimension order with no
 *   fused multiply-add, and E2 = eps*eps rounded once.  No square root is taken.
 *
 * Pointers named "device" must be device memory of the context's GPU (for example
 * from hipMalloc or a PyTorch CUDA tensor).  The caller owns every input and output
 * buffer; the library keeps no reference to them after the stream work of the call.
 * Calls are asynchronous on `stream` (a hipStream_t; NULL = the default stream).
 * A context must not be used by two host threads at once, and two calls on one
 * context must not run concurrently on different streams (they share scratch).
 *
 * Return codes: 0 on success, otherwise one of DBSCAN_E*.  Argument errors are
 * reported synchronously.  Data-dependent errors (non-finite coordinates) are
 * detected on the GPU; dbscan_get_stats() returns them after synchronising the
 * stream.  Outputs are undefined when an error occurs.  Any finite input is
 * accepted: when the cell grid would need more than 64 Morton key bits the key is
 * coarsened by a power of two (key_shift) and the float64 diameter guard splits
 * the resulting large cells, so the result is unchanged (only slower).
 */
#ifndef PAPER_1912_06255_DBSCAN_H
#define PAPER_1912_06255_DBSCAN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DBSCAN_OK 0
#define DBSCAN_EINVAL (-1)     /* bad argument: n<0, d not in [1,8], eps not finite or <= 0,
                                  min_pts < 1, NULL pointer with n > 0, n > DBSCAN_MAX_N */
#define DBSCAN_ENOMEM (-2)     /* device scratch could not be allocated */
#define DBSCAN_EHIP (-3)       /* a HIP runtime call failed */
#define DBSCAN_ENONFINITE (-4) /* a coordinate is NaN or infinite */
#define DBSCAN_EINTERNAL (-5)  /* an internal bounded wait expired (should not happen) */
#define DBSCAN_ETOOLARGE (-6)  /* dbscan_noalloc: the call needs more than its fixed scratch */

#define DBSCAN_MAX_N 1073741823LL /* 2^30 - 1 points per call */
#define DBSCAN_MAX_D 8

/* Distance arithmetic of the pairwise decisions.  Both modes return identical
 * outputs: DBSCAN_FP32_FILTER decides most pairs from float32 cell-local
 * coordinates with a proven error band and re-decides in float64 the pairs whose
 * float32 result falls inside the band (by default for d <= 3 only; see
 * DBSCAN_OPT_FILTER_MAX_D). */
#define DBSCAN_PLAIN_FP64 0
#define DBSCAN_FP32_FILTER 1

typedef struct dbscan_ctx dbscan_ctx;

/* Counters of the last completed call on a context. */
typedef struct {
  int64_t n_points;      /* n of the call */
  int64_t n_cells;       /* non-empty cells after splitting unsafe ones */
  int64_t n_unsafe;      /* grid cells whose float64 diameter test failed (split) */
  int64_t n_core;        /* core points */
  int64_t bcp_calls;     /* cell pairs that reached a closest-pair test */
  int64_t uf_links;      /* successful union-find links */
  int64_t fp64_rechecks; /* pairs re-decided in float64 (FP32 filter mode) */
  int64_t pair_tests;    /* point-pair distance decisions made by ClusterCore */
  int32_t key_bits;      /* bits of the Morton cell key */
  int32_t key_shift;     /* key coordinate = floor(cell index / 2^key_shift) */
  uint32_t status;       /* 0 or a bit set of DBSCAN_STATUS_* */
  uint32_t reserved;
  float filter_tin;      /* float32 filter thresholds of the last grid built in */
  float filter_tout;     /* DBSCAN_FP32_FILTER mode: IN if D32 <= tin, OUT if > tout */
} dbscan_stats;

#define DBSCAN_STATUS_NONFINITE 1u
#define DBSCAN_STATUS_WAIT_EXPIRED 4u

/* Create a context bound to HIP device `device`.  *out receives the handle. */
int dbscan_ctx_create(dbscan_ctx **out, int device);

/* Free a context and its device scratch.  Synchronises the device first. */
int dbscan_ctx_destroy(dbscan_ctx *ctx);

/*
 * Exact DBSCAN of one point cloud (paper, Algorithm 1).
 *   points      device, float64 [n][d] row-major (point i at points + i*d)
 *   n, d        number of points (0 allowed) and dimension (1..8)
 *   eps         radius, finite and > 0
 *   min_pts     density threshold >= 1 (the point itself counts)
 *   mode        DBSCAN_PLAIN_FP64 or DBSCAN_FP32_FILTER
 *   core_flags  device, uint8 [n] output
 *   cluster_id  device, int32 [n] output
 *   stream      hipStream_t or NULL
 * Scratch grows inside the context on demand (a synchronous allocation the first
 * time a larger n is seen); dbscan_reserve() does it ahead of time.
 */
int dbscan(dbscan_ctx *ctx, const double *points, int64_t n, int32_t d, double eps,
           int32_t min_pts, int32_t mode, uint8_t *core_flags, int32_t *cluster_id,
           void *stream);

/*
 * Approximate DBSCAN (paper, section "Preliminaries": Gan and Tao's relaxation;
 * section "Approximate DBSCAN"): as dbscan(), except that two core points whose
 * distance lies in (eps, eps(1 + rho)] may or may not end up in one cluster.
 * Core flags are exact; core points within eps always share a cluster; a pair of
 * core cells is joined only through a pair of core points within eps(1 + rho),
 * decided as the float64 test D <= fl(R^2), R = fl(eps * fl(1 + rho)); cluster
 * ids are the smallest core input index of each cluster and non-core points take
 * the smallest id among clusters with a core point within eps (-1: none), as in
 * dbscan().  The output need not be unique: any output of this definition is
 * correct.  rho = 0 gives dbscan()'s result.
 *   rho         relaxation >= 0 and finite (eps (1 + rho) squared finite)
 *   (other arguments as for dbscan())
 * Returns DBSCAN_EINVAL for a bad rho, else as dbscan().
 */
int dbscan_approx(dbscan_ctx *ctx, const double *points, int64_t n, int32_t d, double eps,
                  int32_t min_pts, double rho, int32_t mode, uint8_t *core_flags,
                  int32_t *cluster_id, void *stream);

/*
 * A batch: many point clouds, each with one or more (eps, minPts) settings
 * (paper, Algorithm 1 run once per cloud and setting).  Results are identical to
 * one dbscan() call per (cloud, setting).
 *   points       device, float64 [n][d] row-major
 *   n, d         as for dbscan() (n = 0 allowed)
 *   n_settings   >= 1
 *   eps, min_pts HOST arrays [n_settings]
 *   core_flags   device, uint8 [n_settings][n]: setting s at core_flags + s*n
 *   cluster_id   device, int32 [n_settings][n]
 */
typedef struct {
  const double *points;
  int64_t n;
  int32_t d;
  int32_t n_settings;
  const double *eps;
  const int32_t *min_pts;
  uint8_t *core_flags;
  int32_t *cluster_id;
} dbscan_instance;

/*
 * Run a batch on `stream`.  Settings of one cloud with the same eps share its
 * grid, cell tree and one MarkCore neighbour count (taken up to the largest
 * minPts of that eps).  With DBSCAN_OPT_BATCH_GRAPH on (the default) the whole
 * batch is captured into one HIP graph the first time a batch description
 * (pointers, sizes, settings, mode, options) is seen and replayed as a single
 * graph launch on later identical calls; the first call also instantiates the
 * graph.  Scratch is sized for the largest cloud.  Counters read afterwards with
 * dbscan_get_stats() cover the whole batch (bcp_calls, uf_links, fp64_rechecks,
 * status) or its last cloud and setting (cells, core points).
 */
int dbscan_batch(dbscan_ctx *ctx, const dbscan_instance *inst, int32_t count, int32_t mode,
                 void *stream);

/* Pre-size the context's scratch for clouds of up to n points of dimension d. */
int dbscan_reserve(dbscan_ctx *ctx, int64_t n, int32_t d);

/*
 * Synchronise `stream` and copy the counters and status of the last call into
 * *out.  Returns DBSCAN_ENONFINITE / DBSCAN_EINTERNAL when the call hit that
 * condition, else DBSCAN_OK.
 */
int dbscan_get_stats(dbscan_ctx *ctx, void *stream, dbscan_stats *out);

/*
 * Phase timing.  With profiling on, each call records HIP events on its stream
 * between its phases (grid box, keys, radix sort, cell runs, cell boxes and
 * guard, box tree, MarkCore counts, core flags, ClusterCore, relabel,
 * ClusterBorder, output scatter, and ClusterCore of a setting started from the
 * union-find of the previous one, timed apart); a profiled dbscan_batch() runs
 * eagerly (no graph) and records the
 * same boundaries for every cloud and setting.  dbscan_phase_times()
 * synchronises `stream` and writes up to `cap` per-phase durations in
 * milliseconds of the last call, each summed over every occurrence of the phase
 * in that call (a batch repeats the setting phases once per setting and the grid
 * phases once per cloud and eps); it returns the number of phases
 * (DBSCAN_NUM_PHASES) or a negative error code.  dbscan_phase_stats() does the
 * same and also writes the number of occurrences of each phase to
 * `occurrences` (may be NULL).
 */
#define DBSCAN_NUM_PHASES 13
int dbscan_set_profiling(dbscan_ctx *ctx, int on);
int dbscan_phase_times(dbscan_ctx *ctx, void *stream, float *ms, int32_t cap);
int dbscan_phase_stats(dbscan_ctx *ctx, void *stream, float *ms, int32_t *occurrences,
                       int32_t cap);
const char *dbscan_phase_name(int32_t phase);

/*
 * Tuning options of a context (they change speed, never results).
 *   DBSCAN_OPT_BCP_ROUNDS  0: one pass tests every neighbour cell pair;
 *                          1: rounds over the levels of the cell tree, each
 *                             pruning subtrees already joined;
 *                          -1: automatic (one pass for d <= 3, rounds above;
 *                             the default)
 *   DBSCAN_OPT_UNIT_LEVEL  in rounds, tree nodes up to this level whose core
 *                          cells already form one component are tested as one
 *                          unit (0..5; -1: automatic = 1, the default)
 *   DBSCAN_OPT_FINE_BITS   sub-cell Morton bits per dimension appended to the
 *                          sort key, ordering the points inside every cell
 *                          (-1: automatic = 0, else 0..8)
 *   DBSCAN_OPT_SUBCELL_MIN with DBSCAN_OPT_FINE_BITS at 0 bits, cells of at
 *                          least this many points are put into
 *                          sub-cell order after the grid is built, the leaves
 *                          of the paper's per-cell quadtree (section "Range
 *                          Counting"): MarkCore and ClusterCore then skip or
 *                          count whole 64-point chunks by their boxes
 *                          (2..2^31-1; 0: never; -1: automatic = 2048, the
 *                          default)
 *   DBSCAN_OPT_FORCE_RECHECK  1: the float32 filter sends every pair to the
 *                          float64 recheck (for testing; default 0)
 *   DBSCAN_OPT_BATCH_GRAPH 1: dbscan_batch() captures and replays a HIP graph
 *                          (default); 0: it launches its kernels directly
 *   DBSCAN_OPT_BCP_SPLIT   most waves per ClusterCore unit: the unit's points
 *                          are cut into up to this many segments of at least
 *                          192 points and of at least the mean cell size, one
 *                          wave each (1..64; -1: automatic = 1, the default)
 *   DBSCAN_OPT_FILTER_MAX_D  DBSCAN_FP32_FILTER calls take their pair decisions
 *                          through the float32 filter only for d up to this
 *                          value; above it they decide in float64 directly
 *                          (0..8; -1: automatic = 3, the default).  Results
 *                          are the same either way.
 *   DBSCAN_OPT_SPARSE      MarkCore, ClusterCore and ClusterBorder with the
 *                          points of 64 consecutive sorted positions batched per
 *                          tree walk, instead of one wave and one walk per cell.
 *                          1: always; 0 or -1 (automatic, the default): never
 *                          (the batched kernels measured slower on every grid
 *                          tried).  Results are the same either way.
 *   DBSCAN_OPT_GROUP_CLOUDS  dbscan_batch() only: instances with a single setting
 *                          and the same dimension (and options) form a group
 *                          whose grids share every kernel launch, each grid
 *                          keeping its own arrays (the batch's scratch grows by
 *                          the sum of their sizes).  -1 (automatic, the
 *                          default): groups of at least two instances, in more
 *                          than 3 dimensions only of instances of at most 2^17
 *                          points; 1: every such instance, alone or not, of any
 *                          size; 0: never (one chain of launches per instance).
 *                          Results are the same either way.
 *   DBSCAN_OPT_MARK_SPLIT  MarkCore waves per cell (their candidate chunks dealt out
 *                          among them), up to 3 dimensions in grids of at least
 *                          32 points per cell on average: 1, 2, 4 or 8 (-1:
 *                          automatic = 4).
 *   DBSCAN_OPT_DENSE_GROUP ClusterCore (up to 3 dimensions) takes a 64-cell group
 *                          of neighbours cell by cell, refreshing roots before each,
 *                          when it holds at least this many points per live cell:
 *                          1..64 (-1: automatic = 8).
 *   DBSCAN_OPT_CELLS       how the cells are built in 2 dimensions: 0 (default,
 *                          also -1) grid cells of side eps / sqrt(d); 1 the box
 *                          method (section "Box Computation"): points sorted by
 *                          x and cut into strips of width at most eps / sqrt(2),
 *                          each strip sorted by y and cut into boxes the same
 *                          way, both cuts by binary search and pointer jumping.
 *                          The result does not change (it is the unique DBSCAN
 *                          result); other dimensions ignore the option, and a
 *                          batch builds such grids one at a time (no grouping,
 *                          no grid cut from a finer eps).
 * dbscan_set_option() returns DBSCAN_EINVAL for an unknown option or value.
 */
#define DBSCAN_OPT_BCP_ROUNDS 1
#define DBSCAN_OPT_UNIT_LEVEL 2
#define DBSCAN_OPT_FINE_BITS 3
#define DBSCAN_OPT_FORCE_RECHECK 4
#define DBSCAN_OPT_BATCH_GRAPH 5
#define DBSCAN_OPT_BCP_SPLIT 6
#define DBSCAN_OPT_FILTER_MAX_D 7
#define DBSCAN_OPT_SUBCELL_MIN 8
#define DBSCAN_OPT_SPARSE 9
#define DBSCAN_OPT_GROUP_CLOUDS 10
#define DBSCAN_OPT_MARK_SPLIT 11
#define DBSCAN_OPT_DENSE_GROUP 12
#define DBSCAN_OPT_CELLS 13
int dbscan_set_option(dbscan_ctx *ctx, int32_t option, int64_t value);
int dbscan_get_option(dbscan_ctx *ctx, int32_t option, int64_t *value);

/*
 * Autotuner over the tuning options (one pass or rounds, the unit level,
 * waves per unit, sub-cell order bits, the sub-cell threshold among 2048, 512
 * and none and, for d <= 3, MarkCore's waves per cell among 1, 2, 4 and 8, and
 * ClusterCore's cell-by-cell threshold among 4, 8, 16 and 24).  dbscan_tune() runs the given
 * instance with the default options and then changes one option at a time
 * (two sweeps of coordinate descent; a change must be 2% faster), timing each
 * candidate as the median of three runs with HIP events on `stream`.  The best
 * set is stored in the context for the instance's class (d, mode and
 * n in [2^k, 2^(k+1))), and later dbscan() / dbscan_batch() calls of that
 * class use it for every option left automatic (-1); options set explicitly
 * with dbscan_set_option() still win.  Results never depend on the options, so
 * core_flags / cluster_id hold the instance's exact result afterwards.  The
 * call synchronises with `stream`.  Returns DBSCAN_EINVAL for n == 0 or bad
 * arguments (as dbscan()), or the first error of a run.
 *
 * dbscan_tune_save() writes the table as text ("dbscan-tune 4", then one line
 * "d mode k rounds unit_level split fine_bits subcell_min mark_split
 * dense_group ms" per class); dbscan_tune_load() merges such a file into the
 * table (also the earlier versions: 1 lacks subcell_min, 1 and 2 lack
 * mark_split and dense_group, and up to 3 the subcell_min of d > 3 was unused;
 * all of these read as automatic; a malformed file leaves the table unchanged
 * and returns DBSCAN_EINVAL); dbscan_tune_clear() empties it.  None of the
 * three touches the GPU.
 */
typedef struct dbscan_tuned {
  int32_t bcp_rounds, unit_level, bcp_split, fine_bits; /* the chosen options */
  int32_t subcell_min; /* chosen sub-cell threshold (0: none; as DBSCAN_OPT_SUBCELL_MIN) */
  float ms;         /* median time of one call with them */
  float ms_default; /* the same with the default options */
  int32_t trials;   /* option sets timed */
  int32_t size_class; /* k: the class holds n in [2^k, 2^(k+1)) */
  int32_t mark_split, dense_group; /* as DBSCAN_OPT_MARK_SPLIT / _DENSE_GROUP */
} dbscan_tuned;
int dbscan_tune(dbscan_ctx *ctx, const double *points, int64_t n, int32_t d,
                double eps, int32_t min_pts, int32_t mode, uint8_t *core_flags,
                int32_t *cluster_id, void *stream, dbscan_tuned *out);
int dbscan_tune_save(dbscan_ctx *ctx, const char *path);
int dbscan_tune_load(dbscan_ctx *ctx, const char *path);
int dbscan_tune_clear(dbscan_ctx *ctx);

/*
 * Full cluster membership of the last dbscan() call on this context (paper,
 * section "Preliminaries": a border point belongs to every cluster that has a
 * core point within eps; Algorithm 4 before its reduction to one id).  For every
 * point, in input order: a core point has exactly its cluster id, a border point
 * every distinct cluster id within eps, noise none; ids ascending.
 *
 *   offsets  device int64[n + 1], written: CSR offsets (offsets[0] = 0)
 *   ids      device int32[ids_cap] or NULL; when not NULL, the ids are written
 *            at ids[offsets[i] .. offsets[i+1])
 *   total    host: receives offsets[n]
 *
 * Call once with ids == NULL to learn *total, then with ids_cap >= *total.
 * Uses the state the call left in the context (sorted points, core flags, cell
 * labels, box tree), so it must follow that dbscan() before any other call on the
 * context other than dbscan_get_stats / dbscan_membership; after dbscan_batch()
 * (or before any call) it returns DBSCAN_EINVAL, as it does for ids_cap < *total.
 * Every decision is the float64 test, whatever the mode of the call.  Returns
 * DBSCAN_EINTERNAL if a point is within eps of more than 256 distinct clusters
 * (impossible for d <= 8: core points of different clusters are more than eps
 * apart, so at most 240 fit within eps of one point).  Synchronises with stream.
 */
int dbscan_membership(dbscan_ctx *ctx, int64_t *offsets, int32_t *ids, int64_t ids_cap,
                      int64_t *total, void *stream);

/*
 * Allocation-free variant of dbscan(), for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same computation and outputs as dbscan() with the default
 * options; no context is involved and no device memory is allocated or freed
 * by the call (it calls no hipMalloc, hipFree or allocating routine).
 *
 * Its scratch is one file-scope device array of DBSCAN_NOALLOC_SCRATCH_BYTES
 * (64 MiB) per GPU, held by each GPU the library runs on until the process
 * ends.  The call runs on the calling thread's current device; its first call
 * on a device looks up the array's address there.  Every call on a GPU shares
 * that GPU's array and leaves its contents behind, so calls that overlap on one
 * GPU (other streams or threads) race and must not be issued; consecutive calls
 * on one stream are fine.
 *   points, n, d, eps, min_pts, mode, core_flags, cluster_id, stream
 *                as for dbscan()
 *   status       device uint32 or NULL: receives the call's DBSCAN_STATUS_*
 *                bits (0 = fine; DBSCAN_STATUS_NONFINITE = a coordinate is NaN
 *                or infinite, outputs undefined) when the stream reaches the
 *                end of the call
 * Limit: the call's scratch, about (80 + 38 d) bytes per point plus a few KiB,
 * must fit the array: n up to 569,088 points in 1D, 348,992 in 3D and 177,432
 * in 8D.  Larger inputs return DBSCAN_ETOOLARGE before any work is queued.
 * Argument errors return DBSCAN_EINVAL as for dbscan().
 */
#define DBSCAN_NOALLOC_SCRATCH_BYTES (64u << 20)
int dbscan_noalloc(const double *points, int64_t n, int32_t d, double eps, int32_t min_pts,
                   int32_t mode, uint8_t *core_flags, int32_t *cluster_id, uint32_t *status,
                   void *stream);

/* Static description of a return code. */
const char *dbscan_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* PAPER_1912_06255_DBSCAN_H */
