/*
 * sj.h -- C ABI of libsj, an MI355X (gfx950) implementation of the per-tick
 * spatial join of moving-object positions against rectangular range queries
 * described in Lettich, Orlando, Silvestri, Jensen, "Manycore processing of
 * repeated range queries over massive moving objects observations".
 *
 * Problem (Section "Problem setting and statement"): objects o_0..o_{N-1}
 * send position updates and issue range queries; time is cut into ticks and
 * at the end of each tick every query issued during the tick is answered on
 * the last known positions of all objects (Definition 1: an object is in the
 * result of a query iff its point lies in the closed query rectangle).
 *
 * Method (Sections "Index Creation and Indexing in QUAD", "Filtering",
 * "Bitmap decoding", "Optimizations"): the space is partitioned by a
 * point-region quadtree whose leaves hold at most th objects; each query is
 * split into one subquery per leaf it touches, classified covering (the
 * leaf lies inside the query: its objects are reported without tests) or
 * intersecting (its objects are tested); results are produced lock-free by a
 * count pass, an exclusive scan and a write pass.
 *
 * Conventions
 *  - Every pointer named d_* is a device pointer (HBM of the GPU the scene
 *    was created on); everything else is host memory.
 *  - All calls are asynchronous on the scene's stream unless stated; input
 *    buffers must stay valid and unmodified until the stream has passed the
 *    call.  Calls on one scene must not overlap; distinct scenes are
 *    independent (and may share a stream).
 *  - The library allocates no device memory: the caller provides one device
 *    workspace of sj_workspace_bytes(cfg) bytes (256-byte aligned) at
 *    creation and owns it; the scene borrows it until sj_scene_destroy.
 *  - Return values: SJ_OK (0) or a negative SJ_E* code.  Errors found on the
 *    device (bad ids or coordinates, capacity overflow) are latched in the
 *    scene and returned by the next call that synchronises
 *    (sj_fetch_results, sj_stats); sj_last_error gives a message.
 */
#ifndef SJ_H
#define SJ_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sj_scene sj_scene;

enum sj_status {
  SJ_OK = 0,
  SJ_EINVAL = -1,    /* bad argument: null/misaligned pointer, size above the
                        configured capacity, object id >= capacity_objects */
  SJ_ENOSPACE = -2,  /* workspace smaller than sj_workspace_bytes(cfg) */
  SJ_EOVERFLOW = -3, /* a tick produced more subqueries, covering entries or
                        result ids than configured; nothing partial was
                        reported for that tick; grow the capacities and run
                        the tick again (run_tick does not change positions) */
  SJ_EDATA = -4,     /* non-finite coordinate, or a query with x^a > x^b or
                        y^a > y^b; such entries are ignored */
  SJ_EDEVICE = -5,   /* a HIP runtime call failed */
  SJ_ESTATE = -6     /* call out of order (e.g. fetch before any run_tick) */
};

/* Configuration flags (sj_config.flags). */
enum sj_flags {
  SJ_COVERING = 1u << 0, /* covering-subquery optimisation (Section
                            "Optimizations"); off = every subquery is tested;
                            results are identical either way */
  SJ_REORDER = 1u << 1,  /* task scheduling optimisation: leaves processed
                            heaviest first, weight = intersecting subqueries x
                            objects (Section "Optimizations") */
  SJ_PROFILE = 1u << 2,  /* record per-phase device times (sj_phase_times) */
  SJ_TIMING_LOG = 1u << 3, /* per-leaf join timing log (sj_timing_log) */
  SJ_THRESH_MLP = 1u << 4, /* builds pick their threshold with the cost
                              model installed by sj_set_cost_model */
  SJ_SCHEDULE_MLP = 1u << 5, /* with SJ_REORDER and a cost model installed:
                              join tasks run in the order of the model's
                              predicted task time instead of the weight
                              |Q_I^c| x |P^c| (learned schedule) */
  SJ_UNIFORM_GRID = 1u << 6, /* the UG method's index instead of the
                              quadtree (Definition "MBR partitioning into a
                              uniform grid"): the frame cut into grid_split
                              columns and rows along its finest cells, cells
                              numbered by Morton code, materialised on every
                              tick; same query split and join.  Not with
                              SJ_THRESH_MLP, SJ_SCHEDULE_MLP or
                              SJ_TIMING_LOG. */
  SJ_ATOMIC_RESULTS = 1u << 7, /* the paper's baseline filter (UG_Baseline,
                              Algorithm SQB) in place of the lock-free count,
                              scan and write: intersecting results are
                              appended as (query, object) pairs through an
                              LDS buffer and a global atomic counter, in no
                              particular order (sj_results.d_pairs).  An
                              ablation; results are the same sets. */
  SJ_CU_COUNTERS = 1u << 8   /* containment tests per compute unit of the
                              filtering pass (sj_cu_counters; the S3
                              imbalance study) */
};

/* Quadtree reuse across ticks (the paper builds the partitioning on the
 * first tick and builds it again when the distribution changes
 * significantly). */
enum sj_rebuild {
  SJ_REBUILD_AUTO = 0,   /* rebuild on the first tick, after sj_build_index,
                            every rebuild_period ticks, and on the tick after
                            one where a leaf below l_max held more than 2*th
                            objects or more than 1% of the objects lay
                            outside the index frame */
  SJ_REBUILD_ALWAYS = 1, /* rebuild on every tick */
  SJ_REBUILD_NEVER = 2,  /* rebuild only on the first tick and after
                            sj_build_index */
  SJ_REBUILD_COST = 3    /* rebuild when keeping the quadtree has cost as
                            much as a rebuild (rent or buy): after a build,
                            each kept tick adds its device time above the
                            fastest kept tick since the build, and the tick
                            after the sum reaches the build tick's own
                            excess over that fastest tick rebuilds.  Within
                            twice the least total excess for excesses that
                            grow as objects drift.  Also on the first tick
                            and after sj_build_index. */
};

typedef struct sj_config {
  uint32_t capacity_objects;    /* N: object ids are 0..N-1 */
  uint32_t capacity_queries;    /* largest nq of one sj_run_tick */
  uint64_t capacity_subqueries; /* intersecting subqueries per tick
                                   (0: 32 * capacity_queries) */
  uint64_t capacity_covering;   /* covering subqueries per tick
                                   (0: 32 * capacity_queries) */
  uint64_t capacity_results;    /* result ids of intersecting subqueries per
                                   tick (0: 64 * capacity_queries) */
  uint32_t th_quad;             /* leaf split threshold: a quadrant with more
                                   than th_quad objects is split (0: 64) */
  uint32_t th_min;              /* smallest threshold the scene will be built
                                   with; sizes the leaf table (0: th_quad) */
  uint32_t l_max;               /* deepest quadtree level, 1..16 (0: 16) */
  uint32_t flags;               /* sj_flags (SJ_COVERING | SJ_REORDER is the
                                   paper's configuration) */
  uint32_t rebuild_policy;      /* sj_rebuild */
  uint32_t rebuild_period;      /* SJ_REBUILD_AUTO period in ticks (0: 32) */
  uint32_t split_slots;         /* subqueries per query remembered between the
                                   count and write passes of query splitting;
                                   queries with more are walked twice (0: 32) */
  uint32_t tune_every;          /* SJ_THRESH_MLP: host-decided builds between
                                   two tunings; the first build is tuned (0: 8) */
  uint32_t grid_split;          /* SJ_UNIFORM_GRID: columns (= rows) of the
                                   grid, the paper's split factor, 1..4096 */
} sj_config;

/* Compressed results of the last tick (Sections "Bitmap decoding" and
 * "Optimizations").  The result of query k (input order of the tick) is a
 * list of runs of object ids, reached through the query's processing
 * position p = d_query_pos[k] (the tick processes large batches in a
 * spatial order; p = k otherwise):
 *   intersecting part, one run per intersecting subquery (the decoded
 *     bitmap of the query against one leaf): for every slot s in
 *     [d_isect_slot_off[p], d_isect_slot_off[p+1]), run r = d_slot_run[s]
 *     is d_isect_id[d_run_off[r] .. d_run_off[r+1]);
 *   covering part: for every c in [d_cov_off[p], d_cov_off[p+1]), leaf
 *     L = d_cov_leaf[c] contributes all objects
 *     d_sorted_id[d_leaf_beg[L] .. d_leaf_beg[L+1]).
 * Runs are stored in the join's order (the runs of one leaf's subqueries
 * side by side), not by query.  Order inside a query is unspecified
 * (intersecting runs in the order of the query's split, then covering
 * leaves in that order; ids inside a run in d_sorted_id order); lists of
 * distinct leaves are disjoint, so the result set is their concatenation
 * (sj_expand_results gives per-query lists, with SJ_SORTED in the canonical
 * ascending order).  A query superseded by a later query of the same object
 * in the tick, or one rejected as invalid, has an empty result.  Pointers
 * are device views into the workspace, valid until the next call on the
 * scene. */
typedef struct sj_results {
  uint32_t nq;
  uint32_t n_leaves;
  uint64_t n_isect_ids;       /* = d_run_off[n_runs] */
  uint64_t n_cov_entries;     /* = d_cov_off[nq] */
  uint64_t total_pairs;       /* sum over queries of |res(q)| */
  uint64_t n_runs;            /* intersecting subqueries = d_isect_slot_off[nq] */
  const uint32_t *d_query_pos; /* [nq] processing position of query k */
  const uint32_t *d_isect_slot_off; /* [nq + 1], by processing position */
  const uint32_t *d_slot_run;  /* [n_runs] */
  const uint64_t *d_run_off;   /* [n_runs + 1] */
  const uint32_t *d_isect_id;  /* [n_isect_ids] */
  const uint32_t *d_cov_off;   /* [nq + 1], by processing position */
  const uint32_t *d_cov_leaf;
  const uint32_t *d_leaf_beg;  /* [n_leaves + 1] */
  const uint32_t *d_sorted_id; /* [n_present] object ids grouped by leaf,
                                  leaves in Morton order (leaf L's objects
                                  are d_leaf_beg[L] .. d_leaf_beg[L+1]) */
  /* Counters of the tick, from the same read-back (0 for the result
   * counts when the tick's results overflowed): */
  uint32_t n_present;         /* objects with a position (= d_leaf_beg[n_leaves]) */
  uint32_t n_tasks;           /* leaves with at least one intersecting subquery */
  uint64_t n_subqueries;      /* intersecting subqueries on leaves with objects */
  uint64_t cov_pairs;         /* result pairs given by covering leaves */
  uint64_t tests;             /* containment tests of the filtering */
  uint32_t error_bits;        /* SJ_ERR_* bits of the tick */
  uint32_t reserved;
  /* SJ_ATOMIC_RESULTS: the intersecting results are these pairs instead of
   * runs (n_runs is 0): d_pairs[2 i] = query index k, d_pairs[2 i + 1] =
   * object id, for i < n_pairs, in no particular order. */
  uint64_t n_pairs;
  const uint32_t *d_pairs;
} sj_results;

/* Counters of the last tick (read back by sj_stats, which synchronises). */
typedef struct sj_tick_stats {
  uint32_t n_present;     /* objects with a position */
  uint32_t n_leaves;      /* quadtree leaves (including empty ones) */
  uint32_t n_nodes;       /* internal quadtree nodes */
  uint32_t l_deep;        /* deepest level holding a leaf */
  uint32_t th;            /* threshold of the current quadtree */
  uint32_t rebuilt;       /* 1 if the quadtree was built on this tick */
  uint32_t n_tasks;       /* leaves with at least one intersecting subquery */
  uint32_t max_leaf;      /* largest object count of a leaf above l_max */
  uint64_t n_isect;       /* intersecting subqueries */
  uint64_t n_cov;         /* covering subqueries */
  uint64_t n_isect_ids;   /* result ids written by the join */
  uint64_t cov_pairs;     /* pairs reported through covering leaves */
  uint64_t tests;         /* containment tests: sum over leaves of
                             |intersecting subqueries| * |objects| */
  uint32_t error_bits;    /* latched device error flags of this tick */
  uint32_t tick;          /* ticks run so far */
  uint32_t knn_fallback;  /* after sj_run_knn: queries answered by the
                             fallback scan over every object */
  uint32_t reserved;
} sj_tick_stats;

/* Phases timed when SJ_PROFILE is set (device time in milliseconds of the
 * last tick, from events on the scene's stream). */
enum sj_phase {
  SJ_PH_UPDATES = 0, /* sj_apply_updates since the previous tick */
  SJ_PH_INDEX,       /* MBR, Morton codes, radix sort, gather */
  SJ_PH_BUILD,       /* quadtree construction (0 on ticks that reuse it) */
  SJ_PH_LEAVES,      /* object ranges of the leaves */
  SJ_PH_SPLIT,       /* query splitting: count, scans, write */
  SJ_PH_SCHEDULE,    /* task list (and heaviest-first order) */
  SJ_PH_JOIN_COUNT,  /* join count pass */
  SJ_PH_JOIN_SCAN,   /* result offsets */
  SJ_PH_JOIN_WRITE,  /* join write pass */
  SJ_PH_COUNT
};

/* Bytes of device workspace needed by a scene with this configuration. */
size_t sj_workspace_bytes(const sj_config *cfg);

/* Creates a scene on the current HIP device.  d_workspace: caller-owned
 * device buffer of at least sj_workspace_bytes(cfg) bytes, 256-byte aligned.
 * stream: stream all work of the scene is ordered on.  Initialises the
 * workspace (asynchronously); no object has a position yet. */
int sj_scene_create(const sj_config *cfg, void *d_workspace, size_t ws_bytes,
                    hipStream_t stream, sj_scene **out);

/* Releases host-side state (events); the workspace is the caller's. */
int sj_scene_destroy(sj_scene *scene);

/* Position updates (tick batching): m updates (d_id[k], d_x[k], d_y[k]);
 * within the tick the last update of an object wins (later call, then later
 * index).  An object never updated has no position and is in no result.
 * Updates with id >= capacity_objects (SJ_EINVAL) or a non-finite
 * coordinate (SJ_EDATA) are ignored and latched. */
int sj_apply_updates(sj_scene *scene, const uint32_t *d_id, const float *d_x,
                     const float *d_y, uint32_t m);

/* Marks the quadtree for construction on the next sj_run_tick with split
 * threshold th (0: keep the current one); th must be >= th_min.  Results
 * do not depend on the threshold. */
int sj_build_index(sj_scene *scene, uint32_t th);

/* Closes the tick and answers nq range queries (timeslice semantics: on the
 * positions after every earlier sj_apply_updates).  Query k is issued by
 * object d_qid[k]; its rectangle has lower-left corner (d_xa[k], d_ya[k])
 * and upper-right corner (d_xb[k], d_yb[k]) and may extend beyond the
 * objects' MBR.  If an object issues several queries in one tick the last
 * one is answered.  nq <= capacity_queries. */
int sj_run_tick(sj_scene *scene, const uint32_t *d_qid, const float *d_xa,
                const float *d_ya, const float *d_xb, const float *d_yb,
                uint32_t nq);

/* One tick as a single HIP graph launch: the same work and results as
 * sj_apply_updates(d_id, d_x, d_y, m) followed by sj_run_tick(...), on the
 * scene's stream.  The graph is captured on first use for each quadtree
 * decision (keep, build, decided on the device) and replayed afterwards;
 * it is captured again when m or nq differs from the captured sizes.  The
 * graph reads the input arrays through a small block in the workspace that
 * one kernel launched before it writes, so any buffers replay the same
 * graph without copies.  The graph holds kernels only.  If updates were already
 * enqueued for this tick by sj_apply_updates, the tick runs eagerly. */
int sj_tick_graph(sj_scene *scene, const uint32_t *d_id, const float *d_x, const float *d_y,
                  uint32_t m, const uint32_t *d_qid, const float *d_xa, const float *d_ya,
                  const float *d_xb, const float *d_yb, uint32_t nq);

/* Synchronises the stream and returns views of the compressed results of
 * the last tick, or the latched error of the tick. */
int sj_fetch_results(sj_scene *scene, sj_results *out);

/* Expanded results (Section "Bitmap decoding": the per-query lists the
 * paper's decoding produces, with the covering leaves of Section
 * "Optimizations" expanded): per-query CSR of the last tick.
 *   d_sel == NULL: every query of the tick, in input order (n_sel ignored).
 *   d_sel != NULL: the n_sel query indices d_sel[0 .. n_sel) (device, each
 *     < nq; repeats allowed; n_sel <= capacity_queries), in that order.
 * List i is d_ids[d_off[i] .. d_off[i+1]) (d_off: n + 1 u64, device).  Ids
 * in a list are unordered unless flags has SJ_SORTED (ascending ids, the
 * canonical order).  Two-call protocol: with d_ids == NULL only *n_pairs is
 * set (the number of ids to provide room for; with a selection d_off is
 * written too).  Otherwise the lists are written if ids_cap suffices, else
 * SJ_EINVAL.  SJ_EINVAL also for an index >= nq, a misaligned pointer, or
 * unknown flags.  Synchronises. */
#define SJ_SORTED 1u
int sj_expand_results(sj_scene *scene, const uint32_t *d_sel, uint32_t n_sel, uint32_t flags,
                      uint64_t *d_off, uint32_t *d_ids, uint64_t ids_cap, uint64_t *n_pairs);

/* Per-query result size and order-independent pair-set hash
 * H(q) = sum over id in res(q) of mix64((qid << 32) | id) mod 2^64, mix64
 * being the SplitMix64 output function; written to d_count[nq],
 * d_hash[nq].  Asynchronous. */
int sj_result_hashes(sj_scene *scene, uint64_t *d_count, uint64_t *d_hash);

/* Asynchronously copies counters of the last tick to d_out[8] (device
 * memory, u64): [0] total pairs, [1] result ids of intersecting subqueries,
 * [2] pairs reported through covering leaves, [3] intersecting subqueries,
 * [4] covering subqueries, [5] containment tests, [6] tasks (leaves joined),
 * [7] latched error bits.  Lets a caller collect per-tick totals without
 * synchronising. */
int sj_tick_counters(sj_scene *scene, uint64_t *d_out);

/* SJ_CU_COUNTERS: containment tests of the last tick's filtering pass per
 * compute-unit slot, copied to out[0 .. n) (host memory, n <= 4096).  Slot
 * = XCC id << 8 | shader engine << 5 | shader array << 4 | CU id, from the
 * waves' hardware id registers; unused slots stay 0.  Synchronises.  The
 * paper's SM imbalance (Experimental evaluation, S3) is the relative
 * difference between the largest and the smallest count of the CUs. */
int sj_cu_counters(sj_scene *scene, uint64_t *out, uint32_t n);

/* Counters of the last tick; synchronises; returns the latched error. */
int sj_stats(sj_scene *scene, sj_tick_stats *out);

/* Learned threshold (not in the paper, which fixes th_quad after a sweep,
 * Experimental evaluation S5; the terms of the cost follow the
 * Computational Complexity section).  With SJ_THRESH_MLP and a model
 * installed, a tick that builds the quadtree on the host's decision (the
 * host decides when a call that synchronises, such as sj_fetch_results or
 * sj_stats, has read the scene's state after the previous tick), the first
 * such build and then every tune_every-th, first builds and splits at every
 * candidate threshold (on the first tuning; later tunings try the
 * candidates within a factor of two of the current threshold), predicts
 *   cost = coef[0] * sum over active leaves c of exp(MLP(f_c))
 *        + coef[1] |Q_I| + coef[2] |Q_C| + coef[3] * leaves
 *        + coef[4] * max over active leaves c of exp(MLP(f'_c))
 *        + coef[5] * P(leaves) * objects
 * with f_c = (log2(1 + |P^c|), log2(1 + |Q_I^c|), level / 16, mean over the
 * intersecting subqueries of c of the fraction of c's area they cover), f'_c
 * = f_c with |Q_I^c| capped at 64 (a join task takes at most 64 subqueries
 * of a leaf), and
 * builds the cheapest (the first of equal costs; a candidate that overflows
 * a capacity is infeasible; with none feasible the threshold is kept).
 * P(L) = ceil(bit length of (L - 1) / 8), the radix passes of the
 * leaf-keyed sort of the ticks that keep the quadtree.  The sum is the
 * join's work and the maximum its critical path, since one wave runs a
 * join task.
 * Results do not depend on it.
 * d_w: sj_mlp_param_count() BF16 parameters (device, copied); cand: n_cand
 * (1..8) ascending thresholds, each >= th_min.  Synchronises the scene's
 * stream.  Errors: SJ_EINVAL (null pointers, bad n_cand, candidates not
 * ascending or below th_min). */
#define SJ_COST_TERMS 6
int sj_set_cost_model(sj_scene *scene, const uint16_t *d_w, const float coef[SJ_COST_TERMS],
                      const uint32_t *cand, uint32_t n_cand);

typedef struct sj_tune_info {
  uint32_t n_cand;
  uint32_t cand[8];
  float cost[8];        /* predicted cost per candidate (inf: infeasible) */
  float mlp_sum[8];     /* sum over active leaves of exp(MLP) */
  float mlp_max[8];     /* largest exp(MLP) of an active leaf */
  uint32_t chosen;      /* threshold of the last tuning */
  uint32_t n_tunes;     /* tunings so far */
  uint32_t tuned_tick;  /* ticks completed before the last tuning */
} sj_tune_info;

/* Outcome of the last tuning; synchronises. */
int sj_tune_info_get(sj_scene *scene, sj_tune_info *out);

/* Per-leaf timing log of the last tick (SJ_TIMING_LOG): for every leaf,
 * 8 floats: objects, intersecting subqueries, level, mean overlap area
 * fraction of its intersecting subqueries with the leaf, device-clock ticks
 * of the wave that joined it in the count pass and in the write pass, 0, 0.
 * clock_mhz converts ticks to microseconds.  Device view valid until the
 * next call; synchronises. */
typedef struct sj_timing_view {
  uint32_t n_leaves;
  float clock_mhz;
  const float *d_records; /* [n_leaves][8] */
} sj_timing_view;

int sj_timing_log(sj_scene *scene, sj_timing_view *out);

/* Device times of the phases of the last tick (SJ_PROFILE), n <=
 * SJ_PH_COUNT floats.  Synchronises.  After a graph tick (sj_tick_graph)
 * only SJ_PH_JOIN_WRITE is timed (the pass runs as a graph of its own
 * between two events); the other entries are 0. */
int sj_phase_times(sj_scene *scene, float *ms, int n);

/* Largest k of a k-nearest-neighbour query. */
#define SJ_KNN_MAX 64u

/* Closes the tick like sj_run_tick and answers nq k-nearest-neighbour
 * queries instead of range queries (the paper leaves repeated kNN queries
 * over moving objects to future work, Section "Conclusions", proposing to
 * reuse its pipeline; this is that reuse).  Query i, issued by object
 * d_qid[i] at point (d_qx[i], d_qy[i]), asks for the k present objects of
 * smallest key (d2, id), where d2 = fl32(fl32(dx*dx) + fl32(dy*dy)),
 * dx = fl32(px - qx), dy = fl32(py - qy), each operation rounded to
 * binary32 on its own; ties go to the smaller id.  Output (device,
 * caller-owned, row-major nq x k): d_out_id[i*k + j], d_out_d2[i*k + j] is
 * the (j+1)-th nearest; slots past the present objects hold id 0xffffffff
 * and d2 = +inf; a query superseded by a later query of the same object in
 * the tick, or one at a non-finite point (SJ_EDATA), gets only such slots.
 * How: a candidate square per query from the quadtree (the k-th distance
 * to the objects of the point's leaf, or the farthest corner of the
 * smallest enclosing quadrant holding k objects), the tick's query split
 * and join on those squares, then a per-query selection; a query whose
 * square cannot be proved to hold its k nearest is answered by a scan over
 * every object (counted in sj_tick_stats.knn_fallback).  sj_fetch_results
 * afterwards returns the squares' range results.  1 <= k <= SJ_KNN_MAX,
 * nq <= capacity_queries; not with SJ_UNIFORM_GRID or SJ_ATOMIC_RESULTS
 * (SJ_EINVAL).  Synchronises: returns after the outputs are written, with
 * the tick's status (SJ_EOVERFLOW: outputs not written; grow the
 * capacities). */
int sj_run_knn(sj_scene *scene, const uint32_t *d_qid, const float *d_qx, const float *d_qy,
               uint32_t nq, uint32_t k, uint32_t *d_out_id, float *d_out_d2);

/* Internal arrays for tests and tools (device views, valid until the next
 * call): sorted Morton codes and ids of present objects, leaf table in
 * Morton order (start code at the finest level, level), and the current
 * frame. */
typedef struct sj_index_view {
  uint32_t n_present, n_leaves, l_deep;
  float x0, y0;
  int32_t e;                 /* frame side is 2^e */
  const uint32_t *d_codes;   /* [n_present] sort keys: level-16 Morton codes
                                after a tick that built the quadtree, leaf
                                indices after one that kept it */
  const uint32_t *d_ids;     /* [n_present] */
  const uint32_t *d_leaf_start; /* [n_leaves] */
  const uint32_t *d_leaf_level; /* [n_leaves] */
  const uint32_t *d_leaf_beg;   /* [n_leaves + 1] */
  const float *d_pos;           /* [capacity_objects][2]: (x, y) by id (NaN: no
                                   position) */
} sj_index_view;

int sj_index_view_get(sj_scene *scene, sj_index_view *out);

/* ------------------------------------------------------------------------
 * Tick serving: many scenes on one device with continuous batching (the
 * batching of ticks and the latency definitions of Section "Problem
 * setting and statement": latency = queueing + processing).
 *
 * The server carves every resident scene's workspace and output slots
 * from one caller-owned device pool with its own first-fit
 * allocator: admission succeeds while the scene fits (an HBM budget), and
 * retiring or evicting a scene returns its memory.  Every scene has its own
 * stream.  Tick requests queue per scene in submission order;
 * sj_server_poll retires finished ticks and starts queued ones, up to
 * max_running at once, so ticks of different scenes overlap on the device.
 * A tick replays the scene's captured graph (sj_tick_graph) on the
 * request's own input arrays, then writes per-query counts and pair-set
 * hashes (sj_result_hashes) and the tick counters (sj_tick_counters) into
 * the scene's output slots.
 *
 * Eviction: a scene's results depend only on the last-known positions of
 * its objects (Definition 1), so an idle scene can leave the device as a
 * host copy of its positions (with its configuration and current leaf
 * threshold) and come back later with the same results.  Scenes added with
 * sj_server_add are admitted on demand when a request of theirs comes up,
 * and evicted when idle (least recently used first) to make room for
 * another; sj_server_evict evicts any idle scene explicitly.  A re-admitted
 * scene builds a new quadtree on its next tick and forgets a cost model set
 * on it (its tuned threshold is kept).  Not thread-safe.
 * ------------------------------------------------------------------------ */
typedef struct sj_server sj_server;

typedef struct sj_served {
  uint64_t tag;                 /* the submission's tag */
  uint32_t scene_id;
  int32_t status;               /* SJ_OK or the tick's error */
  uint32_t nq;
  const uint64_t *d_count;      /* [nq] result sizes        (SJ_SERVE_DIGEST, else */
  const uint64_t *d_hash;       /* [nq] pair-set hashes      NULL; valid until the
                                   scene's next tick */
  const uint64_t *d_counters;   /* [8] as sj_tick_counters   after this one is */
} sj_served;                    /*                           retired by a poll) */

typedef struct sj_server_stats {
  uint64_t pool_bytes, pool_used;
  uint32_t scenes;      /* registered scenes (resident or evicted) */
  uint32_t running, queued;
  uint32_t resident;    /* scenes holding pool memory */
  uint32_t admissions;  /* scenes made resident so far (re-admissions included) */
  uint32_t evictions;   /* scenes moved to host memory so far */
} sj_server_stats;

/* Device bytes a scene takes from the pool (workspace + output slots). */
size_t sj_server_scene_bytes(const sj_config *cfg, uint32_t max_updates);

/* d_pool: caller-owned device memory, 256-byte aligned, pool_bytes long.
 * max_running: ticks in flight at once (0: 4). */
int sj_server_create(void *d_pool, size_t pool_bytes, uint32_t max_running, sj_server **out);
int sj_server_destroy(sj_server *server);

/* Admits a scene if sj_server_scene_bytes(cfg, max_updates) fit in the pool
 * now; SJ_ENOSPACE otherwise (nothing is reserved; try again later). */
int sj_server_admit(sj_server *server, const sj_config *cfg, uint32_t max_updates,
                    uint32_t *scene_id);

/* Registers a scene that is made resident when its first request comes up
 * (evicting idle scenes added this way if the pool is full) and may be
 * evicted when idle.  SJ_ENOSPACE if it is larger than the whole pool. */
int sj_server_add(sj_server *server, const sj_config *cfg, uint32_t max_updates,
                  uint32_t *scene_id);

/* Moves a resident scene with no tick running to host memory (pinned; its
 * positions, configuration and current threshold) and returns its pool
 * memory; synchronises its stream.  Its queued requests stay queued and
 * bring it back.  The result views of its last tick (sj_served, the scene
 * object) become invalid.  SJ_ESTATE if it is not resident or runs a tick. */
int sj_server_evict(sj_server *server, uint32_t scene_id);

/* Releases an idle scene (no tick queued or running) and its memory. */
int sj_server_retire(sj_server *server, uint32_t scene_id);

/* Queues a tick for a scene: device inputs as sj_apply_updates + sj_run_tick
 * (4-byte aligned; the tick reads them in place, so they must stay valid and
 * unmodified until it is retired); tags must be unique per
 * scene.  d_record (device, 10 u64, may be NULL) receives the tick's record
 * when it finishes: the 8 counters of sj_tick_counters, then (with
 * SJ_SERVE_DIGEST, else 0, 0) the sum of the per-query pair-set hashes and
 * the sum of the result sizes (mod 2^64).  SJ_SERVE_DIGEST also makes the
 * per-query counts and hashes of sj_served available; it reads every result,
 * so it is for checking, not for serving.  Non-blocking. */
#define SJ_SERVE_DIGEST 1u
int sj_server_submit(sj_server *server, uint32_t scene_id, const uint32_t *d_id,
                     const float *d_x, const float *d_y, uint32_t m, const uint32_t *d_qid,
                     const float *d_xa, const float *d_ya, const float *d_xb,
                     const float *d_yb, uint32_t nq, uint64_t tag, uint64_t *d_record,
                     uint32_t flags);

/* Retires finished ticks (at most cap, written to done[0 .. *n_done)) and
 * starts queued ticks in submission order, admitting scenes that are not
 * resident (and evicting idle scenes added with sj_server_add, least
 * recently used first, but none whose tick this call retired).  The outputs
 * of a retired tick of such a scene stay valid until the next poll.
 * Non-blocking. */
int sj_server_poll(sj_server *server, sj_served *done, uint32_t cap, uint32_t *n_done);

int sj_server_info(const sj_server *server, sj_server_stats *out);

/* The scene object of a resident scene (results of its last retired tick
 * stay readable until its next tick starts or it is evicted). */
int sj_server_scene(sj_server *server, uint32_t scene_id, sj_scene **out);

const char *sj_server_last_error(const sj_server *server);

/* ------------------------------------------------------------------------
 * Cost model: an MLP 4 -> 64 -> 64 -> 1 with ReLU that predicts the join
 * time of a quadtree leaf (natural log of microseconds).  Inputs per leaf
 * (float[4]): log2(1 + objects), log2(1 + intersecting subqueries),
 * level / 16, mean overlap area fraction of its intersecting subqueries.
 * Parameters: sj_mlp_param_count() values, layout W1[64][4], b1[64],
 * W2[64][64], b2[64], w3[64], b3; used as BF16 (round to nearest even of
 * FP32 masters), arithmetic in FP32.  Not part of the paper: it chooses the
 * split threshold (the paper's th_quad, fixed there) for the quadtree.
 * All pointers are device pointers; calls are asynchronous on `stream`.
 * ------------------------------------------------------------------------ */
uint32_t sj_mlp_param_count(void);

/* d_w[i] = BF16 rounding of d_master[i]. */
int sj_mlp_round(const float *d_master, uint16_t *d_w, hipStream_t stream);

/* d_y[s] = MLP(d_x[4 s .. 4 s + 3]) for s < n. */
int sj_mlp_forward(const uint16_t *d_w, const float *d_x, uint32_t n, float *d_y,
                   hipStream_t stream);

/* Gradient of L = (1/n) sum_s (MLP(x_s) - t_s)^2 with respect to the BF16
 * parameters: d_grad[0 .. P) (P = sj_mlp_param_count()), and d_grad[P] = L.
 * d_scratch: sj_mlp_scratch_bytes(n) bytes.  Deterministic. */
size_t sj_mlp_scratch_bytes(uint32_t n);
int sj_mlp_grad(const uint16_t *d_w, const float *d_x, const float *d_t, uint32_t n,
                float *d_grad, void *d_scratch, size_t scratch_bytes, hipStream_t stream);

/* sj_mlp_grad without a caller-provided scratch buffer, for callers that
 * cannot allocate device memory (code under graph capture, serving loops
 * that refine the model between ticks, harnesses that forbid hipMalloc).
 * The per-block partial gradients live in a fixed array inside the library
 * (sj_mlp_noalloc_scratch_bytes() = 4,655,104 bytes per GPU, held until the
 * process ends); its size does not depend on n, so no n is refused for it.
 * Same kernels and result as sj_mlp_grad, bit for bit.  The call allocates
 * nothing (on its first call on a GPU it looks up the array's address on
 * that GPU).  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (on different streams, or from different threads
 * without ordering) race and give wrong gradients; serialise them. */
size_t sj_mlp_noalloc_scratch_bytes(void);
int sj_mlp_grad_noalloc(const uint16_t *d_w, const float *d_x, const float *d_t, uint32_t n,
                        float *d_grad, hipStream_t stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, step >= 1)
 * on the FP32 masters with moments d_m, d_v; writes the BF16 copy d_w. */
int sj_mlp_adam(float *d_master, const float *d_grad, float *d_m, float *d_v, uint16_t *d_w,
                uint32_t step, float lr, hipStream_t stream);

/* Message for the last error of the scene; with NULL, of the last failed
 * scene creation or call that takes no scene (server creation, sj_mlp_*). */
const char *sj_last_error(const sj_scene *scene);

#ifdef __cplusplus
}
#endif

#endif /* SJ_H */
