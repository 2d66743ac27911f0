// Device buffers of a scene and the host launchers of the tick pipeline.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sj_host.h"

namespace sj {

struct Ctl;
struct TuneState;

constexpr unsigned kJoinBlocks = 4096;  // 16384 waves for the join passes

// Typed views of the caller's workspace (carved by sj_api.hip).
struct Bufs {
  Ctl *ctl;
  TickIn *tin;                          // input arrays of the current tick
  // objects (by id) and per-tick sorted arrays
  float2 *pos;                          // position by id (NaN x: no position)
  uint64_t *ustamp, *qstamp;
  uint32_t *keyA, *valA, *keyB, *valB;  // sorted (code, id) end in A
  float2 *sxy;                          // positions in sorted order
  float2 *sxy2;                         // the sort's other buffer of positions
  uint32_t *blk;                        // per-block present counts/offsets
  uint64_t *red;                        // per-block partials (kRedSlots)
  uint64_t *part;                       // scan partials (kMaxScanJobs)
  uint32_t *hist, *tot;                 // radix sort histograms
  // quadtree
  uint4 *front[2];
  uint32_t *lstart, *llevel, *lstart2, *llevel2;
  uint32_t *nopen, *node_off;
  uint4 *nodes;
  uint32_t *table;                      // start table (4^tcap entries)
  uint32_t *leaf_beg, *leaf_sqoff;
  // schedule
  uint32_t *tkey;                       // order key of every join task (TCAP)
  uint32_t *qkey, *qord, *qkey2, *qord2;  // spatial processing order of the queries (Q)
  uint32_t *tkhist;                     // 256 task-key totals, 256 placement cursors
  uint2 *vtask;                         // further chunks of heavy leaves: (leaf, chunk)
  uint32_t *xbase;                      // per leaf: task index of its second chunk
  uint4 *trec;                          // tasks in run order: subquery and object ranges
  uint32_t *tleaf;                      // tasks in run order: leaf
  // queries and subqueries
  float4 *qrect;                        // rectangles in processing order
  uint32_t *q_ni, *q_nc, *q_ioff, *q_coff;  // per query in processing order
  uint32_t *qpos;                       // processing position of query k
  uint32_t *qlist;                      // visited leaves per query (slots each)
  uint32_t *sq;                         // subqueries grouped by leaf: index of the rectangle
  uint32_t *slot_sq;                    // per intersecting slot (query order): its subquery
  uint32_t *sq_cnt;                     // result ids per subquery (subquery order)
  uint64_t *res_off;                    // their scan: subquery i's run of result ids
  uint32_t *cov_leaf, *res_ids;
  float *tlog;                          // per-leaf timing log (or null)
  uint2 *pairs;                         // appended (query, object) pairs of the baseline
                                        // filter (or null: lock-free join)
  uint64_t *cu_tests;                   // containment tests per CU slot (or null)
  float *kq_rect;                       // kNN candidate squares: xa, ya, xb, yb arrays of Q
                                        // (or null: the scene takes no kNN queries)
  uint32_t *kq_fb;                      // kNN queries left to the fallback scan (Q)
  TuneState *tune;                      // threshold tuner state
  // capacities
  uint32_t N, Q, LCAP, NCAP, FCAP, slots, tcap, TCAP;
  uint64_t S, C, R;
};

// ug_split: columns of the uniform-grid index (0: quadtree), ug_bits its
// cells' bits per axis.
void launch_ctl_init(Ctl *ctl, uint32_t th, uint32_t ug_split, uint32_t ug_bits, uint32_t policy,
                     hipStream_t s);
void launch_request_build(Ctl *ctl, uint32_t th, hipStream_t s);
void launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s);
void launch_fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s);
// Writes the input arrays of a (parts 1: updates, 2: queries) into B.tin,
// where the kernels of the following launches read them.
void launch_tick_in(const Bufs &B, const TickIn &a, uint32_t parts, hipStream_t s);
void launch_updates(const Bufs &B, uint32_t m, uint64_t seq_off, hipStream_t s);
// key_bits: with decision 0, the width of the leaf keys if the host knows
// it (then exactly the passes it needs run), else 0.
void launch_index(const Bufs &B, uint32_t decision, uint32_t policy, uint64_t upd_total,
                  uint32_t nq, uint32_t key_bits, hipStream_t s);
void launch_build(const Bufs &B, uint32_t l_max, hipStream_t s);
void launch_leaves(const Bufs &B, hipStream_t s);
// Returns the processing order of the queries (rank -> query index) when the
// batch is ordered spatially, else null (the identity).
const uint32_t *launch_split(const Bufs &B, uint32_t nq, uint32_t covering, hipStream_t s);
void launch_schedule(const Bufs &B, uint32_t reorder, uint32_t l_max, bool learned,
                     hipStream_t s);
// Task keys from the cost model's predicted task times (learned schedule).
void launch_schedule_mlp(const Bufs &B, hipStream_t s);
void launch_join_count(const Bufs &B, hipStream_t s);
void launch_join_scan(const Bufs &B, uint64_t cap_res, uint32_t policy, uint32_t period,
                      hipStream_t s);
// The baseline filter (appended pairs) in place of count, scan and write,
// then the tick's totals.
void launch_join_sqb(const Bufs &B, uint32_t nq, const uint32_t *qord, hipStream_t s);
void launch_join_top_sqb(const Bufs &B, uint64_t cap_res, uint32_t policy, uint32_t period,
                         hipStream_t s);
void launch_pairs_hash(const Bufs &B, const uint32_t *qid, uint64_t *cnt, uint64_t *hash,
                       hipStream_t s);
void launch_pairs_count(const Bufs &B, uint32_t *cnt, hipStream_t s);
void launch_pairs_scatter(const Bufs &B, const uint64_t *off, uint32_t *cursor, uint32_t *ids,
                          hipStream_t s);
void launch_join_write(const Bufs &B, uint32_t nq, hipStream_t s);
// Trial builds and splits at every candidate threshold, cost prediction,
// and the choice of the threshold that the tick's build then uses.
// The candidates [c_lo, c_hi) are tried; the others keep an infinite cost.
void launch_tune(const Bufs &B, uint32_t c_lo, uint32_t c_hi, uint32_t l_max, uint32_t nq,
                 uint32_t covering, hipStream_t s);
// Host handle of the join write kernel (to find its node in a captured graph).
const void *join_write_kernel();
void launch_ctl_out(const Bufs &B, Ctl *host, hipStream_t s);
// k-nearest-neighbour queries: the candidate square of every query point
// (after the leaves of the tick are known, before the query split reads
// the squares as the tick's rectangles), and the selection of the k
// nearest among each square's results (after the join write pass).
void launch_knn_radius(const Bufs &B, const float *qx, const float *qy, uint32_t nq, uint32_t k,
                       hipStream_t s);
void launch_knn_select(const Bufs &B, const float *qx, const float *qy, uint32_t nq, uint32_t k,
                       uint32_t *out_id, float *out_d2, hipStream_t s);
void launch_counters(const Bufs &B, uint64_t *out, hipStream_t s);
void launch_hash(const Bufs &B, uint32_t nq, const uint32_t *qid, uint64_t *cnt, uint64_t *hash,
                 hipStream_t s);
// Expansion of the results of the queries sel[0 .. n) (sel null: queries
// 0 .. n-1 of the tick, n = nq): per-list sizes scanned into off[n + 1]
// (bad: set to 1 if a selected index is >= nq), then the ids, each list
// sorted ascending if asked.
void launch_expand_count(const Bufs &B, uint32_t nq, const uint32_t *sel, uint32_t n,
                         uint64_t *off, uint32_t *bad, hipStream_t s);
void launch_expand(const Bufs &B, uint32_t nq, const uint32_t *sel, uint32_t n, uint64_t *off,
                   uint32_t *ids, bool sorted, hipStream_t s);

}  // namespace sj
