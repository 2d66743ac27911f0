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
  uint32_t *leaf_beg, *leaf_nsq, *leaf_sqoff;
  uint32_t *leaf_ovf, *leaf_ovfc;       // subqueries past a query's list: count, cursor
  // schedule
  uint32_t *tkey;                       // order key of every join task (TCAP)
  uint32_t *qkey, *qord, *qkey2, *qord2;  // spatial processing order of the queries (Q)
  uint32_t *tkhist;                     // 256 task-key totals, 256 placement cursors
  uint2 *vtask;                         // further chunks of heavy leaves: (leaf, chunk)
  uint32_t *xbase;                      // per leaf: task index of its second chunk
  uint4 *trec;                          // tasks in run order: subquery and object ranges
  uint32_t *tleaf;                      // tasks in run order: leaf
  // queries and subqueries
  float4 *qrect;
  uint32_t *q_ni, *q_nc, *q_ioff, *q_coff;
  uint64_t *q_roff;
  uint32_t *qlist;                      // visited leaves per query (slots each)
  uint32_t *qpos;                       // their positions in the leaves' groups
  uint2 *sq;                            // subqueries grouped by leaf: (query, slot)
  uint32_t *sq_cnt;
  uint64_t *res_off;
  uint32_t *cov_leaf, *res_ids;
  float *tlog;                          // per-leaf timing log (or null)
  TuneState *tune;                      // threshold tuner state
  // capacities
  uint32_t N, Q, LCAP, NCAP, FCAP, slots, tcap, TCAP;
  uint64_t S, C, R;
};

void launch_ctl_init(Ctl *ctl, uint32_t th, hipStream_t s);
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
void launch_split(const Bufs &B, uint32_t nq, uint32_t covering, hipStream_t s);
void launch_schedule(const Bufs &B, uint32_t reorder, uint32_t l_max, bool learned,
                     hipStream_t s);
// Task keys from the cost model's predicted task times (learned schedule).
void launch_schedule_mlp(const Bufs &B, hipStream_t s);
void launch_join_count(const Bufs &B, hipStream_t s);
void launch_join_scan(const Bufs &B, uint64_t cap_res, uint32_t policy, uint32_t period,
                      hipStream_t s);
void launch_join_write(const Bufs &B, uint32_t nq, hipStream_t s);
// Trial builds and splits at every candidate threshold, cost prediction,
// and the choice of the threshold that the tick's build then uses.
void launch_tune(const Bufs &B, uint32_t n_cand, uint32_t l_max, uint32_t nq, uint32_t covering,
                 hipStream_t s);
// Host handle of the join write kernel (to find its node in a captured graph).
const void *join_write_kernel();
void launch_ctl_out(const Bufs &B, Ctl *host, hipStream_t s);
void launch_counters(const Bufs &B, uint64_t *out, hipStream_t s);
void launch_hash(const Bufs &B, uint32_t nq, const uint32_t *qid, uint64_t *cnt, uint64_t *hash,
                 hipStream_t s);
void launch_expand_count(const Bufs &B, uint32_t nq, uint64_t *off, hipStream_t s);
void launch_expand(const Bufs &B, uint32_t nq, uint64_t *off, uint32_t *ids, hipStream_t s);

}  // namespace sj
