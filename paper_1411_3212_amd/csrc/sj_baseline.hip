// The paper's baseline filter, kept as an ablation of the lock-free join
// (Section "Filtering phase in UG_Baseline", Algorithm SQB; study S1):
// results are appended as they are found, with atomics, instead of being
// counted, scanned and written to known places.
//
// A task (at most kTaskSub intersecting subqueries of one leaf) is taken by
// one block of one wave.  Lane k owns subquery k and tests it against every
// object of the leaf in turn (the objects are read by all lanes at once, a
// broadcast load).  A hit is appended to a buffer of (query, object) pairs
// in LDS through an atomic on the buffer's counter; when the next round
// might not fit, the wave reserves room for the buffer's contents with one
// atomic on the tick's global result counter and copies them out.  The
// pairs land in no particular order; a query's pairs are found by scanning
// all of them.  Covering subqueries are reported as in the lock-free path.
#include "sj_device.h"
#include "sj_kernels.h"

namespace sj {

constexpr uint32_t kSqbBuf = 2048;  // pairs buffered in LDS per wave

__global__ void __launch_bounds__(kWave) k_join_sqb(Ctl *ctl, const uint4 *trec,
                                                    const uint32_t *__restrict__ sq,
                                                    const float4 *__restrict__ qrect,
                                                    const float2 *__restrict__ sxy,
                                                    const uint32_t *__restrict__ sid,
                                                    const uint32_t *qord, uint2 *pairs,
                                                    uint64_t cap, uint32_t nq,
                                                    uint64_t *cu_tests) {
  __shared__ uint2 buf[kSqbBuf];
  __shared__ uint32_t cnt;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->qry_seq += nq;
    ctl->tick += 1;
  }
  if (!ctl->go_split) return;
  const uint32_t nt = ctl->n_run;
  const uint32_t lane = threadIdx.x;
  if (lane == 0) cnt = 0;
  __syncthreads();
  bool ovf = false;
  // copies the buffer out at a place reserved on the global counter
  auto flush = [&]() {
    const uint32_t n = cnt;
    uint64_t base = 0;
    if (lane == 0 && n)
      base = atomicAdd((unsigned long long *)&ctl->n_res, (unsigned long long)n);
    base = ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(base >> 32), 0) << 32) |
           (uint32_t)__shfl((int)(uint32_t)base, 0);
    for (uint32_t i = lane; i < n; i += kWave)
      if (base + i < cap) pairs[base + i] = buf[i];
    ovf = ovf || base + n > cap;
    __syncthreads();
    if (lane == 0) cnt = 0;
    __syncthreads();
  };
  for (uint32_t t = blockIdx.x; t < nt; t += gridDim.x) {
    const uint4 rec = trec[t];
    const uint32_t sb = rec.x, se = rec.y, ob = rec.z, oe = rec.w;
    if (sb >= se || ob >= oe) continue;
    const bool mine = sb + lane < se;
    const uint32_t g = mine ? sq[sb + lane] : 0u;
    const float4 r = mine ? qrect[g] : make_float4(1.f, 1.f, 0.f, 0.f);  // empty for idle lanes
    const uint32_t k = mine ? (qord ? qord[g] : g) : 0u;
    if (cu_tests && lane == 0)
      atomicAdd((unsigned long long *)&cu_tests[cu_slot()],
                (unsigned long long)(se - sb) * (oe - ob));
    for (uint32_t o = ob; o < oe; ++o) {
      if (cnt + (uint32_t)kWave > kSqbBuf) flush();  // the next round could overfill it
      const float2 p = sxy[o];
      if (r.x <= p.x && p.x <= r.z && r.y <= p.y && p.y <= r.w) {
        const uint32_t at = atomicAdd(&cnt, 1u);
        buf[at] = make_uint2(k, sid[o]);
      }
      __syncthreads();
    }
  }
  flush();
  flag_error(ctl, kErrOvfRes, ovf);
}

// Per-query result sizes and pair-set hashes of the appended pairs, added
// to what the covering leaves gave (k_hash ran first).
__global__ void __launch_bounds__(kBlock) k_pairs_hash(const Ctl *ctl, const uint2 *pairs,
                                                       uint64_t cap, const uint32_t *qid,
                                                       uint64_t *out_cnt, uint64_t *out_hash) {
  if (!ctl->go_join) return;
  const uint64_t n = ctl->n_res < cap ? ctl->n_res : cap;
  for (uint64_t i = blockIdx.x * (uint64_t)kBlock + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * kBlock) {
    const uint2 pr = pairs[i];
    atomicAdd((unsigned long long *)&out_cnt[pr.x], 1ull);
    atomicAdd((unsigned long long *)&out_hash[pr.x],
              (unsigned long long)mix64(((uint64_t)qid[pr.x] << 32) | pr.y));
  }
}

// Expansion of the appended pairs: per-query pair counts (cnt, added to
// the covering sizes already there), then each pair at the query's next
// free place (cursor, zeroed first) in front of its covering ids.
__global__ void __launch_bounds__(kBlock) k_pairs_count(const Ctl *ctl, const uint2 *pairs,
                                                        uint64_t cap, uint32_t *cnt) {
  if (!ctl->go_join) return;
  const uint64_t n = ctl->n_res < cap ? ctl->n_res : cap;
  for (uint64_t i = blockIdx.x * (uint64_t)kBlock + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * kBlock)
    atomicAdd(&cnt[pairs[i].x], 1u);
}

__global__ void __launch_bounds__(kBlock) k_pairs_scatter(const Ctl *ctl, const uint2 *pairs,
                                                          uint64_t cap, const uint64_t *off,
                                                          uint32_t *cursor, uint32_t *ids) {
  if (!ctl->go_join) return;
  const uint64_t n = ctl->n_res < cap ? ctl->n_res : cap;
  for (uint64_t i = blockIdx.x * (uint64_t)kBlock + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * kBlock) {
    const uint2 pr = pairs[i];
    ids[off[pr.x] + atomicAdd(&cursor[pr.x], 1u)] = pr.y;
  }
}

#define LAUNCH(k, g, b, s, ...) hipLaunchKernelGGL(k, dim3(g), dim3(b), 0, s, __VA_ARGS__)

void launch_join_sqb(const Bufs &B, uint32_t nq, const uint32_t *qord, hipStream_t s) {
  LAUNCH(k_join_sqb, kJoinBlocks * 4u, kWave, s, B.ctl, (const uint4 *)B.trec,
         (const uint32_t *)B.sq, (const float4 *)B.qrect, (const float2 *)B.sxy,
         (const uint32_t *)B.valA, qord, B.pairs, B.R, nq, B.cu_tests);
}

void launch_pairs_hash(const Bufs &B, const uint32_t *qid, uint64_t *cnt, uint64_t *hash,
                       hipStream_t s) {
  LAUNCH(k_pairs_hash, 4096, kBlock, s, (const Ctl *)B.ctl, (const uint2 *)B.pairs, B.R, qid, cnt,
         hash);
}

void launch_pairs_count(const Bufs &B, uint32_t *cnt, hipStream_t s) {
  LAUNCH(k_pairs_count, 4096, kBlock, s, (const Ctl *)B.ctl, (const uint2 *)B.pairs, B.R, cnt);
}

void launch_pairs_scatter(const Bufs &B, const uint64_t *off, uint32_t *cursor, uint32_t *ids,
                          hipStream_t s) {
  LAUNCH(k_pairs_scatter, 4096, kBlock, s, (const Ctl *)B.ctl, (const uint2 *)B.pairs, B.R, off,
         cursor, ids);
}

}  // namespace sj
