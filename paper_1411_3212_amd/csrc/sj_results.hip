// Kernels that read a tick's compressed results after the tick: per-query
// result sizes and pair-set hashes, and the expansion of the results into
// per-query id lists (optionally sorted).  None of them runs inside a tick.
#include "sj_device.h"
#include "sj_kernels.h"

namespace sj {


// The results of query k, at processing position p = qpos[k], are runs of
// ids: for every intersecting slot s in [q_ioff[p], q_ioff[p+1]), the run of
// subquery i = slot_sq[s], res_ids[res_off[i] .. res_off[i+1]); for every
// covering leaf L in cov_leaf[q_coff[p] .. q_coff[p+1]), its objects
// sid[leaf_beg[L] .. leaf_beg[L+1]).  A wave takes a query and walks its
// runs in that order.
struct Runs {
  const uint32_t *q_ioff, *slot_sq, *res_ids, *q_coff, *cov_leaf, *leaf_beg, *sid, *qpos;
  const uint64_t *res_off;
  uint32_t isect;  // 0: the intersecting results are appended pairs, not runs
};

// f(id, position in the query's list) for every id of query k, lane by lane.
template <typename F>
__device__ __forceinline__ uint64_t for_each_id(const Runs &R, uint32_t k, uint32_t lane, F f) {
  uint64_t pos = 0;
  const uint32_t p = R.qpos[k];
  for (uint32_t s = R.isect ? R.q_ioff[p] : 0u; s < (R.isect ? R.q_ioff[p + 1] : 0u); ++s) {
    const uint32_t i = R.slot_sq[s];
    const uint64_t a = R.res_off[i], b = R.res_off[i + 1];
    for (uint64_t j = a + lane; j < b; j += kWave) f(R.res_ids[j], pos + (j - a));
    pos += b - a;
  }
  for (uint32_t e = R.q_coff[p]; e < R.q_coff[p + 1]; ++e) {
    const uint32_t leaf = R.cov_leaf[e];
    const uint32_t lb = R.leaf_beg[leaf], le = R.leaf_beg[leaf + 1];
    for (uint32_t j = lb + lane; j < le; j += kWave) f(R.sid[j], pos + (j - lb));
    pos += le - lb;
  }
  return pos;
}

// Result size of query k (one thread).
__device__ __forceinline__ uint64_t result_size(const Runs &R, uint32_t k) {
  uint64_t c = 0;
  const uint32_t p = R.qpos[k];
  for (uint32_t s = R.isect ? R.q_ioff[p] : 0u; s < (R.isect ? R.q_ioff[p + 1] : 0u); ++s) {
    const uint32_t i = R.slot_sq[s];
    c += R.res_off[i + 1] - R.res_off[i];
  }
  for (uint32_t e = R.q_coff[p]; e < R.q_coff[p + 1]; ++e)
    c += R.leaf_beg[R.cov_leaf[e] + 1] - R.leaf_beg[R.cov_leaf[e]];
  return c;
}

__global__ void __launch_bounds__(kBlock) k_hash(const Ctl *ctl, uint32_t nq, const uint32_t *qid,
                                                 Runs R, uint64_t *out_cnt, uint64_t *out_hash) {
  const uint32_t lane = lane_id();
  const uint32_t nwaves = gridDim.x * kWavesPerBlock;
  const bool ok = ctl->go_join != 0;
  for (uint32_t k = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; k < nq; k += nwaves) {
    if (!ok) {
      if (lane == 0) out_cnt[k] = out_hash[k] = 0ull;
      continue;
    }
    const uint64_t hi = (uint64_t)qid[k] << 32;
    uint64_t h = 0;
    const uint64_t c = for_each_id(R, k, lane, [&](uint32_t id, uint64_t) { h += mix64(hi | id); });
    h = wave_sum(h);
    if (lane == 0) {
      out_cnt[k] = c;
      out_hash[k] = h;
    }
  }
}

// Expansion of the compressed results, per query (all of the tick's queries,
// or the query indices of a selection sel[0 .. n)): count, then the ids of
// the intersecting runs followed by every covering leaf's objects.  A
// selected index >= nq is flagged in *bad and selects an empty list.
__global__ void __launch_bounds__(kBlock) k_exp_count(const Ctl *ctl, uint32_t nq,
                                                      const uint32_t *sel, uint32_t n, Runs R,
                                                      uint32_t *cnt, uint32_t *bad) {
  const bool ok = ctl->go_join != 0;
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const uint32_t k = sel ? sel[i] : i;
    if (k >= nq) *bad = 1u;
    cnt[i] = ok && k < nq ? (uint32_t)result_size(R, k) : 0u;
  }
}

// pos0 (optional): per query, the places already taken at the front of its
// list (appended pairs).
__global__ void __launch_bounds__(kBlock) k_exp_write(const Ctl *ctl, uint32_t nq,
                                                      const uint32_t *sel, uint32_t n, Runs R,
                                                      const uint64_t *off, const uint32_t *pos0,
                                                      uint32_t *ids) {
  if (!ctl->go_join) return;
  const uint32_t lane = lane_id();
  const uint32_t nwaves = gridDim.x * kWavesPerBlock;
  for (uint32_t i = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; i < n; i += nwaves) {
    const uint32_t k = sel ? sel[i] : i;
    if (k >= nq) continue;
    uint32_t *dst = ids + off[i] + (pos0 ? pos0[k] : 0u);
    for_each_id(R, k, lane, [&](uint32_t id, uint64_t p) { dst[p] = id; });
  }
}

// Ascending sort of a[0 .. n) by one block: a bitonic network whose
// comparators all put the smaller key at the lower index (the first step of
// each merge compares mirrored positions), so entries past n act as +inf
// padding and their comparators are skipped.  a is in LDS or in global
// memory (the block's barriers order the steps in either).
__device__ void block_bitonic_sort(uint32_t *a, uint32_t n) {
  uint32_t P = 1;
  while (P < n) P <<= 1;
  for (uint32_t k = 2; k <= P; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t q = threadIdx.x; q < P / 2; q += blockDim.x) {
        const uint32_t i = j == (k >> 1) ? (q / j) * k + (q % j) : (q / j) * 2u * j + (q % j);
        const uint32_t p = j == (k >> 1) ? i ^ (k - 1u) : i + j;
        if (p < n) {
          const uint32_t x = a[i], y = a[p];
          if (y < x) {
            a[i] = y;
            a[p] = x;
          }
        }
      }
      __syncthreads();
    }
  }
}

// Canonical order of expanded lists: every list ids[off[i] .. off[i+1])
// sorted ascending, one block per list; lists of up to kSortLds ids are
// sorted in LDS, longer ones in place.
constexpr uint32_t kSortLds = 8192;

__global__ void __launch_bounds__(kBlock) k_exp_sort(uint32_t n, const uint64_t *off,
                                                     uint32_t *ids) {
  __shared__ uint32_t lds[kSortLds];
  for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
    const uint64_t a = off[i];
    const uint32_t len = (uint32_t)(off[i + 1] - a);
    if (len < 2u) continue;
    uint32_t *seg = ids + a;
    if (len <= kSortLds) {
      for (uint32_t j = threadIdx.x; j < len; j += kBlock) lds[j] = seg[j];
      __syncthreads();
      block_bitonic_sort(lds, len);
      for (uint32_t j = threadIdx.x; j < len; j += kBlock) seg[j] = lds[j];
      __syncthreads();
    } else {
      block_bitonic_sort(seg, len);
    }
  }
}

#define LAUNCH(k, g, b, s, ...) hipLaunchKernelGGL(k, dim3(g), dim3(b), 0, s, __VA_ARGS__)

static Runs runs_of(const Bufs &B) {
  return Runs{(const uint32_t *)B.q_ioff,  (const uint32_t *)B.slot_sq,
              (const uint32_t *)B.res_ids, (const uint32_t *)B.q_coff,
              (const uint32_t *)B.cov_leaf, (const uint32_t *)B.leaf_beg,
              (const uint32_t *)B.valA,    (const uint32_t *)B.qpos,
              (const uint64_t *)B.res_off,
              B.pairs ? 0u : 1u};
}

void launch_hash(const Bufs &B, uint32_t nq, const uint32_t *qid, uint64_t *cnt, uint64_t *hash,
                 hipStream_t s) {
  LAUNCH(k_hash, grid_for((uint64_t)nq * kWave, 4096), kBlock, s, (const Ctl *)B.ctl, nq, qid,
         runs_of(B), cnt, hash);
  if (B.pairs) launch_pairs_hash(B, qid, cnt, hash, s);
}

void launch_expand_count(const Bufs &B, uint32_t nq, const uint32_t *sel, uint32_t n,
                         uint64_t *off, uint32_t *bad, hipStream_t s) {
  LAUNCH(k_exp_count, grid_for(n, 4096), kBlock, s, (const Ctl *)B.ctl, nq, sel, n, runs_of(B),
         B.q_ni, bad);
  if (B.pairs) launch_pairs_count(B, B.q_ni, s);  // every query (no selection with pairs)
  ScanJobs jobs{};
  jobs.j[0] = job_u64(B.q_ni, off, nullptr, n);
  mscan(jobs, 1, B.part, nullptr, nullptr, s);
}

void launch_expand(const Bufs &B, uint32_t nq, const uint32_t *sel, uint32_t n, uint64_t *off,
                   uint32_t *ids, bool sorted, hipStream_t s) {
  if (B.pairs) {  // the pairs first, at each query's cursor, then the covering ids
    launch_fill_u32(B.q_nc, nq, 0u, s);
    launch_pairs_scatter(B, (const uint64_t *)off, B.q_nc, ids, s);
  }
  LAUNCH(k_exp_write, grid_for((uint64_t)n * kWave, 4096), kBlock, s, (const Ctl *)B.ctl, nq, sel,
         n, runs_of(B), (const uint64_t *)off, B.pairs ? (const uint32_t *)B.q_nc : nullptr,
         ids);
  if (sorted)
    LAUNCH(k_exp_sort, n < 65536u ? (n ? n : 1u) : 65536u, kBlock, s, n, (const uint64_t *)off,
           ids);
}

}  // namespace sj
