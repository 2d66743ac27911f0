// Threshold tuner: picks the leaf threshold of a quadtree build with the
// learned cost model.  For every candidate threshold it builds the quadtree
// (Algorithm 1) on the tick's sorted codes, splits the tick's queries
// against it, and predicts the cost of the tick's filtering and decoding
// from the terms of their complexity (Computational Complexity section,
// filtering and decoding equations): per active leaf c, the MLP predicts the
// join time of |P^c| objects against |Q_I^c| intersecting subqueries; the
// sum over leaves is the join's work, and the prediction for a leaf of at
// most kTaskSub subqueries (one join task, one wave) bounds its critical
// path through the largest such value; the split and the leaf passes add
// terms linear in |Q_I|, |Q_C| and the number of leaves, and the sort of
// the ticks that keep the tree a term per radix pass over the objects (leaf
// keys take fewer passes when there are fewer leaves).  The cheapest
// candidate is then built for the tick.  The paper fixes the threshold by hand after a sweep
// (Experimental evaluation, S5); this replaces the sweep, and the results
// of a tick do not depend on it.
//
// Everything runs on the device, with a launch sequence that depends only on
// the number of candidates, so a tuning tick can be captured in a graph.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "sj_device.h"
#include "sj_kernels.h"
#include "sj_mlp.h"

namespace sj {

// Clean state for one build at threshold th: the tick's errors as they were
// before the trial builds, an empty frontier holding the root.
__device__ void reset_build(Ctl *ctl, const TuneState *ts, uint4 *front0, uint32_t th) {
  ctl->err = ts->err_saved;
  ctl->th_cur = th;
  for (int l = 0; l < kFine + 2; ++l) ctl->fcount[l] = 0;
  ctl->fcount[0] = 1;
  ctl->n_leaves = 0;
  ctl->l_deep = 0;
  ctl->go_split = 0;
  ctl->n_isect = ctl->n_cov = 0;
  ctl->n32[0] = ctl->n32[1] = 0;
  front0[0] = make_uint4(0u, 0u, ctl->n_present, 0u);
}

// Candidates that this tuning does not try keep an infinite cost.
__global__ void k_tune_begin(Ctl *ctl, TuneState *ts) {
  ts->err_saved = ctl->err;
  ts->th_before = ctl->th_cur;
  for (int c = 0; c < kMaxCand; ++c) {
    ts->cost[c] = INFINITY;
    ts->msum[c] = ts->mmax[c] = 0.0f;
  }
}

__global__ void k_tune_set(Ctl *ctl, const TuneState *ts, uint32_t c, uint4 *front0) {
  reset_build(ctl, ts, front0, ts->cand[c]);
}

// The network staged in LDS as FP32 for wave-cooperative inference (W2
// rows padded to 65 so that lane i reading row i hits distinct banks).
struct MlpLds {
  float W2[kH][kH + 1];
  float W1[kH][kF];
  float b1[kH], b2[kH], w3[kH];
  float b3;
};

// All threads of the block take part; a barrier follows.
__device__ void stage_mlp(MlpLds &m, const uint16_t *w) {
  for (int i = threadIdx.x; i < kH * kH; i += blockDim.x) m.W2[i / kH][i % kH] = bf2f(w[kOW2 + i]);
  for (int i = threadIdx.x; i < kH * kF; i += blockDim.x) m.W1[i / kF][i % kF] = bf2f(w[kOW1 + i]);
  if (threadIdx.x < kH) {
    m.b1[threadIdx.x] = bf2f(w[kOB1 + threadIdx.x]);
    m.b2[threadIdx.x] = bf2f(w[kOB2 + threadIdx.x]);
    m.w3[threadIdx.x] = bf2f(w[kOW3 + threadIdx.x]);
  }
  if (threadIdx.x == 0) m.b3 = bf2f(w[kOB3]);
  __syncthreads();
}

// Output of the network for one input; called by all lanes of a wave with
// the same input: lane j computes hidden unit j of both layers (the first
// layer's outputs are broadcast lane by lane) and a wave sum gives y.
__device__ __forceinline__ float wave_mlp(const MlpLds &m, float x0, float x1, float x2,
                                          float x3) {
  const uint32_t lane = lane_id();
  float a = m.b1[lane];
  a = fmaf(m.W1[lane][0], x0, a);
  a = fmaf(m.W1[lane][1], x1, a);
  a = fmaf(m.W1[lane][2], x2, a);
  a = fmaf(m.W1[lane][3], x3, a);
  const float h1 = a > 0.0f ? a : 0.0f;
  float a2 = m.b2[lane];
  for (int j = 0; j < kH; ++j) a2 = fmaf(m.W2[lane][j], readlane_f(h1, j), a2);
  const float h2 = a2 > 0.0f ? a2 : 0.0f;
  return wave_sum(m.w3[lane] * h2) + m.b3;
}

// Mean over the intersecting subqueries [sb, se) of leaf t of the fraction
// of the leaf's area their rectangle covers (whole wave).
__device__ __forceinline__ float mean_overlap(const Ctl *ctl, const uint32_t *lstart,
                                              const uint32_t *llevel, uint32_t t, uint32_t sb,
                                              uint32_t se, const uint32_t *sq,
                                              const float4 *qrect) {
  float ov = 0.0f;
  for (uint32_t i = sb + lane_id(); i < se; i += kWave)
    ov += overlap_frac(ctl, lstart, llevel, t, qrect[sq[i]]);
  return wave_sum(ov) / (float)(se - sb);
}

// Per-block partials of the sum over active leaves of exp(MLP(features))
// and of the maximum of exp(MLP(features of one join task)), the subquery
// count capped at kTaskSub.  One wave per leaf.
__global__ void __launch_bounds__(kBlock) k_cost_leaves(const Ctl *ctl, const TuneState *ts,
                                                        const uint32_t *leaf_beg,
                                                        const uint32_t *leaf_sqoff,
                                                        const uint32_t *sq, const float4 *qrect,
                                                        const uint32_t *lstart,
                                                        const uint32_t *llevel, uint64_t *red) {
  __shared__ MlpLds m;
  __shared__ double sacc[kWavesPerBlock], smax[kWavesPerBlock];
  stage_mlp(m, ts->w);
  const uint32_t lane = lane_id();
  double acc = 0.0, mx = 0.0;
  if (ctl->go_split) {
    const uint32_t n = ctl->n_leaves;
    const uint32_t nwaves = gridDim.x * kWavesPerBlock;
    const uint32_t w0 =
        __builtin_amdgcn_readfirstlane(blockIdx.x * kWavesPerBlock + threadIdx.x / kWave);
    for (uint32_t t = w0; t < n; t += nwaves) {
      const uint32_t cnt = leaf_beg[t + 1] - leaf_beg[t];
      const uint32_t sb = leaf_sqoff[t], se = leaf_sqoff[t + 1];
      if (cnt == 0 || sb == se) continue;
      const float ov = mean_overlap(ctl, lstart, llevel, t, sb, se, sq, qrect);
      const uint32_t nsq = se - sb;
      const float x0 = log2f(1.0f + (float)cnt);
      const float x2 = (float)llevel[t] * (1.0f / 16.0f);
      const double e = (double)expf(wave_mlp(m, x0, log2f(1.0f + (float)nsq), x2, ov));
      const double et =
          nsq <= kTaskSub ? e
                          : (double)expf(wave_mlp(m, x0, log2f(1.0f + (float)kTaskSub), x2, ov));
      acc += e;
      mx = et > mx ? et : mx;
    }
  }
  if (lane == 0) {
    sacc[threadIdx.x / kWave] = acc;
    smax[threadIdx.x / kWave] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0, mm = 0.0;
    for (int w = 0; w < kWavesPerBlock; ++w) {
      s += sacc[w];
      mm = smax[w] > mm ? smax[w] : mm;
    }
    red[kRedCost * kChunkBlocks + blockIdx.x] = (uint64_t)__double_as_longlong(s);
    red[kRedCostMax * kChunkBlocks + blockIdx.x] = (uint64_t)__double_as_longlong(mm);
  }
}

// Learned schedule: the key of every join task of a leaf from the
// network's prediction for that task (its subquery count is kTaskSub, or
// what remains for the last one): 254 - min(254, 16 (ln us + 4)), so the
// counting sort over the keys puts the longest predicted tasks first.
// Keys of tasks without work stay 255 (not run).
__device__ __forceinline__ uint32_t time_key(float y) {
  const float q = 16.0f * (y + 4.0f);
  const uint32_t k = !(q > 0.0f) ? 0u : (q >= 254.0f ? 254u : (uint32_t)q);
  return 254u - k;
}

__global__ void __launch_bounds__(kBlock) k_task_keys_mlp(const Ctl *ctl, const TuneState *ts,
                                                          const uint32_t *leaf_beg,
                                                          const uint32_t *leaf_sqoff,
                                                          const uint32_t *sq,
                                                          const float4 *qrect,
                                                          const uint32_t *lstart,
                                                          const uint32_t *llevel,
                                                          const uint32_t *xbase, uint32_t tcap,
                                                          uint32_t *tkey, uint32_t *tkhist) {
  __shared__ MlpLds m;
  __shared__ uint32_t lh[256];
  static_assert(kBlock == 256, "one key count per thread");
  stage_mlp(m, ts->w);
  lh[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t n = ctl->go_split ? ctl->n_leaves : 0u;
  const uint32_t nwaves = gridDim.x * kWavesPerBlock;
  const uint32_t w0 =
      __builtin_amdgcn_readfirstlane(blockIdx.x * kWavesPerBlock + threadIdx.x / kWave);
  for (uint32_t t = w0; t < n; t += nwaves) {
    const uint32_t cnt = leaf_beg[t + 1] - leaf_beg[t];
    const uint32_t sb = leaf_sqoff[t], se = leaf_sqoff[t + 1];
    if (cnt == 0 || sb == se) continue;
    const float ov = mean_overlap(ctl, lstart, llevel, t, sb, se, sq, qrect);
    const uint32_t nsq = se - sb, more = (nsq - 1u) / kTaskSub;
    const float x0 = log2f(1.0f + (float)cnt);
    const float x2 = (float)llevel[t] * (1.0f / 16.0f);
    const uint32_t first = nsq < kTaskSub ? nsq : kTaskSub;
    const uint32_t kf = time_key(wave_mlp(m, x0, log2f(1.0f + (float)first), x2, ov));
    const uint32_t last = nsq - more * kTaskSub;
    const uint32_t kl =
        more == 0u ? kf : time_key(wave_mlp(m, x0, log2f(1.0f + (float)last), x2, ov));
    if (lane_id() == 0) {
      tkey[t] = kf;
      atomicAdd(&lh[kf], 1u);
    }
    // further tasks: full chunks, the last one holds what remains
    for (uint32_t c = 1u + lane_id(); c <= more; c += kWave) {
      const uint32_t e = xbase[t] + c - 1u;
      if (e < tcap) {
        const uint32_t k = c == more ? kl : kf;
        tkey[e] = k;
        atomicAdd(&lh[k], 1u);
      }
    }
  }
  __syncthreads();
  const uint32_t c = lh[threadIdx.x];
  if (c) atomicAdd(&tkhist[threadIdx.x], c);
}

// Predicted cost of candidate c (one block of kChunkBlocks threads): the
// MLP sum and maximum plus the linear terms; infinite when the candidate
// overflowed a capacity.
__global__ void __launch_bounds__(kChunkBlocks) k_tune_cost(const Ctl *ctl, TuneState *ts,
                                                            uint32_t c, const uint64_t *red) {
  __shared__ double lds[kChunkBlocks / kWave], ldm[kChunkBlocks / kWave];
  double v = __longlong_as_double((long long)red[kRedCost * kChunkBlocks + threadIdx.x]);
  double u = __longlong_as_double((long long)red[kRedCostMax * kChunkBlocks + threadIdx.x]);
  v = wave_sum(v);
  u = wave_max(u);
  if (lane_id() == 0) {
    lds[threadIdx.x / kWave] = v;
    ldm[threadIdx.x / kWave] = u;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double s = 0.0, m = 0.0;
  for (int w = 0; w < kChunkBlocks / kWave; ++w) {
    s += lds[w];
    m = ldm[w] > m ? ldm[w] : m;
  }
  const bool ok = ctl->go_split && !(ctl->err & kErrOverflow);
  // radix passes of the leaf-keyed sort on the ticks that keep this tree
  const uint32_t nl = ctl->n_leaves;
  const uint32_t passes = nl > 1u ? (32u - (uint32_t)__clz((int)(nl - 1u)) + 7u) / 8u : 0u;
  const double cost = (double)ts->coef[0] * s + (double)ts->coef[1] * (double)ctl->n_isect +
                      (double)ts->coef[2] * (double)ctl->n_cov + (double)ts->coef[3] * (double)nl +
                      (double)ts->coef[4] * m +
                      (double)ts->coef[5] * (double)passes * (double)ctl->n_present;
  ts->cost[c] = ok ? (float)cost : INFINITY;
  ts->msum[c] = (float)s;
  ts->mmax[c] = (float)m;
}

// Cheapest candidate (the first of equal costs; the threshold before the
// tuning when none is feasible), then a clean state for its build.
__global__ void k_tune_pick(Ctl *ctl, TuneState *ts, uint4 *front0) {
  uint32_t best = ts->th_before;
  float bc = INFINITY;
  for (uint32_t c = 0; c < ts->n_cand && c < (uint32_t)kMaxCand; ++c) {
    if (ts->cost[c] < bc) {
      bc = ts->cost[c];
      best = ts->cand[c];
    }
  }
  ts->chosen = best;
  ts->n_tunes += 1;
  ts->tuned_tick = ctl->tick;
  reset_build(ctl, ts, front0, best);
}

#define LAUNCH(k, g, b, s, ...) hipLaunchKernelGGL(k, dim3(g), dim3(b), 0, s, __VA_ARGS__)

void launch_schedule_mlp(const Bufs &B, hipStream_t s) {
  LAUNCH(k_task_keys_mlp, kChunkBlocks, kBlock, s, (const Ctl *)B.ctl, (const TuneState *)B.tune,
         (const uint32_t *)B.leaf_beg, (const uint32_t *)B.leaf_sqoff, (const uint32_t *)B.sq,
         (const float4 *)B.qrect, (const uint32_t *)B.lstart, (const uint32_t *)B.llevel,
         (const uint32_t *)B.xbase, B.TCAP, B.tkey, B.tkhist);
}

void launch_tune(const Bufs &B, uint32_t c_lo, uint32_t c_hi, uint32_t l_max, uint32_t nq,
                 uint32_t covering, hipStream_t s) {
  LAUNCH(k_tune_begin, 1, 1, s, B.ctl, B.tune);
  for (uint32_t c = c_lo; c < c_hi; ++c) {
    LAUNCH(k_tune_set, 1, 1, s, B.ctl, (const TuneState *)B.tune, c, B.front[0]);
    launch_build(B, l_max, s);
    launch_leaves(B, s);
    launch_split(B, nq, covering, s);
    LAUNCH(k_cost_leaves, kChunkBlocks, kBlock, s, (const Ctl *)B.ctl, (const TuneState *)B.tune,
           (const uint32_t *)B.leaf_beg, (const uint32_t *)B.leaf_sqoff, (const uint32_t *)B.sq,
           (const float4 *)B.qrect, (const uint32_t *)B.lstart, (const uint32_t *)B.llevel, B.red);
    LAUNCH(k_tune_cost, 1, kChunkBlocks, s, (const Ctl *)B.ctl, B.tune, c,
           (const uint64_t *)B.red);
  }
  LAUNCH(k_tune_pick, 1, 1, s, B.ctl, B.tune, B.front[0]);
}

}  // namespace sj
