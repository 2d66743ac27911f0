// Repeated k-nearest-neighbour queries on the range-query pipeline (the
// paper's stated future work, Section "Conclusions": reuse the pipeline for
// kNN queries issued by moving objects).
//
// A query (qid, qx, qy) asks for the k present objects of smallest key
// (d2, id), d2 = fl32(fl32(dx*dx) + fl32(dy*dy)) with dx = fl32(px - qx),
// dy = fl32(py - qy).  A tick of kNN queries is a tick of range queries
// whose rectangles are candidate squares, plus a selection:
//   radius     per query, one wave: a square around the query point that
//              holds its k nearest objects.  The smallest quadrant holding
//              the point with at least k objects (its leaf, or an ancestor:
//              a run of whole leaves in Morton order, one range of the
//              sorted objects) gives the half side: a distance within
//              which k of its objects lie (an upper bound of the k-th
//              nearest distance over all objects): every lane keeps the
//              smallest distance of the objects it scans, and the k-th
//              smallest of those 64 minima belongs to k distinct objects
//              (k <= 64, and at least k lanes scan one); for a quadrant of
//              more than kKnnScanMax objects, the distance to its farthest
//              corner.
//   range      the tick's split, schedule and join on those squares:
//              candidates as runs of ids and covering leaves.
//   select     per query, one wave: the k smallest keys among the
//              candidates, kept as a sorted list across the lanes and
//              merged with each batch of 64 candidates by a bitonic
//              network.  Completeness is proved, not assumed: every object
//              outside the square has d2 >= LB, the smallest binary32 square
//              of the distances from the point to the square's sides
//              (rounding is monotone), so the list is exact when it holds k
//              candidates and its k-th d2 is below LB.  A query that fails
//              the proof (possible only through rounding at the square's
//              edge or objects outside the index frame) is listed for
//              the fallback.
//   fallback   one wave per listed query scans every present object.
#include <float.h>

#include "sj_device.h"
#include "sj_kernels.h"
#include "sj_tree.h"

namespace sj {

constexpr uint64_t kNoKey = ~0ull;  // an empty slot (above every real key)
// Quadrants of at most this many objects bound a query's k-th distance by
// their objects' distances; larger ones by their farthest corner.
constexpr uint32_t kKnnScanMax = 4096;

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
  const int lo = __shfl((int)(uint32_t)v, src, kWave);
  const int hi = __shfl((int)(uint32_t)(v >> 32), src, kWave);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}
__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
  const int lo = __shfl_xor((int)(uint32_t)v, m, kWave);
  const int hi = __shfl_xor((int)(uint32_t)(v >> 32), m, kWave);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// One key per lane sorted ascending with the lane index (bitonic network).
__device__ __forceinline__ uint64_t wave_sort_u64(uint64_t v, uint32_t lane) {
#pragma unroll
  for (uint32_t size = 2; size <= (uint32_t)kWave; size <<= 1) {
#pragma unroll
    for (uint32_t j = size >> 1; j > 0; j >>= 1) {
      const uint64_t o = shfl_xor_u64(v, (int)j);
      const bool keep_min = ((lane & j) == 0) == ((lane & size) == 0);
      v = keep_min ? (o < v ? o : v) : (o > v ? o : v);
    }
  }
  return v;
}

// best: lane i holds the i-th smallest key seen so far.  The 64 smallest of
// best and a batch of 64 keys: the batch sorted, reversed against best,
// lane-wise minima (a bitonic sequence holding the 64 smallest), then a
// bitonic merge.
__device__ __forceinline__ uint64_t topk_merge(uint64_t best, uint64_t key, uint32_t lane) {
  const uint64_t b = wave_sort_u64(key, lane);
  const uint64_t r = shfl_u64(b, (int)((uint32_t)kWave - 1u - lane));
  uint64_t c = r < best ? r : best;
#pragma unroll
  for (uint32_t j = (uint32_t)kWave >> 1; j > 0; j >>= 1) {
    const uint64_t o = shfl_xor_u64(c, (int)j);
    c = (lane & j) == 0 ? (o < c ? o : c) : (o > c ? o : c);
  }
  return c;
}

// The squared distance of the definition, each operation rounded on its own.
__device__ __forceinline__ float knn_d2(float2 p, float x, float y) {
  const float dx = __fsub_rn(p.x, x), dy = __fsub_rn(p.y, y);
  return __fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy));
}
__device__ __forceinline__ uint64_t knn_key(float d2, uint32_t id) {
  return ((uint64_t)__float_as_uint(d2) << 32) | id;
}

// The same for 32-bit keys, ascending across the lanes (the radius needs
// distances only).
__device__ __forceinline__ uint32_t wave_sort_u32(uint32_t v, uint32_t lane) {
#pragma unroll
  for (uint32_t size = 2; size <= (uint32_t)kWave; size <<= 1) {
#pragma unroll
    for (uint32_t j = size >> 1; j > 0; j >>= 1) {
      const uint32_t o = (uint32_t)__shfl_xor((int)v, (int)j, kWave);
      const bool keep_min = ((lane & j) == 0) == ((lane & size) == 0);
      v = keep_min ? (o < v ? o : v) : (o > v ? o : v);
    }
  }
  return v;
}

// Adds a batch (one key per lane, kNoKey for none) to the wave's list when
// one of its keys is below the k-th of the list.
__device__ __forceinline__ uint64_t topk_add(uint64_t best, uint64_t key, uint32_t k,
                                             uint32_t lane) {
  const uint64_t kth = shfl_u64(best, (int)(k - 1u));
  if (ballot(key < kth)) best = topk_merge(best, key, lane);
  return best;
}

// Query q is its object's latest of the tick (seq: the query sequence
// number before the tick; the join's write pass advances it by nq).
__device__ __forceinline__ bool knn_live(uint64_t seq, const uint64_t *qstamp, uint32_t o,
                                         uint32_t N, uint32_t q) {
  return o < N && qstamp[o] == seq + q + 1;
}

// ----------------------------------------------------------------- radius --
// The candidate squares are the tick's query rectangles: four arrays of Q
// binary32 (xa, ya, xb, yb), the layout the query split reads.
__device__ __forceinline__ void put_rect(float *rect, uint32_t Q, uint32_t q, float4 r,
                                         uint32_t lane) {
  if (lane < 4u)
    rect[(uint64_t)lane * Q + q] = lane == 0u ? r.x : lane == 1u ? r.y : lane == 2u ? r.z : r.w;
}
__global__ void __launch_bounds__(kBlock) k_knn_radius(
    const Ctl *ctl, const TickIn *tin, const float *qx, const float *qy, uint32_t nq, uint32_t N,
    const uint64_t *qstamp, Tree tr, const uint32_t *leaf_beg, const float2 *sxy, uint32_t k,
    float *rect, uint32_t Q) {
  const uint32_t lane = lane_id();
  const uint32_t nw = gridDim.x * kWavesPerBlock;
  // no usable quadtree (its capacity overflowed: the tick reports it): the
  // largest squares
  const uint32_t nl = (ctl->err & kErrOvfTree) ? 0u : ctl->n_leaves;
  const float x0 = ctl->x0, y0 = ctl->y0, sc = ctl->scale;
  const double inv = 1.0 / (double)sc;  // cell side (a power of two)
  tr.tlev = ctl->tlev;
  const uint32_t *__restrict__ qid = tin->qid;
  for (uint32_t q = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; q < nq; q += nw) {
    const float x = qx[q], y = qy[q];
    float4 r = make_float4(x, y, x, y);
    if (!knn_live(ctl->qry_seq, qstamp, qid[q], N, q) || !isfinite(x) || !isfinite(y)) {
      // a superseded query: any rectangle (the split skips it); a live
      // query at a non-finite point: an invalid one, reported by the split
      put_rect(rect, Q, q, isfinite(x) && isfinite(y) ? r : make_float4(NAN, NAN, NAN, NAN),
               lane);
      continue;
    }
    const uint32_t ci = cell_of(x, x0, sc), cj = cell_of(y, y0, sc);
    const uint32_t code = morton2(ci, cj);
    double h = INFINITY;
    if (nl > 0u) {
      // the smallest quadrant holding the point with k objects or more: the
      // point's leaf, or an ancestor (a run of whole leaves in Morton order,
      // whose objects are one range of the sorted order)
      const uint32_t L = leaf_of(tr, code);
      uint32_t ob = leaf_beg[L], oe = leaf_beg[L + 1];
      int lq = (int)tr.llevel[L];
      for (int l = lq - 1; oe - ob < k && l >= 0; --l) {
        const uint32_t s = 2u * (uint32_t)(kFine - l);
        const uint64_t c0 = s >= 32u ? 0ull : (uint64_t)(code >> s) << s;
        const uint64_t c1 = c0 + (1ull << s);
        const uint32_t lo = lower_bound_u32(tr.lstart, 0u, nl, (uint32_t)c0);
        const uint32_t hi =
            c1 > 0xffffffffull ? nl : lower_bound_u32(tr.lstart, lo, nl, (uint32_t)c1);
        ob = leaf_beg[lo];
        oe = leaf_beg[hi];
        lq = l;
      }
      if (oe - ob >= k && oe - ob <= kKnnScanMax) {
        // the k-th smallest of the lanes' smallest distances (binary32 bits
        // of d2 >= 0 order like the values; a lane without objects keeps
        // the largest key)
        uint32_t m = 0xffffffffu;
        for (uint32_t i0 = ob; i0 < oe; i0 += kWave) {
          const uint32_t i = i0 + lane;
          if (i < oe) m = min(m, __float_as_uint(knn_d2(sxy[i], x, y)));
        }
        const uint32_t srt = wave_sort_u32(m, lane);
        const float d2k = __uint_as_float((uint32_t)__shfl((int)srt, (int)(k - 1u), kWave));
        h = sqrt((double)d2k) * (1.0 + 1.0 / 1024.0);
      } else if (oe - ob >= k) {
        // a large quadrant: its farthest corner from the point
        const uint32_t m = (uint32_t)(kFine - lq);
        const double qi0 = (double)((ci >> m) << m), qj0 = (double)((cj >> m) << m);
        const double w = (double)(1u << m);
        const double X0 = (double)x0 + qi0 * inv, X1 = X0 + w * inv;
        const double Y0 = (double)y0 + qj0 * inv, Y1 = Y0 + w * inv;
        const double mx = fmax(fabs((double)x - X0), fabs(X1 - (double)x));
        const double my = fmax(fabs((double)y - Y0), fabs(Y1 - (double)y));
        h = sqrt(mx * mx + my * my) * (1.0 + 1.0 / 1024.0);
      }
    }
    // a margin above the bound (so that a k-th distance of 0, e.g. at a
    // point shared by k objects, still leaves the sides strictly away from
    // the point); fewer than k objects in all: the largest square
    h += (fabs((double)x) + fabs((double)y)) * (1.0 / 1048576.0) + 1e-30;
    if (h < (double)FLT_MAX)
      r = make_float4((float)((double)x - h), (float)((double)y - h), (float)((double)x + h),
                      (float)((double)y + h));
    if (!(h < (double)FLT_MAX) || !isfinite(r.x) || !isfinite(r.y) || !isfinite(r.z) ||
        !isfinite(r.w))
      r = make_float4(-FLT_MAX, -FLT_MAX, FLT_MAX, FLT_MAX);
    put_rect(rect, Q, q, r, lane);
  }
}

// ----------------------------------------------------------------- select --
// Candidate segments of a query: intersecting runs (ids, positions by id)
// and covering leaves (a range of the sorted order).  Segments are taken 64
// at a time (lane i holds segment i's start and length), their elements
// 64 at a time across segment boundaries.
struct KnnIn {
  const uint32_t *q_ioff, *slot_sq, *res_ids, *q_coff, *cov_leaf, *leaf_beg, *sid, *qpos;
  const uint64_t *res_off;
  const float2 *pos, *sxy;
};

// Adds the elements of up to 64 segments; lane i: segment i's start and
// length (0 past the last).  run: elements are ids in res_ids (positions by
// id), else indices of the sorted order.  Returns the number of elements.
__device__ __forceinline__ uint64_t add_segments(const KnnIn &I, uint64_t beg, uint32_t len,
                                                 bool run, float x, float y, uint32_t k,
                                                 uint32_t lane, uint64_t *best) {
  const uint32_t inc = wave_incl_scan<uint32_t>(len);  // per query: below 2^32 candidates
  const uint32_t tot = (uint32_t)__shfl((int)inc, kWave - 1, kWave);
  for (uint32_t e0 = 0; e0 < tot; e0 += kWave) {
    const uint32_t e = e0 + lane;
    // segment of element e: the number of segments whose inclusive end is <= e
    uint32_t j = 0;
#pragma unroll
    for (uint32_t step = 32; step > 0; step >>= 1) {
      const uint32_t t = j + step - 1u;
      if ((uint32_t)__shfl((int)inc, (int)t, kWave) <= e) j += step;
    }
    uint64_t key = kNoKey;
    const uint32_t jj = j < (uint32_t)kWave ? j : (uint32_t)kWave - 1u;
    const uint32_t sb = (uint32_t)__shfl((int)inc, (int)jj, kWave) -
                        (uint32_t)__shfl((int)len, (int)jj, kWave);
    const uint64_t b = shfl_u64(beg, (int)jj);
    if (e < tot) {
      const uint64_t idx = b + (e - sb);
      if (run) {
        const uint32_t id = I.res_ids[idx];
        key = knn_key(knn_d2(I.pos[id], x, y), id);
      } else {
        key = knn_key(knn_d2(I.sxy[idx], x, y), I.sid[idx]);
      }
    }
    *best = topk_add(*best, key, k, lane);
  }
  return tot;
}

__device__ __forceinline__ void knn_store(uint64_t best, uint32_t k, uint32_t q, uint32_t lane,
                                          uint32_t *out_id, float *out_d2) {
  if (lane < k) {
    const bool none = best == kNoKey;
    out_id[(uint64_t)q * k + lane] = none ? 0xffffffffu : (uint32_t)best;
    out_d2[(uint64_t)q * k + lane] = none ? INFINITY : __uint_as_float((uint32_t)(best >> 32));
  }
}

__global__ void __launch_bounds__(kBlock) k_knn_select(
    Ctl *ctl, const TickIn *tin, const float *qx, const float *qy, uint32_t nq, uint32_t N,
    const uint64_t *qstamp, KnnIn I, const float *rect, uint32_t Q, uint32_t k,
    uint32_t *out_id, float *out_d2, uint32_t *fb) {
  const uint32_t lane = lane_id();
  const uint32_t nw = gridDim.x * kWavesPerBlock;
  const bool ok = ctl->go_join != 0;
  const uint64_t seq = ctl->qry_seq - nq;  // after the write pass
  const uint32_t *__restrict__ qid = tin->qid;
  for (uint32_t q = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; q < nq; q += nw) {
    const float x = qx[q], y = qy[q];
    uint64_t best = kNoKey;
    if (!ok || !knn_live(seq, qstamp, qid[q], N, q) || !isfinite(x) || !isfinite(y)) {
      knn_store(best, k, q, lane, out_id, out_d2);
      continue;
    }
    uint64_t n = 0;
    const uint32_t pq = I.qpos[q];  // the query's processing position: its slots
    const uint32_t s0 = I.q_ioff[pq], s1 = I.q_ioff[pq + 1];
    for (uint32_t s = s0; s < s1; s += kWave) {
      uint64_t b = 0;
      uint32_t len = 0;
      if (s + lane < s1) {
        const uint32_t i = I.slot_sq[s + lane];
        b = I.res_off[i];
        len = (uint32_t)(I.res_off[i + 1] - b);
      }
      n += add_segments(I, b, len, true, x, y, k, lane, &best);
    }
    const uint32_t c0 = I.q_coff[pq], c1 = I.q_coff[pq + 1];
    for (uint32_t c = c0; c < c1; c += kWave) {
      uint64_t b = 0;
      uint32_t len = 0;
      if (c + lane < c1) {
        const uint32_t L = I.cov_leaf[c + lane];
        b = I.leaf_beg[L];
        len = I.leaf_beg[L + 1] - (uint32_t)b;
      }
      n += add_segments(I, b, len, false, x, y, k, lane, &best);
    }
    // completeness: every object outside the square has d2 >= lb
    const float4 r = make_float4(rect[q], rect[(uint64_t)Q + q], rect[2ull * Q + q],
                                 rect[3ull * Q + q]);
    const bool all = r.x == -FLT_MAX && r.y == -FLT_MAX && r.z == FLT_MAX && r.w == FLT_MAX;
    const float ex = fminf(__fsub_rn(x, r.x), __fsub_rn(r.z, x));
    const float ey = fminf(__fsub_rn(y, r.y), __fsub_rn(r.w, y));
    const float lb = fminf(__fmul_rn(ex, ex), __fmul_rn(ey, ey));
    const float d2k = __uint_as_float((uint32_t)(shfl_u64(best, (int)(k - 1u)) >> 32));
    const bool done = all || (n >= k && ex >= 0.0f && ey >= 0.0f && d2k < lb);
    if (done) {
      knn_store(best, k, q, lane, out_id, out_d2);
    } else if (lane == 0) {
      fb[atomicAdd(&ctl->n_knn_fb, 1u)] = q;
    }
  }
}

// --------------------------------------------------------------- fallback --
__global__ void __launch_bounds__(kBlock) k_knn_fallback(const Ctl *ctl, const float *qx,
                                                         const float *qy, const float2 *sxy,
                                                         const uint32_t *sid, uint32_t k,
                                                         const uint32_t *fb, uint32_t *out_id,
                                                         float *out_d2) {
  const uint32_t lane = lane_id();
  const uint32_t nw = gridDim.x * kWavesPerBlock;
  const uint32_t nf = ctl->n_knn_fb, np = ctl->n_present;
  for (uint32_t f = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; f < nf; f += nw) {
    const uint32_t q = fb[f];
    const float x = qx[q], y = qy[q];
    uint64_t best = kNoKey;
    for (uint32_t i0 = 0; i0 < np; i0 += kWave) {
      const uint32_t i = i0 + lane;
      const uint64_t key = i < np ? knn_key(knn_d2(sxy[i], x, y), sid[i]) : kNoKey;
      best = topk_add(best, key, k, lane);
    }
    knn_store(best, k, q, lane, out_id, out_d2);
  }
}

__global__ void k_knn_reset(Ctl *ctl) { ctl->n_knn_fb = 0; }

#define LAUNCH(kern, grid, block, stream, ...) \
  hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, stream, __VA_ARGS__)

static unsigned wave_grid(uint32_t n) {
  const uint32_t b = (n + kWavesPerBlock - 1u) / kWavesPerBlock;
  return b < 1u ? 1u : (b > 8192u ? 8192u : b);
}

void launch_knn_radius(const Bufs &B, const float *qx, const float *qy, uint32_t nq, uint32_t k,
                       hipStream_t s) {
  LAUNCH(k_knn_reset, 1, 1, s, B.ctl);
  if (!nq) return;
  LAUNCH(k_knn_radius, wave_grid(nq), kBlock, s, (const Ctl *)B.ctl, (const TickIn *)B.tin, qx,
         qy, nq, B.N, (const uint64_t *)B.qstamp, tree_of(B), (const uint32_t *)B.leaf_beg,
         (const float2 *)B.sxy, k, B.kq_rect, B.Q);
}

void launch_knn_select(const Bufs &B, const float *qx, const float *qy, uint32_t nq, uint32_t k,
                       uint32_t *out_id, float *out_d2, hipStream_t s) {
  if (!nq) return;
  KnnIn I{B.q_ioff, B.slot_sq, B.res_ids, B.q_coff, B.cov_leaf, B.leaf_beg, B.valA, B.qpos,
          B.res_off, (const float2 *)B.pos, (const float2 *)B.sxy};
  LAUNCH(k_knn_select, wave_grid(nq), kBlock, s, B.ctl, (const TickIn *)B.tin, qx, qy, nq, B.N,
         (const uint64_t *)B.qstamp, I, (const float *)B.kq_rect, B.Q, k, out_id, out_d2,
         B.kq_fb);
  LAUNCH(k_knn_fallback, 64, kBlock, s, (const Ctl *)B.ctl, qx, qy, (const float2 *)B.sxy,
         (const uint32_t *)B.valA, k, (const uint32_t *)B.kq_fb, out_id, out_d2);
}

}  // namespace sj
