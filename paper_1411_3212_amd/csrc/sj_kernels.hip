// Kernels of the per-tick spatial join (gfx950, wave64).
//
// Pipeline of one tick (paper Section "Query processing pipeline"):
//   updates      last-writer-wins scatter of (id, x, y) into positions by id
//   index        MBR -> frame -> Morton codes -> LDS-staged radix sort whose
//                last pass also gathers the positions in sorted order
//                (index creation, first steps of Algorithm 1)
//   build        level-wise PR-quadtree split under the threshold, leaves in
//                Morton order, node table and a start table at level
//                min(l_deep, 8) (the paper's z_map, capped) for queries
//                (Algorithm 1; only on ticks that build)
//   leaves       object range of every leaf in the sorted order
//   split        per query: the leaves it touches, intersecting / covering;
//                count -> exclusive scans -> write, subqueries grouped by
//                leaf (query indexing and sorting of subqueries)
//   schedule     leaves ordered by decreasing log2 of their weight
//                |intersecting subqueries| x |objects| (task scheduling)
//   join         one wave per leaf: ballot of the closed containment test
//                per intersecting subquery; count -> scan -> write of ids
//                (filtering with bitmaps + decoding)
// Sums and maxima go through per-block partials reduced by the single-block
// kernels of the pipeline (no same-address atomics from every block).
#include "sj_device.h"
#include "sj_kernels.h"
#include "sj_tree.h"

namespace sj {

constexpr uint32_t kTableScanMax = 1024;  // queries over more table cells start at the root
// ------------------------------------------------------------- utilities --

__global__ void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_u64(uint64_t *p, uint64_t n, uint64_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_ctl_init(Ctl *ctl, uint32_t th, uint32_t ug_split, uint32_t ug_bits,
                           uint32_t policy) {
  Ctl c;
  uint8_t *b = (uint8_t *)&c;
  for (unsigned i = 0; i < sizeof(Ctl); ++i) b[i] = 0;
  c.th_cur = th;
  c.policy = policy;
  c.b_cost = -1.0f;
  c.scale = 65536.0f;
  c.ug_split = ug_split;
  c.ug_bits = ug_bits;
  *ctl = c;
}

__global__ void k_request_build(Ctl *ctl, uint32_t th) {
  ctl->force = 1u;
  if (th) ctl->th_next = th;
}


// --------------------------------------------------------------- updates --
// Tick batching: within a tick the most recent update of an object wins.
// Update k of a call gets the sequence number upd_seq + seq_off + k + 1
// (seq_off: updates of earlier calls in the same tick; upd_seq advances by
// the tick's total when the tick runs); an atomic max per object keeps the
// latest, then only that one is written.

__global__ void __launch_bounds__(kBlock) k_upd_stamp(const TickIn *tin, uint32_t m, uint32_t N,
                                                      uint64_t seq_off, uint64_t *stamp,
                                                      Ctl *ctl) {
  const uint32_t *__restrict__ id = tin->id;
  const float *__restrict__ x = tin->x, *__restrict__ y = tin->y;
  const uint64_t seq = ctl->upd_seq + seq_off;
  const uint32_t mr = (m + kWave - 1) / kWave * kWave;
  for (uint32_t k = blockIdx.x * kBlock + threadIdx.x; k < mr; k += gridDim.x * kBlock) {
    bool bad_id = false, bad_xy = false;
    if (k < m) {
      const uint32_t o = id[k];
      const float xv = x[k], yv = y[k];
      bad_id = o >= N;
      bad_xy = !bad_id && !(isfinite(xv) && isfinite(yv));
      if (!bad_id && !bad_xy)
        atomicMax((unsigned long long *)&stamp[o], (unsigned long long)(seq + k + 1));
    }
    const uint64_t mi = ballot(bad_id), mx = ballot(bad_xy);
    if ((mi | mx) && lane_id() == 0)
      atomicOr(&ctl->err_upd, (mi ? kErrUpdId : 0u) | (mx ? kErrUpdCoord : 0u));
  }
}

__global__ void __launch_bounds__(kBlock) k_upd_write(const TickIn *tin, uint32_t m, uint32_t N,
                                                      uint64_t seq_off, const uint64_t *stamp,
                                                      const Ctl *ctl, float2 *pos) {
  const uint32_t *__restrict__ id = tin->id;
  const float *__restrict__ x = tin->x, *__restrict__ y = tin->y;
  const uint64_t seq = ctl->upd_seq + seq_off;
  for (uint32_t k = blockIdx.x * kBlock + threadIdx.x; k < m; k += gridDim.x * kBlock) {
    const uint32_t o = id[k];
    if (o < N && stamp[o] == seq + k + 1) pos[o] = make_float2(x[k], y[k]);
  }
}

// ----------------------------------------------------------------- index --

// Per block of ids: present count (position not NaN), MBR and number of
// present objects outside the current frame, as partials.
__global__ void __launch_bounds__(kBlock) k_mbr(const float2 *pos, uint32_t N, const Ctl *ctl,
                                                uint32_t *blk, uint64_t *red) {
  __shared__ float s_mnx[kWavesPerBlock], s_mny[kWavesPerBlock], s_mxx[kWavesPerBlock],
      s_mxy[kWavesPerBlock];
  __shared__ uint32_t s_cnt[kWavesPerBlock], s_out[kWavesPerBlock];
  const uint32_t chunk = (N + gridDim.x - 1) / gridDim.x;
  const uint64_t b0 = (uint64_t)blockIdx.x * chunk;
  const uint64_t b1 = b0 + chunk < N ? b0 + chunk : N;
  const bool built = ctl->built != 0;
  const float x0 = ctl->x0, y0 = ctl->y0, sc = ctl->scale;
  float mnx = INFINITY, mny = INFINITY, mxx = -INFINITY, mxy = -INFINITY;
  uint32_t cnt = 0, out = 0;
  // four rows of loads in flight per thread (positions past the chunk read
  // as absent)
  constexpr uint32_t kRows = 4;
  for (uint64_t t0 = b0; t0 < b1; t0 += kBlock * kRows) {
    float2 p[kRows];
#pragma unroll
    for (uint32_t j = 0; j < kRows; ++j) {
      const uint64_t i = t0 + j * kBlock + threadIdx.x;
      p[j] = i < b1 ? pos[i] : make_float2(NAN, NAN);
    }
#pragma unroll
    for (uint32_t j = 0; j < kRows; ++j) {
      const float xv = p[j].x, yv = p[j].y;
      if (xv == xv) {
        ++cnt;
        mnx = fminf(mnx, xv);
        mxx = fmaxf(mxx, xv);
        mny = fminf(mny, yv);
        mxy = fmaxf(mxy, yv);
        if (built) {
          const float tx = __fmul_rn(__fsub_rn(xv, x0), sc),
                      ty = __fmul_rn(__fsub_rn(yv, y0), sc);
          out += !(tx >= 0.0f && tx < 65536.0f && ty >= 0.0f && ty < 65536.0f);
        }
      }
    }
  }
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    mnx = fminf(mnx, __shfl_xor(mnx, o, kWave));
    mny = fminf(mny, __shfl_xor(mny, o, kWave));
    mxx = fmaxf(mxx, __shfl_xor(mxx, o, kWave));
    mxy = fmaxf(mxy, __shfl_xor(mxy, o, kWave));
  }
  cnt = wave_sum(cnt);
  out = wave_sum(out);
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) {
    s_mnx[w] = mnx; s_mny[w] = mny; s_mxx[w] = mxx; s_mxy[w] = mxy;
    s_cnt[w] = cnt; s_out[w] = out;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < kWavesPerBlock; ++i) {
      mnx = fminf(mnx, s_mnx[i]); mny = fminf(mny, s_mny[i]);
      mxx = fmaxf(mxx, s_mxx[i]); mxy = fmaxf(mxy, s_mxy[i]);
      cnt += s_cnt[i]; out += s_out[i];
    }
    const uint32_t b = blockIdx.x;
    blk[b] = cnt;
    red[kRedMinX * kChunkBlocks + b] = cnt ? fenc(mnx) : 0xffffffffu;
    red[kRedMinY * kChunkBlocks + b] = cnt ? fenc(mny) : 0xffffffffu;
    red[kRedMaxX * kChunkBlocks + b] = cnt ? fenc(mxx) : 0u;
    red[kRedMaxY * kChunkBlocks + b] = cnt ? fenc(mxy) : 0u;
    red[kRedOutside * kChunkBlocks + b] = out;
  }
}

// Side exponent of the frame: smallest e >= -100 with 2^e >= m.
__device__ __forceinline__ int32_t frame_exp(float m) {
  if (!(m > 0.0f)) return -100;
  const uint32_t b = __float_as_uint(m);
  const int32_t ex = (int32_t)((b >> 23) & 0xffu);
  if (ex == 0) return -100;
  int32_t e = ex - 127 + ((b & 0x7fffffu) ? 1 : 0);
  return e < -100 ? -100 : e;
}

template <bool MAX>
__device__ __forceinline__ uint32_t block_minmax_1024(uint32_t v, uint32_t *lds) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const uint32_t u = __shfl_xor(v, o, kWave);
    v = MAX ? (u > v ? u : v) : (u < v ? u : v);
  }
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) lds[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < kChunkBlocks / kWave; ++i)
      v = MAX ? (lds[i] > v ? lds[i] : v) : (lds[i] < v ? lds[i] : v);
    lds[0] = v;
  }
  __syncthreads();
  v = lds[0];
  __syncthreads();
  return v;
}

// Start of a tick (one block of 1024 threads): MBR from the partials,
// offsets of the present objects per block, rebuild decision, frame, reset
// of the tick's counters.  decision: 0 keep the quadtree, 1 build it, 2 let
// the automatic policy decide (the host launches the build kernels for 1
// and 2; they do nothing unless ctl->rebuild is set).
__global__ void __launch_bounds__(kChunkBlocks) k_decide(Ctl *ctl, uint32_t *blk,
                                                         const uint64_t *red, uint4 *front0,
                                                         uint32_t *tkhist, uint32_t decision,
                                                         uint32_t policy, uint64_t upd_total) {
  __shared__ uint32_t lds[kChunkBlocks / kWave + 1];
  const int t = threadIdx.x;
  if (t < 512) tkhist[t] = 0;  // task-order totals and cursors of this tick
  // every partial is loaded before the first reduction waits on a barrier
  const uint32_t p_mnx = (uint32_t)red[kRedMinX * kChunkBlocks + t];
  const uint32_t p_mny = (uint32_t)red[kRedMinY * kChunkBlocks + t];
  const uint32_t p_mxx = (uint32_t)red[kRedMaxX * kChunkBlocks + t];
  const uint32_t p_mxy = (uint32_t)red[kRedMaxY * kChunkBlocks + t];
  const uint32_t p_out = (uint32_t)red[kRedOutside * kChunkBlocks + t];
  const uint32_t p_cnt = blk[t];
  const uint32_t mnx = block_minmax_1024<false>(p_mnx, lds);
  const uint32_t mny = block_minmax_1024<false>(p_mny, lds);
  const uint32_t mxx = block_minmax_1024<true>(p_mxx, lds);
  const uint32_t mxy = block_minmax_1024<true>(p_mxy, lds);
  uint32_t outside;
  block_excl_scan<uint32_t, kChunkBlocks>(p_out, lds, &outside);
  uint32_t total;
  const uint32_t ex = block_excl_scan<uint32_t, kChunkBlocks>(p_cnt, lds, &total);
  blk[t] = ex;
  if (t != 0) return;
  ctl->err = ctl->err_upd;
  ctl->err_upd = 0;
  ctl->upd_seq += upd_total;
  ctl->n_present = total;
  ctl->n_outside = outside;
  ctl->go_split = 0;
  ctl->go_join = 0;
  ctl->n_isect = ctl->n_cov = ctl->n_res = ctl->cov_pairs = ctl->tests = 0;
  ctl->n32[0] = ctl->n32[1] = 0;
  ctl->n_tasks = 0;
  ctl->n_run = 0;
  ctl->max_leaf = 0;
  bool r;
  if (decision == 0u)
    r = false;
  else if (decision == 1u)
    r = true;
  else
    r = ctl->force || !ctl->built || policy == 1u ||
        ((policy == 0u || policy == 3u) && ctl->want_rebuild);
  ctl->rebuild = r ? 1u : 0u;
  ctl->t_start = __builtin_amdgcn_s_memrealtime();
  if (!r) {
    ctl->since_build += 1;
    // leaf keys are below n_leaves: the radix passes above their width
    // have nothing to sort (at least one pass gathers the positions)
    const uint32_t nl = ctl->n_leaves;
    const uint32_t bits = nl > 1u ? 32u - (uint32_t)__clz((int)(nl - 1u)) : 0u;
    const uint32_t w = (bits + 7u) / 8u * 8u;
    ctl->sort_skip = w < 8u ? 8u : w;
    return;
  }
  ctl->sort_skip = 32u;
  if (ctl->th_next) ctl->th_cur = ctl->th_next;
  ctl->th_next = 0;
  ctl->force = 0;
  ctl->built = 1;
  ctl->since_build = 0;
  float x0 = 0.0f, y0 = 0.0f;
  int32_t e = 0;
  if (total) {
    x0 = fdec(mnx);
    y0 = fdec(mny);
    const float w = __fsub_rn(fdec(mxx), x0), h = __fsub_rn(fdec(mxy), y0);
    e = frame_exp(w > h ? w : h);
  }
  ctl->x0 = x0;
  ctl->y0 = y0;
  ctl->e = e;
  ctl->scale = __uint_as_float((uint32_t)(127 + kFine - e) << 23);
  for (int l = 0; l < kFine + 2; ++l) ctl->fcount[l] = 0;
  ctl->fcount[0] = 1;
  ctl->n_leaves = 0;
  ctl->l_deep = 0;
  front0[0] = make_uint4(0u, 0u, total, 0u);
  if (ctl->ug_split) {
    // uniform grid: every cell of the Morton range is a leaf, the sort keys
    // (cell codes) are below 4^ug_bits
    const uint32_t b = ctl->ug_bits;
    ctl->n_leaves = 1u << (2u * b);
    ctl->l_deep = b;
    ctl->sort_skip = (2u * b + 7u) / 8u * 8u < 8u ? 8u : (2u * b + 7u) / 8u * 8u;
  }
}

// Sort keys of present objects, compacted in id order with their ids and
// positions (which the sort carries along): their Morton codes when the
// tick builds the quadtree, else the index of the leaf holding them (the
// leaves are in Morton order, so grouping by leaf is what the join needs,
// and leaf indices take fewer radix digits than codes).  Then
// the sequence stamps of the tick's queries (the latest query of an object
// is the one answered).
__global__ void __launch_bounds__(kBlock) k_morton(const float2 *pos, uint32_t N, Tree tr,
                                                   Ctl *ctl, const uint32_t *blk, uint32_t *keys,
                                                   uint32_t *vals, float2 *cpos,
                                                   const TickIn *tin, uint32_t nq,
                                                   uint64_t *qstamp) {
  // A tile is kMortonRows rows of kBlock ids: every row's loads and table
  // lookups are issued before the first is waited for, and one block scan
  // ranks all rows (one 16-bit field per row).
  constexpr uint32_t kMortonRows = 4;
  __shared__ uint64_t lds[kWavesPerBlock + 1];
  const uint32_t chunk = (N + gridDim.x - 1) / gridDim.x;
  const uint64_t b0 = (uint64_t)blockIdx.x * chunk;
  const uint64_t b1 = b0 + chunk < N ? b0 + chunk : N;
  const float x0 = ctl->x0, y0 = ctl->y0, sc = ctl->scale;
  const bool keep = !ctl->rebuild;  // the quadtree is kept: sort by leaf
  const uint32_t ug = ctl->ug_split;  // uniform grid: sort by grid cell
  tr.tlev = ctl->tlev;
  uint32_t base = blk[blockIdx.x];
  for (uint64_t t0 = b0; t0 < b1; t0 += kBlock * kMortonRows) {
    float2 p[kMortonRows];
    uint32_t key[kMortonRows];
    uint64_t flags = 0;
#pragma unroll
    for (uint32_t j = 0; j < kMortonRows; ++j) {
      const uint64_t i = t0 + j * kBlock + threadIdx.x;
      p[j] = i < b1 ? pos[i] : make_float2(NAN, NAN);
    }
#pragma unroll
    for (uint32_t j = 0; j < kMortonRows; ++j) {
      const bool pres = p[j].x == p[j].x;
      flags |= (uint64_t)(pres ? 1u : 0u) << (16u * j);
      const uint32_t ci = cell_of(p[j].x, x0, sc), cj = cell_of(p[j].y, y0, sc);
      key[j] = !pres ? 0u : ug ? morton2(ug_col(ci, ug), ug_col(cj, ug)) : morton2(ci, cj);
    }
    if (keep) {
      uint32_t e[kMortonRows];
#pragma unroll
      for (uint32_t j = 0; j < kMortonRows; ++j)
        e[j] = (flags >> (16u * j)) & 1u ? table_entry(tr, key[j]) : kLeafBit;
#pragma unroll
      for (uint32_t j = 0; j < kMortonRows; ++j) key[j] = leaf_from(tr, e[j], key[j]);
    }
    uint64_t tot;
    const uint64_t ex = block_excl_scan<uint64_t, kBlock>(flags, lds, &tot);
#pragma unroll
    for (uint32_t j = 0; j < kMortonRows; ++j) {
      if ((flags >> (16u * j)) & 1u) {
        const uint32_t r = base + (uint32_t)((ex >> (16u * j)) & 0xffffu);
        keys[r] = key[j];
        vals[r] = (uint32_t)(t0 + j * kBlock + threadIdx.x);
        cpos[r] = p[j];
      }
      base += (uint32_t)((tot >> (16u * j)) & 0xffffu);
    }
  }
  const uint64_t seq = ctl->qry_seq;
  const uint32_t *__restrict__ qid = tin->qid;
  const uint32_t nr = (nq + kWave - 1) / kWave * kWave;
  for (uint32_t k = blockIdx.x * kBlock + threadIdx.x; k < nr; k += gridDim.x * kBlock) {
    bool bad = false;
    if (k < nq) {
      const uint32_t o = qid[k];
      bad = o >= N;
      if (!bad) atomicMax((unsigned long long *)&qstamp[o], (unsigned long long)(seq + k + 1));
    }
    flag_error(ctl, kErrQueryId, bad);
  }
}

// ----------------------------------------------------------------- build --
// Algorithm 1 on the device: the frontier of level l-1 holds the quadrants
// to split as intervals of the sorted codes; each is cut into its four
// level-l children (one wave per quadrant); a child with more than th
// objects below l_max joins the next frontier, every other child (empty
// ones included) becomes a leaf.

// First index in [lo, hi) whose code is >= key (hi if none), by the whole
// wave: 63 lanes probe evenly spaced positions and a ballot keeps the
// interval that holds the answer, so a range of n codes takes about
// log64(n) dependent loads.  Every lane returns the same value.
__device__ __forceinline__ uint32_t wave_lower_bound(const uint32_t *codes, uint32_t lo,
                                                     uint32_t hi, uint32_t key) {
  const uint32_t lane = lane_id();
  while (hi - lo > (uint32_t)kWave) {
    const uint64_t span = hi - lo;
    const uint32_t p = lo + (uint32_t)((span * (lane + 1u)) >> 6);  // lo < p < hi for lane < 63
    const bool ge = lane < (uint32_t)kWave - 1u && codes[p] >= key;
    const uint64_t m = ballot(ge);
    const uint32_t f = m ? (uint32_t)__ffsll((unsigned long long)m) - 1u : (uint32_t)kWave - 1u;
    const uint32_t pf = (uint32_t)readlane_i((int)p, (int)f);
    const uint32_t pb = f ? (uint32_t)readlane_i((int)p, (int)f - 1) : 0u;
    const uint32_t nlo = f ? pb + 1u : lo;
    hi = f < (uint32_t)kWave - 1u ? pf : hi;
    lo = nlo;
  }
  const bool ge = lo + lane < hi && codes[lo + lane] >= key;
  const uint64_t m = ballot(ge);
  return m ? lo + (uint32_t)__ffsll((unsigned long long)m) - 1u : hi;
}

// Quadrants per level up to which a whole wave splits each quadrant (the top
// levels: few quadrants over long code ranges); below it a lane per quadrant
// (many short ranges, one append per wave).
constexpr uint32_t kWaveSplitMax = 1024;

__global__ void __launch_bounds__(kBlock) k_tree_level(Ctl *ctl, uint32_t l, uint32_t l_max,
                                                       const uint32_t *codes, const uint4 *fin,
                                                       uint4 *fout, uint32_t fcap,
                                                       uint32_t *lstart, uint32_t *llevel,
                                                       uint32_t lcap) {
  if (!ctl->rebuild) return;
  const uint32_t F = min(ctl->fcount[l - 1], fcap);
  if (F == 0) return;
  const uint32_t th = ctl->th_cur;
  const uint32_t shift = 2u * (kFine - l);
  const uint32_t lane = lane_id();
  bool ovf = false;
  uint32_t deep = 0;
  if (F <= kWaveSplitMax) {
    const uint32_t nwaves = gridDim.x * kWavesPerBlock;
    const uint32_t w0 =
        __builtin_amdgcn_readfirstlane(blockIdx.x * kWavesPerBlock + threadIdx.x / kWave);
    for (uint32_t f = w0; f < F; f += nwaves) {
      const uint4 e = fin[f];
      const uint32_t zp = e.x, b0 = e.y, b4 = e.z;
      // boundaries of the four children: one ballot round when the quadrant
      // holds at most a wave of codes, else three wave searches
      uint32_t bnd[5];
      bnd[0] = b0;
      bnd[4] = b4;
      if (b4 - b0 <= (uint32_t)kWave) {
        const bool v = b0 + lane < b4;
        const uint32_t d = v ? (codes[b0 + lane] >> shift) & 3u : 4u;
#pragma unroll
        for (uint32_t k = 1; k < 4; ++k) bnd[k] = b0 + (uint32_t)__popcll(ballot(d < k));
      } else {
#pragma unroll
        for (uint32_t k = 1; k < 4; ++k)
          bnd[k] = wave_lower_bound(codes, bnd[k - 1], b4, (zp * 4u + k) << shift);
      }
      // lane k < 4 decides child k
      const bool child = lane < 4u;
      uint32_t lo = 0, hi = 0;
#pragma unroll
      for (uint32_t k = 0; k < 4; ++k)
        if (lane == k) {
          lo = bnd[k];
          hi = bnd[k + 1];
        }
      const bool sp = child && hi - lo > th && l < l_max;
      const bool lf = child && !sp;
      const uint32_t fb = wave_append(&ctl->fcount[l], sp ? 1u : 0u);
      const uint32_t lb = wave_append(&ctl->n_leaves, lf ? 1u : 0u);
      const uint32_t cz = zp * 4u + lane;
      if (sp) {
        if (fb < fcap)
          fout[fb] = make_uint4(cz, lo, hi, 0u);
        else
          ovf = true;
      } else if (lf) {
        if (lb < lcap) {
          lstart[lb] = cz << shift;
          llevel[lb] = l;
        } else {
          ovf = true;
        }
      }
      if (ballot(lf)) deep = l;
    }
  } else {
    const uint32_t nthreads = gridDim.x * kBlock;
    const uint32_t Fr = (F + kWave - 1) / kWave * kWave;
    for (uint32_t f = blockIdx.x * kBlock + threadIdx.x; f < Fr; f += nthreads) {
      const bool valid = f < F;
      uint32_t zp = 0, bnd[5] = {0, 0, 0, 0, 0}, nsplit = 0, nleaf = 0, splitm = 0;
      if (valid) {
        const uint4 e = fin[f];
        zp = e.x;
        bnd[0] = e.y;
        bnd[4] = e.z;
        for (uint32_t k = 1; k < 4; ++k)
          bnd[k] = lower_bound_u32(codes, bnd[k - 1], bnd[4], (zp * 4u + k) << shift);
        for (uint32_t k = 0; k < 4; ++k) {
          const bool sp = bnd[k + 1] - bnd[k] > th && l < l_max;
          splitm |= (sp ? 1u : 0u) << k;
          nsplit += sp;
          nleaf += !sp;
        }
      }
      uint32_t fb = wave_append(&ctl->fcount[l], nsplit);
      uint32_t lb = wave_append(&ctl->n_leaves, nleaf);
      if (valid) {
        for (uint32_t k = 0; k < 4; ++k) {
          const uint32_t cz = zp * 4u + k;
          if ((splitm >> k) & 1u) {
            if (fb < fcap)
              fout[fb] = make_uint4(cz, bnd[k], bnd[k + 1], 0u);
            else
              ovf = true;
            ++fb;
          } else {
            if (lb < lcap) {
              lstart[lb] = cz << shift;
              llevel[lb] = l;
            } else {
              ovf = true;
            }
            ++lb;
          }
        }
      }
      if (ballot(nleaf != 0)) deep = l;
    }
  }
  flag_error(ctl, kErrOvfTree, ovf);
  if (deep && lane == 0) atomicMax(&ctl->l_deep, deep);
}

// The leaf table is sized for the worst case of the smallest threshold, so
// this never fires; if it did, the tick is flagged and no traversal runs.
// Start-table level: about four levels below the depth of a uniform tree
// with th objects per leaf for the capacity n_cap, within [4, 12], the
// allocated level tcap and the deepest leaf.
__global__ void k_tree_done(Ctl *ctl, uint32_t lcap, uint32_t tcap, uint32_t n_cap) {
  if (!ctl->rebuild) return;
  if (ctl->n_leaves > lcap) {
    ctl->n_leaves = lcap;
    ctl->err |= kErrOvfTree;
  }
  const uint64_t per = (uint64_t)n_cap / ((uint64_t)ctl->th_cur + 1u);
  uint32_t lu = 0;
  for (uint64_t c = 1; c < per; c *= 4u) ++lu;
  uint32_t t = lu + 4u > 12u ? 12u : lu + 4u;
  t = t < tcap ? t : tcap;
  ctl->tlev = ctl->l_deep < t ? ctl->l_deep : t;
}

__device__ __forceinline__ uint32_t open_level(uint32_t s) {
  return s == 0u ? 0u : (uint32_t)kFine - (uint32_t)((__ffs(s) - 1) >> 1);
}

// Internal nodes in depth-first order from the Morton-sorted leaves: leaf t
// starts the nodes at levels open_level(start) .. level(t)-1.
__global__ void __launch_bounds__(kBlock) k_nodes_open(const Ctl *ctl, const uint32_t *lstart,
                                                       const uint32_t *llevel, uint32_t *nopen) {
  if (!ctl->rebuild) return;
  const uint32_t n = ctl->n_leaves;
  for (uint32_t t = blockIdx.x * kBlock + threadIdx.x; t < n; t += gridDim.x * kBlock)
    nopen[t] = llevel[t] - open_level(lstart[t]);
}

// One thread per internal node: its leaf t (the last leaf whose first node
// index is <= the node's) and level, then the four children's leaves by four
// interleaved branchless binary searches over the leaf starts, so the
// longest dependent chain is two searches whatever the depth.
__global__ void __launch_bounds__(kBlock) k_nodes_build(Ctl *ctl, const uint32_t *lstart,
                                                        const uint32_t *llevel,
                                                        const uint32_t *node_off, uint4 *nodes,
                                                        uint32_t ncap) {
  if (!ctl->rebuild) return;
  const uint32_t n = ctl->n_leaves;
  if (n == 0) return;
  const uint32_t total = node_off[n];
  bool bad = false;
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < total; i += gridDim.x * kBlock) {
    // t: last index with node_off[t] <= i (node_off[0] = 0 <= i)
    uint32_t base = 0, len = n;
    while (len > 1) {
      const uint32_t half = len >> 1;
      base = node_off[base + half] <= i ? base + half : base;
      len -= half;
    }
    const uint32_t t = base, s = lstart[t], k0 = open_level(s);
    const uint32_t k = k0 + (i - node_off[t]);
    const uint32_t p = k == 0 ? 0u : s >> (2u * (kFine - k));
    uint32_t key[4], b4[4];
#pragma unroll
    for (uint32_t c = 0; c < 4; ++c) {
      key[c] = (p * 4u + c) << (2u * (kFine - k - 1));
      b4[c] = 0;
    }
    for (uint32_t l2 = n; l2 > 1;) {
      const uint32_t half = l2 >> 1;
#pragma unroll
      for (uint32_t c = 0; c < 4; ++c) b4[c] = lstart[b4[c] + half] < key[c] ? b4[c] + half : b4[c];
      l2 -= half;
    }
    uint32_t ref[4];
#pragma unroll
    for (uint32_t c = 0; c < 4; ++c) {
      const uint32_t u = b4[c] + (lstart[b4[c]] < key[c] ? 1u : 0u);  // first start >= key
      if (u >= n || lstart[u] != key[c]) {
        bad = true;
        ref[c] = kLeafBit;
        continue;
      }
      const uint32_t lu = llevel[u];
      ref[c] = lu == k + 1 ? (kLeafBit | u) : node_off[u] + (k + 1 - open_level(key[c]));
    }
    if (i < ncap)
      nodes[i] = make_uint4(ref[0], ref[1], ref[2], ref[3]);
    else
      bad = true;
  }
  flag_error(ctl, kErrOvfTree, bad);
}

// Start table at level T = min(l_deep, cap) in Morton order (the paper's
// z_map, with its depth capped): for every level-T cell, the leaf that
// contains it when that leaf is at a level <= T (entry: flag, level - 1,
// leaf index), otherwise the internal node at level T (entry: node index).
__global__ void __launch_bounds__(kBlock) k_table_build(const Ctl *ctl, const uint32_t *lstart,
                                                        const uint32_t *llevel,
                                                        const uint32_t *node_off,
                                                        uint32_t *table) {
  if (!ctl->rebuild || (ctl->err & kErrOvfTree)) return;
  const uint32_t T = ctl->tlev, n = ctl->n_leaves;
  const uint32_t ncell = 1u << (2 * T), sh = 2u * (kFine - T);
  const uint32_t lane = lane_id();
  const uint32_t nwaves = gridDim.x * kWavesPerBlock;
  const uint32_t w0 =
      __builtin_amdgcn_readfirstlane(blockIdx.x * kWavesPerBlock + threadIdx.x / kWave);
  // a wave takes 64 consecutive cells: the leaves holding its first and last
  // cell (the last leaf whose start is <= the cell's code) bound the search
  // of every lane
  for (uint32_t z0 = w0 * (uint32_t)kWave; z0 < ncell; z0 += nwaves * (uint32_t)kWave) {
    const uint32_t zl = min(z0 + (uint32_t)kWave, ncell) - 1u;
    uint32_t ua = wave_lower_bound(lstart, 0u, n, z0 << sh);
    if (ua == n || lstart[ua] != (z0 << sh)) --ua;
    uint32_t ub = wave_lower_bound(lstart, ua, n, zl << sh);
    if (ub == n || lstart[ub] != (zl << sh)) --ub;
    const uint32_t z = z0 + lane;
    if (z >= ncell) continue;
    const uint32_t code = T == kFine ? z : z << sh;
    uint32_t u = lower_bound_u32(lstart, ua, ub + 1u, code);
    if (u == ub + 1u || lstart[u] != code) --u;
    const uint32_t l = llevel[u];
    table[z] = l <= T ? (kLeafBit | ((l - 1u) << kLeafIdxBits) | u)
                      : node_off[u] + (T - open_level(code));
  }
}

// ---------------------------------------------------------------- leaves --

// Object range of every leaf in the sorted keys: codes after a build
// (first code >= the leaf's start), leaf indices otherwise.
__global__ void __launch_bounds__(kBlock) k_leaf_ranges(const Ctl *ctl, const uint32_t *keys,
                                                        const uint32_t *lstart,
                                                        uint32_t *leaf_beg) {
  const uint32_t n = ctl->n_leaves, np = ctl->n_present;
  // the keys are leaf indices on kept-tree ticks and grid cells (the leaves
  // of a uniform grid)
  const bool by_code = ctl->rebuild != 0 && !ctl->ug_split;
  const uint32_t stride = gridDim.x * kBlock, g = blockIdx.x * kBlock + threadIdx.x;
  // one binary search per leaf, or one pass over the sorted leaf keys when
  // leaves hold at most 48 objects on average (measured: the pass is faster
  // at 31 objects per leaf, the searches at 115); a uniform grid's Morton
  // range holds long runs of cells outside the grid (always empty), which
  // one position of the pass would fill alone, so it takes the searches
  if (by_code || ctl->ug_split || (uint64_t)np > 48ull * n) {
    for (uint32_t t = g; t < n; t += stride)
      leaf_beg[t] = lower_bound_u32(keys, 0u, np, by_code ? lstart[t] : t);
    if (g == 0) leaf_beg[n] = np;
  } else {
    // keys are ascending leaf indices: position i starts every leaf t with
    // keys[i-1] < t <= keys[i] (empty leaves included), and position np
    // every leaf after the last key, up to the end entry t = n; four
    // positions per thread and round, their loads issued together
    constexpr uint32_t kRows = 4;
    for (uint64_t i0 = g; i0 <= np; i0 += (uint64_t)stride * kRows) {
      uint32_t lo[kRows], hi[kRows];
#pragma unroll
      for (uint32_t j = 0; j < kRows; ++j) {
        const uint64_t i = i0 + (uint64_t)j * stride;
        lo[j] = i >= 1u && i <= np ? keys[i - 1] + 1u : 0u;
        hi[j] = i < np ? min(keys[i], n) : n;
      }
#pragma unroll
      for (uint32_t j = 0; j < kRows; ++j) {
        const uint64_t i = i0 + (uint64_t)j * stride;
        if (i <= np)
          for (uint32_t t = lo[j]; t <= hi[j]; ++t) leaf_beg[t] = (uint32_t)i;
      }
    }
  }
}

// ----------------------------------------------------------------- split --
// Query splitting (mapping function g): the corners are mapped through the
// same cell function as the objects (clamped to the frame).  The query's
// cells of the start table give either a leaf directly (kept once per leaf,
// at the cell with minimal coordinates, as the paper does with z_map) or
// an internal node below which a depth-first walk visits every leaf whose
// finest-level cell range overlaps the query's.  A leaf strictly inside the
// query's cell range on both axes is covering, any other is intersecting.
// Leaves without objects are skipped (they are inactive).

struct QBox {
  uint32_t i0, i1, j0, j1;
};


// Depth-first walk below internal node `node` at level depth0 with cell
// coordinates (pi, pj) at that level, one node per iteration: its children
// overlapping the query are classified at once, leaf children visited,
// and the walk descends into the first overlapping internal child, keeping
// the others as a 4-bit mask per level on the stack.
template <typename Visit>
__device__ __forceinline__ void walk_from(const uint4 *__restrict__ nodes, uint32_t *stack,
                                          uint32_t node, uint32_t depth0, uint32_t pi,
                                          uint32_t pj, const QBox q, Visit &visit) {
  uint32_t depth = depth0;
  uint4 rec = nodes[node];
  while (true) {
    const uint32_t s = (uint32_t)kFine - (depth + 1);
    const uint32_t span = (1u << s) - 1u;
    uint32_t imask = 0;
#pragma unroll
    for (uint32_t c = 0; c < 4; ++c) {
      const uint32_t ref = c == 0 ? rec.x : c == 1 ? rec.y : c == 2 ? rec.z : rec.w;
      const uint32_t ilo = (2u * pi + (c & 1u)) << s, jlo = (2u * pj + (c >> 1)) << s;
      const uint32_t ihi = ilo + span, jhi = jlo + span;
      if (!(ilo <= q.i1 && q.i0 <= ihi && jlo <= q.j1 && q.j0 <= jhi)) continue;
      if (ref & kLeafBit)
        visit(ref & ~kLeafBit, q.i0 < ilo && ihi < q.i1 && q.j0 < jlo && jhi < q.j1);
      else if (depth + 1 < (uint32_t)kFine)
        imask |= 1u << c;
    }
    if (!imask) {
      // pop to the deepest level with a pending internal child
      while (true) {
        if (depth == depth0) return;
        --depth;
        pi >>= 1;
        pj >>= 1;
        const uint32_t e = stack[depth * kBlock];
        imask = e >> 28;
        if (imask) {
          node = e & 0x0fffffffu;
          rec = nodes[node];
          break;
        }
      }
    }
    const uint32_t c = (uint32_t)__ffs(imask) - 1u;
    stack[depth * kBlock] = node | ((imask & ~(1u << c)) << 28);
    node = c == 0 ? rec.x : c == 1 ? rec.y : c == 2 ? rec.z : rec.w;
    pi = 2u * pi + (c & 1u);
    pj = 2u * pj + (c >> 1);
    ++depth;
    rec = nodes[node];
  }
}

__device__ __forceinline__ bool query_box(const Ctl *ctl, uint32_t k, uint32_t o, uint32_t N,
                                          const uint64_t *qstamp, uint64_t seq, float4 r,
                                          QBox *q, bool *bad_rect) {
  const bool live = o < N && qstamp[o] == seq + k + 1;
  const bool ok = isfinite(r.x) && isfinite(r.y) && isfinite(r.z) && isfinite(r.w) &&
                  r.x <= r.z && r.y <= r.w;
  *bad_rect = live && !ok;
  if (!(live && ok)) return false;
  const float x0 = ctl->x0, y0 = ctl->y0, sc = ctl->scale;
  q->i0 = cell_of(r.x, x0, sc);
  q->i1 = cell_of(r.z, x0, sc);
  q->j0 = cell_of(r.y, y0, sc);
  q->j1 = cell_of(r.w, y0, sc);
  return true;
}

// Leaves overlapping a query, enumerated by a group of kSplitGroup lanes
// in an order that both split passes reproduce.  The query's cells of the
// start table are taken kSplitGroup at a time (one per lane); in a round,
// first the leaf entries (a leaf is kept at the cell with minimal
// coordinates among the query's cells of that leaf), in cell order, then
// the internal nodes of the round one after the other, each walked by its
// lane.  Queries over more than kTableScanMax cells are walked from the
// root by the group's first lane.  visit(leaf, covering, idx, ri, rc, cnt)
// receives the leaf's index in the query's list, its rank among the
// intersecting (ri) or covering (rc) entries and its object count.
// Inactive leaves are skipped.
constexpr uint32_t kSplitGroup = 16;
constexpr uint32_t kSplitBatch = 2;  // rounds of table cells whose loads go out together

struct LeafCounts {
  uint32_t n, ni, nc;
};

template <typename Visit>
__device__ __forceinline__ LeafCounts group_leaves(const Tree &tr, uint32_t *stack, const QBox q,
                                                   const uint32_t *leaf_beg, uint32_t covering,
                                                   uint32_t lane, uint64_t gm, Visit &visit) {
  const uint32_t gl = lane & (kSplitGroup - 1u);
  const uint32_t T = tr.tlev, sh = (uint32_t)kFine - T;
  const uint32_t ti0 = q.i0 >> sh, ti1 = q.i1 >> sh, tj0 = q.j0 >> sh, tj1 = q.j1 >> sh;
  const uint32_t w = ti1 - ti0 + 1, ncell = w * (tj1 - tj0 + 1);
  const bool from_root = ncell > kTableScanMax;
  const uint32_t rounds = from_root ? 1u : (ncell + kSplitGroup - 1u) / kSplitGroup;
  uint32_t nl = 0, ni = 0, nc = 0;  // the same on every lane of the group
  // kSplitBatch rounds at a time: their table entries are loaded together,
  // then the object ranges of the leaves they keep, then the rounds run in
  // order
  for (uint32_t rd0 = 0; rd0 < rounds; rd0 += kSplitBatch) {
    uint32_t ent[kSplitBatch], lb[kSplitBatch], le[kSplitBatch];
    bool cell[kSplitBatch], kept[kSplitBatch];
#pragma unroll
    for (uint32_t j = 0; j < kSplitBatch; ++j) {
      const uint32_t c = (rd0 + j) * kSplitGroup + gl;
      cell[j] = !from_root && rd0 + j < rounds && c < ncell;
      ent[j] = cell[j] ? tr.table[morton2(ti0 + c % w, tj0 + c / w)] : 0u;
    }
#pragma unroll
    for (uint32_t j = 0; j < kSplitBatch; ++j) {
      kept[j] = false;
      lb[j] = le[j] = 0u;
      if (cell[j] && (ent[j] & kLeafBit)) {
        // a leaf is kept at the query's cell with minimal coordinates in it
        const uint32_t c = (rd0 + j) * kSplitGroup + gl;
        const uint32_t ci = ti0 + c % w, cj = tj0 + c / w;
        const uint32_t l = ((ent[j] >> kLeafIdxBits) & 15u) + 1u, m = T - l;
        const uint32_t li0 = (ci >> m) << m, lj0 = (cj >> m) << m;
        kept[j] = ci == (ti0 > li0 ? ti0 : li0) && cj == (tj0 > lj0 ? tj0 : lj0);
        if (kept[j]) {
          const uint32_t leaf = ent[j] & kLeafIdxMask;
          lb[j] = leaf_beg[leaf];
          le[j] = leaf_beg[leaf + 1];
        }
      }
    }
    for (uint32_t j = 0; j < kSplitBatch && rd0 + j < rounds; ++j) {
      const uint32_t c = (rd0 + j) * kSplitGroup + gl;
      bool a = false, b = false, cv = false;
      uint32_t leaf = 0, node = 0, ci = 0, cj = 0, depth = T;
      if (from_root) {
        b = gl == 0;
        depth = 0;
      } else if (cell[j]) {
        ci = ti0 + c % w;
        cj = tj0 + c / w;
        if (!(ent[j] & kLeafBit)) {
          b = true;
          node = ent[j];
        } else if (kept[j]) {
          const uint32_t l = ((ent[j] >> kLeafIdxBits) & 15u) + 1u, m = T - l;
          const uint32_t li0 = (ci >> m) << m, lj0 = (cj >> m) << m;
          leaf = ent[j] & kLeafIdxMask;
          a = le[j] != lb[j];
          const uint32_t ilo = li0 << sh, jlo = lj0 << sh, span = (1u << (kFine - l)) - 1u;
          cv = a && covering &&
               (q.i0 < ilo && ilo + span < q.i1 && q.j0 < jlo && jlo + span < q.j1);
        }
      }
      const uint64_t ma = ballot(a) & gm, mc = ballot(cv) & gm, mi = ma & ~mc;
      if (a) visit(leaf, cv, nl + mbcnt(ma), ni + mbcnt(mi), nc + mbcnt(mc), le[j] - lb[j]);
      nl += (uint32_t)__popcll(ma);
      ni += (uint32_t)__popcll(mi);
      nc += (uint32_t)__popcll(mc);
      uint64_t mb = ballot(b) & gm;
      while (mb) {
        const uint32_t bl = (uint32_t)__ffsll((unsigned long long)mb) - 1u;
        mb &= mb - 1u;
        uint32_t dl = 0, di = 0, dc = 0;
        if (lane == bl) {
          auto v = [&](uint32_t lf, bool cov0) {
            const uint32_t cnt = leaf_beg[lf + 1] - leaf_beg[lf];
            if (cnt == 0u) return;
            const bool cc = cov0 && covering;
            visit(lf, cc, nl + dl, ni + di, nc + dc, cnt);
            ++dl;
            if (cc)
              ++dc;
            else
              ++di;
          };
          walk_from(tr.nodes, stack, node, depth, ci, cj, q, v);
        }
        nl += (uint32_t)__shfl((int)dl, (int)bl);
        ni += (uint32_t)__shfl((int)di, (int)bl);
        nc += (uint32_t)__shfl((int)dc, (int)bl);
      }
    }
  }
  return LeafCounts{nl, ni, nc};
}

// Leaves of a uniform grid overlapping a query: the cells of the query's
// column and row range in row order, kSplitGroup at a time (one per lane),
// visited like group_leaves' (index in the query's list, rank among the
// intersecting or covering ones).  A cell strictly inside the range on
// both axes is covering.  Cells without objects are skipped.
template <typename Visit>
__device__ __forceinline__ LeafCounts grid_leaves(uint32_t s, const QBox q,
                                                  const uint32_t *leaf_beg, uint32_t covering,
                                                  uint32_t lane, uint64_t gm, Visit &visit) {
  const uint32_t gl = lane & (kSplitGroup - 1u);
  const uint32_t i0 = ug_col(q.i0, s), i1 = ug_col(q.i1, s);
  const uint32_t j0 = ug_col(q.j0, s), j1 = ug_col(q.j1, s);
  const uint32_t w = i1 - i0 + 1u;
  const uint64_t ncell = (uint64_t)w * (j1 - j0 + 1u);
  uint32_t nl = 0, ni = 0, nc = 0;  // the same on every lane of the group
  for (uint64_t c0 = 0; c0 < ncell; c0 += kSplitGroup) {
    const uint64_t c = c0 + gl;
    bool a = false, cv = false;
    uint32_t leaf = 0, cnt = 0;
    if (c < ncell) {
      const uint32_t ci = i0 + (uint32_t)(c % w), cj = j0 + (uint32_t)(c / w);
      leaf = morton2(ci, cj);
      cnt = leaf_beg[leaf + 1] - leaf_beg[leaf];
      a = cnt != 0u;
      cv = a && covering && i0 < ci && ci < i1 && j0 < cj && cj < j1;
    }
    const uint64_t ma = ballot(a) & gm, mc = ballot(cv) & gm, mi = ma & ~mc;
    if (a) visit(leaf, cv, nl + mbcnt(ma), ni + mbcnt(mi), nc + mbcnt(mc), cnt);
    nl += (uint32_t)__popcll(ma);
    ni += (uint32_t)__popcll(mi);
    nc += (uint32_t)__popcll(mc);
  }
  return LeafCounts{nl, ni, nc};
}

// Processing order of a large query batch: by the Morton code of the
// level-8 cell of the query's lower corner (a 16-bit key, two radix
// passes), so that the queries a wave splits together overlap nearby
// leaves and their subquery records land close together in the leaves'
// groups.  Which group splits which query does not change what is
// written, so the results do not depend on the order.
constexpr uint32_t kQueryOrderMin = 1u << 20;

__global__ void __launch_bounds__(kBlock) k_qorder_keys(Ctl *ctl, const TickIn *tin, uint32_t nq,
                                                        uint32_t *qkey, uint32_t *qord) {
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl->n_qord = nq;
  const float *__restrict__ xa = tin->xa, *__restrict__ ya = tin->ya;
  const float x0 = ctl->x0, y0 = ctl->y0, sc = ctl->scale;
  for (uint32_t k = blockIdx.x * kBlock + threadIdx.x; k < nq; k += gridDim.x * kBlock) {
    qkey[k] = morton2(cell_of(xa[k], x0, sc) >> 8, cell_of(ya[k], y0, sc) >> 8);
    qord[k] = k;
  }
}

// Count pass, one query per group of kSplitGroup lanes: the numbers of
// intersecting and covering subqueries per query, and the pairs the
// covering leaves give (per-block partials added into red's 1,024 slots,
// cleared before the pass); the first `slots` entries of a query's list
// (leaf, covering flag) are kept for the write pass.  Per-query arrays are
// indexed by the processing position g (qpos[k] = g), so the scans hand out
// slots in processing order: the subqueries of a spatially ordered batch's
// neighbouring queries get neighbouring slots.  The rectangle of the g-th query in processing order is stored at
// qrect[g], so that the subqueries of one leaf (queries that lie close
// together, processed close together in a spatially ordered batch) read
// nearby rectangles in the join.
__global__ void __launch_bounds__(kBlock) k_q_count(
    Ctl *ctl, const TickIn *tin, uint32_t nq, uint32_t N, const uint64_t *qstamp, Tree tr,
    const uint32_t *leaf_beg, float4 *qrect, uint32_t *q_ni, uint32_t *q_nc, uint32_t *qlist,
    uint32_t slots, uint32_t covering, const uint32_t *qord, uint32_t *qpos, uint64_t *red) {
  __shared__ uint32_t stack[kFine * kBlock];
  __shared__ uint64_t lds[kWavesPerBlock];
  uint64_t covp = 0;
  const uint32_t *__restrict__ qid = tin->qid;
  const float *__restrict__ xa = tin->xa, *__restrict__ ya = tin->ya, *__restrict__ xb = tin->xb,
                            *__restrict__ yb = tin->yb;
  const uint64_t seq = ctl->qry_seq;
  const bool tree_ok = !(ctl->err & kErrOvfTree);
  const uint32_t ug = ctl->ug_split;
  tr.tlev = ctl->tlev;
  const uint32_t lane = lane_id(), gl = lane & (kSplitGroup - 1u);
  const uint64_t gm = ((1ull << kSplitGroup) - 1ull) << (lane - gl);
  const uint32_t ngroups = gridDim.x * (kBlock / kSplitGroup);
  for (uint32_t g = (blockIdx.x * kBlock + threadIdx.x) / kSplitGroup; g < nq; g += ngroups) {
    const uint32_t k = qord ? qord[g] : g;
    bool bad_rect = false;
    uint32_t ni = 0, nc = 0;
    const float4 r = make_float4(xa[k], ya[k], xb[k], yb[k]);
    QBox q;
    if (query_box(ctl, k, qid[k], N, qstamp, seq, r, &q, &bad_rect) && tree_ok) {
      uint32_t *lst = qlist + (uint64_t)g * slots;
      auto visit = [&](uint32_t leaf, bool c, uint32_t i, uint32_t, uint32_t, uint32_t cnt) {
        if (i < slots) lst[i] = leaf | (c ? kLeafBit : 0u);
        if (c) covp += cnt;
      };
      const LeafCounts n =
          ug ? grid_leaves(ug, q, leaf_beg, covering, lane, gm, visit)
             : group_leaves(tr, stack + threadIdx.x, q, leaf_beg, covering, lane, gm, visit);
      ni = n.ni;
      nc = n.nc;
    }
    if (gl == 0) {
      qrect[g] = r;
      q_ni[g] = ni;
      q_nc[g] = nc;
      qpos[k] = g;
    }
    flag_error(ctl, kErrQueryRect, bad_rect);
  }
  covp = wave_sum(covp);
  if (lane_id() == 0) lds[threadIdx.x / kWave] = covp;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
    for (int w = 0; w < kWavesPerBlock; ++w) t += lds[w];
    if (t) atomicAdd((unsigned long long *)&red[kRedCovPairs * kChunkBlocks +
                                                (blockIdx.x & (kChunkBlocks - 1))],
                     (unsigned long long)t);
  }
}

// Top of the split scans: totals, capacity checks.
__global__ void __launch_bounds__(kChunkBlocks) k_split_top(Ctl *ctl, ScanJobs jobs,
                                                            uint64_t *part, uint64_t cap_sq,
                                                            uint64_t cap_cov) {
  __shared__ uint64_t lds[kChunkBlocks / kWave + 1];
  // both partials are loaded before the first scan waits on a barrier
  uint64_t v[2], tot[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) v[q] = part[q * kChunkBlocks + threadIdx.x];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    part[q * kChunkBlocks + threadIdx.x] =
        block_excl_scan<uint64_t, kChunkBlocks>(v[q], lds, &tot[q]);
    if (threadIdx.x == 0) job_store(jobs.j[q], job_n(jobs.j[q]), tot[q]);
  }
  if (threadIdx.x != 0) return;
  uint32_t err = 0;
  if (tot[0] > cap_sq) err |= kErrOvfSubq;
  if (tot[1] > cap_cov) err |= kErrOvfCov;
  if (ctl->err & kErrOvfTree) err |= kErrOvfTree;
  ctl->err |= err;
  ctl->n_isect = tot[0];
  ctl->n_cov = tot[1];
  ctl->n_entries = ctl->n_leaves;
  ctl->go_split = err ? 0u : 1u;
  // radix passes that sort the subqueries by leaf: the digits of n_leaves - 1
  const uint32_t nl = ctl->n_leaves;
  const uint32_t bits = nl > 1u ? 32u - (uint32_t)__clz((int)(nl - 1u)) : 0u;
  ctl->sq_skip = bits <= 8u ? 8u : (bits + 7u) / 8u * 8u;
  ctl->n32[0] = err ? 0u : (uint32_t)tot[0];
  ctl->n32[1] = err ? 0u : (uint32_t)tot[1];
}

// Write pass, one query per group, in processing order: every intersecting
// subquery's leaf at its slot (skey[slot]; the sort by leaf carries the
// slot itself as the value, made by its first pass; sg[slot] = g, the
// index of its query's rectangle), covering leaves per query.  A query
// whose list fit reads it back, kSplitGroup entries at a time; a longer
// one enumerates its leaves again in the same order.  A stable sort by leaf then groups the subqueries
// (k_sq_final), in slot order inside a leaf, so the grouping and the
// results' layout are the same on every run.
__global__ void __launch_bounds__(kBlock) k_q_write(
    Ctl *ctl, const TickIn *tin, uint32_t nq, uint32_t N, const uint64_t *qstamp, Tree tr,
    const uint32_t *leaf_beg, const float4 *qrect, const uint32_t *q_ioff, const uint32_t *q_coff,
    const uint32_t *q_ni, const uint32_t *q_nc, const uint32_t *qlist, uint32_t slots,
    uint32_t *skey, uint32_t *sg, uint32_t *cov_leaf, uint32_t covering,
    const uint32_t *qord) {
  __shared__ uint32_t stack[kFine * kBlock];
  if (ctl->go_split) {
    const uint32_t *__restrict__ qid = tin->qid;
    const uint64_t seq = ctl->qry_seq;
    const uint32_t ug = ctl->ug_split;
    tr.tlev = ctl->tlev;
    const uint32_t lane = lane_id(), gl = lane & (kSplitGroup - 1u);
    const uint64_t gm = ((1ull << kSplitGroup) - 1ull) << (lane - gl);
    // one XCD's queries write neighbouring slots (the grid is a multiple of
    // kXcds)
    const Sweep sw = xcd_sweep(nq, kBlock / kSplitGroup, threadIdx.x / kSplitGroup);
    for (uint32_t g = sw.first; g < sw.end; g += sw.stride) {
      const uint32_t n = q_ni[g] + q_nc[g];
      if (n == 0) continue;
      const uint32_t wi = q_ioff[g], wc = q_coff[g];
      auto put = [&](uint32_t leaf, bool c, uint32_t ri, uint32_t rc) {
        if (c) {
          cov_leaf[wc + rc] = leaf;
        } else {
          skey[wi + ri] = leaf;
          sg[wi + ri] = g;
        }
      };
      if (n <= slots) {
        const uint32_t *lst = qlist + (uint64_t)g * slots;
        uint32_t ri = 0, rc = 0;
        for (uint32_t i0 = 0; i0 < n; i0 += kSplitGroup) {
          const uint32_t i = i0 + gl;
          const bool v = i < n;
          const uint32_t e = v ? lst[i] : 0u;
          const bool c = v && (e & kLeafBit), x = v && !(e & kLeafBit);
          const uint64_t mi = ballot(x) & gm, mc = ballot(c) & gm;
          if (v) put(e & ~kLeafBit, c, ri + mbcnt(mi), rc + mbcnt(mc));
          ri += (uint32_t)__popcll(mi);
          rc += (uint32_t)__popcll(mc);
        }
      } else {
        const uint32_t k = qord ? qord[g] : g;
        QBox q;
        bool bad_rect;
        query_box(ctl, k, qid[k], N, qstamp, seq, qrect[g], &q, &bad_rect);
        auto visit = [&](uint32_t leaf, bool c, uint32_t, uint32_t ri, uint32_t rc, uint32_t) {
          put(leaf, c, ri, rc);
        };
        if (ug)
          grid_leaves(ug, q, leaf_beg, covering, lane, gm, visit);
        else
          group_leaves(tr, stack + threadIdx.x, q, leaf_beg, covering, lane, gm, visit);
      }
    }
  }
}

// After the sort by leaf (keys skey, values the slots, both in sorted
// order): position p of the grouped subqueries holds slot s = sval[p];
// sq[p] = the index of its query's rectangle (sg[s]), slot_sq[s] = p (sg
// and slot_sq share memory: a slot is read, then written, by the one
// thread of its position).  The slots of neighbouring positions belong to
// queries near the same leaves, so each XCD (work-groups go to the XCDs in
// turn) takes one contiguous eighth of the positions and sweeps it with
// all its work-groups together: the slots in flight then lie in a narrow
// window that the XCD's L2 holds, and in lines that no other XCD writes.
// Every leaf's first position (leaf_sqoff, empty leaves included) is a
// binary search in the sorted keys, one thread per leaf, so a run of
// empty leaves costs no thread a serial loop.
__global__ void __launch_bounds__(kBlock) k_sq_final(const Ctl *ctl, const uint32_t *skey,
                                                     const uint32_t *sval, uint32_t *sq,
                                                     uint32_t *slot_sq, uint32_t *leaf_sqoff) {
  if (!ctl->go_split) return;
  const uint32_t n = ctl->n32[0], nl = ctl->n_leaves;
  const Sweep sw = xcd_sweep(n, kBlock, threadIdx.x);  // the grid is a multiple of kXcds
  for (uint32_t p = sw.first; p < sw.end; p += sw.stride) {
    const uint32_t s = sval[p];
    const uint32_t g = slot_sq[s];
    slot_sq[s] = p;
    sq[p] = g;
  }
  const uint32_t stride = gridDim.x * kBlock, t0 = blockIdx.x * kBlock + threadIdx.x;
  for (uint32_t t = t0; t <= nl; t += stride) leaf_sqoff[t] = lower_bound_u32(skey, 0u, n, t);
}

// -------------------------------------------------------------- schedule --
// Join tasks: a leaf's intersecting subqueries are joined kTaskSub at a
// time, so a leaf that many queries overlap is spread over several waves.
// Task e < n_leaves is the first chunk of leaf e; the further chunks of
// heavy leaves are appended (vtask: leaf, chunk).  Key of a task: 255 - bit
// length of its weight |subqueries of the chunk| x |objects| (ascending =
// heaviest first; 255: no work), or 0 for every task with work when the
// order is not wanted.  A counting sort over the 256 keys gives the run
// order: the keys are counted per block as they are made, and one kernel
// places the tasks with work (tasks of one key in any order) and writes
// their records.  Which task joins which subquery does not depend on the
// order, so neither do the results.  Also the per-block partials of the
// containment-test count, the largest leaf above l_max and the number of
// leaves with work.
__device__ __forceinline__ uint32_t task_key(uint64_t w) {
  return w == 0 ? 255u : 255u - (uint32_t)(64 - __clzll((long long)w));
}

__global__ void __launch_bounds__(kBlock) k_task_keys(Ctl *ctl, const uint32_t *leaf_beg,
                                                      const uint32_t *leaf_sqoff,
                                                      const uint32_t *llevel, uint32_t l_max,
                                                      uint32_t *tkey, uint2 *vtask,
                                                      uint32_t *xbase, uint32_t tcap,
                                                      uint64_t *red, float *tlog,
                                                      uint32_t *tkhist, uint32_t reorder,
                                                      uint32_t count) {
  __shared__ uint64_t s_tests[kWavesPerBlock];
  __shared__ uint32_t s_max[kWavesPerBlock], s_tasks[kWavesPerBlock];
  __shared__ uint32_t lh[256];  // block-local key counts, added to the totals at the end
  static_assert(kBlock == 256, "one key count per thread");
  lh[threadIdx.x] = 0;
  __syncthreads();
  auto key_of = [&](uint64_t w) { return reorder ? task_key(w) : (w ? 0u : 255u); };
  const uint32_t n = ctl->n_leaves;
  const bool ok = ctl->go_split != 0;
  const bool ug = ctl->ug_split != 0;
  uint64_t tests = 0;
  uint32_t mx = 0, nt = 0;
  bool ovf = false;
  const uint32_t nr = (n + kWave - 1) / kWave * kWave;
  for (uint32_t t = blockIdx.x * kBlock + threadIdx.x; t < nr; t += gridDim.x * kBlock) {
    const bool valid = t < n;
    const uint32_t cnt = valid ? leaf_beg[t + 1] - leaf_beg[t] : 0u;
    const uint32_t nsq = valid && ok ? leaf_sqoff[t + 1] - leaf_sqoff[t] : 0u;
    const uint64_t w = (uint64_t)nsq * cnt;
    const uint32_t more = w != 0 ? (nsq - 1u) / kTaskSub : 0u;  // chunks after the first
    const uint32_t base = wave_append(&ctl->n_entries, more);
    if (!valid) continue;
    tests += w;
    nt += w != 0;
    if (ug || llevel[t] < l_max) mx = cnt > mx ? cnt : mx;
    const uint32_t k0 = key_of((uint64_t)(nsq < kTaskSub ? nsq : kTaskSub) * cnt);
    tkey[t] = k0;
    if (count && k0 < 255u) atomicAdd(&lh[k0], 1u);
    if (more) xbase[t] = base;
    for (uint32_t c = 1; c <= more; ++c) {
      const uint32_t e = base + c - 1u;
      if (e >= tcap) {
        ovf = true;
        break;
      }
      const uint32_t sub = nsq - c * kTaskSub;
      vtask[e - n] = make_uint2(t, c);
      const uint32_t ke = key_of((uint64_t)(sub < kTaskSub ? sub : kTaskSub) * cnt);
      tkey[e] = ke;
      if (count && ke < 255u) atomicAdd(&lh[ke], 1u);
    }
    if (tlog) {
      float *rec = tlog + (uint64_t)t * 8;
      rec[0] = (float)cnt;
      rec[1] = (float)nsq;
      rec[2] = (float)llevel[t];
      rec[3] = rec[4] = rec[5] = rec[6] = rec[7] = 0.0f;
    }
  }
  flag_error(ctl, kErrOvfSubq, ovf);  // unreachable: entries <= leaves + subqueries / kTaskSub
  __syncthreads();
  if (lh[threadIdx.x]) atomicAdd(&tkhist[threadIdx.x], lh[threadIdx.x]);
  tests = wave_sum(tests);
  nt = wave_sum(nt);
  mx = wave_max(mx);
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) {
    s_tests[w] = tests;
    s_max[w] = mx;
    s_tasks[w] = nt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < kWavesPerBlock; ++i) {
      tests += s_tests[i];
      nt += s_tasks[i];
      mx = s_max[i] > mx ? s_max[i] : mx;
    }
    red[kRedTests * kChunkBlocks + blockIdx.x] = tests;
    red[kRedMaxLeaf * kChunkBlocks + blockIdx.x] = mx;
    red[kRedTasks * kChunkBlocks + blockIdx.x] = nt;
  }
}

// ------------------------------------------------------------------ join --
// One wave per task (leaf).  Objects of the leaf are taken 64 at a time, one
// per lane; intersecting subqueries of the leaf 64 at a time, one per lane,
// and broadcast to the wave one after the other.  The ballot of the closed
// containment test is the subquery's 64-bit bitmap word for those objects:
// its popcount is the count (pass 1), and in pass 2 every lane with its bit
// set writes its object id at the subquery's offset plus the number of set
// bits below it (coalesced, no atomics, no bitmap in memory).

// Leaf of join task e and the range [sb, se) of its intersecting subqueries.
__device__ __forceinline__ void task_range(uint32_t e, uint32_t n_leaves, const uint2 *vtask,
                                           const uint32_t *leaf_sqoff, uint32_t *leaf,
                                           uint32_t *sb, uint32_t *se) {
  uint32_t l = e, c = 0;
  if (e >= n_leaves) {
    const uint2 v = vtask[e - n_leaves];
    l = v.x;
    c = v.y;
  }
  const uint32_t b = leaf_sqoff[l] + c * kTaskSub, end = leaf_sqoff[l + 1];
  *leaf = l;
  *sb = b;
  *se = end < b + kTaskSub ? end : b + kTaskSub;
}

// Task records in run order: (first subquery, end, first object, end) and
// the leaf, so that a join wave starts a task with one load.  Every block
// scans the 256 key totals to the start of each key's run; the tasks of a
// block round are counted per key in LDS, and one atomic per key and round
// reserves their places in the key's run.
__global__ void __launch_bounds__(kBlock) k_task_place(Ctl *ctl, const uint32_t *tkey,
                                                       const uint2 *vtask,
                                                       const uint32_t *leaf_sqoff,
                                                       const uint32_t *leaf_beg,
                                                       uint32_t *tkhist, uint4 *trec,
                                                       uint32_t *tleaf) {
  __shared__ uint32_t kbase[256], lcnt[256], lres[256];
  __shared__ uint32_t lds[kWavesPerBlock + 1];
  static_assert(kBlock == 256, "one key per thread");
  if (!ctl->go_split) return;
  const uint32_t nt = ctl->n_entries, nl = ctl->n_leaves, tid = threadIdx.x;
  uint32_t total;
  kbase[tid] = block_excl_scan<uint32_t, kBlock>(tid < 255u ? tkhist[tid] : 0u, lds, &total);
  if (blockIdx.x == 0 && tid == 0) ctl->n_run = total;
  for (uint32_t e0 = blockIdx.x * kBlock; e0 < nt; e0 += gridDim.x * kBlock) {
    lcnt[tid] = 0;
    __syncthreads();
    const uint32_t e = e0 + tid;
    const uint32_t key = e < nt ? tkey[e] : 255u;
    uint32_t r = 0;
    if (key < 255u) r = atomicAdd(&lcnt[key], 1u);
    __syncthreads();
    if (lcnt[tid]) lres[tid] = atomicAdd(&tkhist[256 + tid], lcnt[tid]);
    __syncthreads();
    if (key < 255u) {
      const uint32_t pos = kbase[key] + lres[key] + r;
      uint32_t leaf, sb, se;
      task_range(e, nl, vtask, leaf_sqoff, &leaf, &sb, &se);
      trec[pos] = make_uint4(sb, se, leaf_beg[leaf], leaf_beg[leaf + 1]);
      tleaf[pos] = leaf;
    }
    __syncthreads();
  }
}

// A task (at most kTaskSub = 64 intersecting subqueries of one leaf) is
// joined by one wave.  The subqueries' rectangles (and, in the write pass,
// their first result offsets) are staged in the wave's LDS slice, so each
// lane reads subquery kk's with one broadcast load; the leaf's objects are
// held in registers, 64 x NCH at a time, one per lane and chunk.  A wave
// reads the record of its next task and that task's subquery entries
// while it joins the current one, and issues a task's object loads
// together with the gathers of its rectangles (and offsets), so a task
// waits for one round of loads.  The containment tests of a subquery
// against a chunk are one ballot per rectangle bound: the count pass adds
// their popcount, the write pass compacts the hits with each lane's rank
// among them.
// The containment test on integer keys: the key of a binary32 coordinate
// orders like the value (IEEE comparison, with -0 equal to +0), so
// xa <= x <= xb is the unsigned range check key(x) - key(xa) <= key(xb) -
// key(xa): two compares per subquery and object instead of four, and half
// the lane masks to combine.
__device__ __forceinline__ uint32_t ckey(float v) {
  const uint32_t u = __float_as_uint(v);
  return u == 0x80000000u ? 0x80000000u : ((u & 0x80000000u) ? ~u : (u | 0x80000000u));
}
__device__ __forceinline__ uint2 pos_key(float2 p) { return make_uint2(ckey(p.x), ckey(p.y)); }
// (key(xa), key(xb) - key(xa), key(ya), key(yb) - key(ya)) of a valid
// rectangle (xa <= xb, ya <= yb, finite).
__device__ __forceinline__ uint4 rect_key(float4 r) {
  const uint32_t xa = ckey(r.x), ya = ckey(r.y);
  return make_uint4(xa, ckey(r.z) - xa, ya, ckey(r.w) - ya);
}

constexpr uint32_t kJoinRegChunks = 12;  // object chunks of 64 in registers
static_assert(kTaskSub <= (uint32_t)kWave, "a task's subqueries fit one wave");

// Orders a wave's LDS stores before its later loads of other lanes' slots
// (and the loads before the next stores).
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint32_t chunk_count(uint32_t o0, uint32_t oe) {
  return min(kJoinRegChunks, (oe - o0 + (uint32_t)kWave - 1u) / (uint32_t)kWave);
}

// Calls f with the chunk count n (1..kJoinRegChunks) as a constant, so a
// block's rounds test exactly its chunks.
template <uint32_t N> struct Chunks { static constexpr uint32_t value = N; };
template <typename F>
__device__ __forceinline__ auto by_chunks(uint32_t n, F f) {
  switch (n) {
    case 1: return f(Chunks<1>{});
    case 2: return f(Chunks<2>{});
    case 3: return f(Chunks<3>{});
    case 4: return f(Chunks<4>{});
    case 5: return f(Chunks<5>{});
    case 6: return f(Chunks<6>{});
    case 7: return f(Chunks<7>{});
    case 8: return f(Chunks<8>{});
    case 9: return f(Chunks<9>{});
    case 10: return f(Chunks<10>{});
    case 11: return f(Chunks<11>{});
    default: return f(Chunks<12>{});
  }
}
static_assert(kJoinRegChunks == 12, "by_chunks covers 1..12 chunks");

// Task records are read one task ahead with lane l holding component
// l & 3, so the load stays in flight until the components are read out.
// The loads made ahead are issued on every path, at an in-range index, so
// that the count of loads in flight is fixed and waiting for the oldest
// does not wait for the others.
__device__ __forceinline__ uint32_t rec_load(const uint32_t *trec32, uint32_t t, uint32_t nt,
                                             uint32_t lane) {
  return trec32[(uint64_t)(t < nt ? t : 0u) * 4u + (lane & 3u)];
}
// Past the last task (t >= nt): an empty record.
__device__ __forceinline__ uint4 rec_read(uint32_t v, uint32_t t, uint32_t nt) {
  const uint4 r = make_uint4((uint32_t)__builtin_amdgcn_readlane((int)v, 0),
                             (uint32_t)__builtin_amdgcn_readlane((int)v, 1),
                             (uint32_t)__builtin_amdgcn_readlane((int)v, 2),
                             (uint32_t)__builtin_amdgcn_readlane((int)v, 3));
  return t < nt ? r : make_uint4(0u, 0u, 0u, 0u);
}
// Lane l's subquery entry of a task (l < its count): the index of its
// query's rectangle.
__device__ __forceinline__ uint32_t sq_entry(const uint32_t *__restrict__ sq, const uint4 rec,
                                             uint32_t lane) {
  return sq[rec.x < rec.y ? min(rec.x + lane, rec.y - 1u) : 0u];
}

// Chunk c of a block at o0 with exactly NCH chunks: lane l holds object
// o0 + 64 c + l when it is below oe (mask h[c]); the other lanes hold a copy
// of the last object, which the mask excludes.  Every chunk but the last
// is full, so its mask is a constant the tests fold away.
template <uint32_t NCH>
__device__ __forceinline__ void load_chunks(const float2 *__restrict__ sxy, uint32_t o0,
                                            uint32_t oe, uint32_t lane, uint2 *p, uint64_t *h) {
#pragma unroll
  for (uint32_t c = 0; c < NCH; ++c) {
    const uint32_t i = o0 + c * (uint32_t)kWave + lane;
    h[c] = c + 1u < NCH ? ~0ull : ballot(i < oe);
    p[c] = pos_key(sxy[c + 1u < NCH ? i : min(i, oe - 1u)]);
  }
}

template <uint32_t NCH>
__device__ __forceinline__ void load_ids(const uint32_t *__restrict__ sid, uint32_t o0,
                                         uint32_t oe, uint32_t lane, uint32_t *id) {
#pragma unroll
  for (uint32_t c = 0; c < NCH; ++c) {
    const uint32_t i = o0 + c * (uint32_t)kWave + lane;
    id[c] = sid[c + 1u < NCH ? i : min(i, oe - 1u)];
  }
}

// Lanes whose object lies in the closed rectangle r: one ballot per bound,
// so the four comparisons stay lane masks.
__device__ __forceinline__ uint64_t hits(const uint4 r, const uint2 p, uint64_t h) {
  return ballot(p.x - r.x <= r.y) & ballot(p.y - r.z <= r.w) & h;
}

// Hits of subqueries 0..nk-1 against NCH chunks; lane kk returns subquery
// kk's.
template <uint32_t NCH>
__device__ __forceinline__ uint32_t count_rounds(const uint4 *wrect, uint32_t nk,
                                                 const uint2 *p, const uint64_t *h,
                                                 uint32_t lane) {
  uint32_t blk = 0;
  for (uint32_t kk = 0; kk < nk; ++kk) {
    const uint4 r = wrect[kk];
    uint32_t tot = 0;
#pragma unroll
    for (uint32_t c = 0; c < NCH; ++c) tot += (uint32_t)__popcll(hits(r, p[c], h[c]));
    blk = lane == kk ? tot : blk;
  }
  return blk;
}

// First block of a task: its object loads go out with the gathers of the
// subquery rectangles (lane kk < nk: subquery kk's, returned in *r).
template <uint32_t NCH>
__device__ __forceinline__ uint32_t count_first(uint4 *wrect, uint32_t nk,
                                                const float2 *__restrict__ sxy, uint32_t ob,
                                                uint32_t oe, const float4 *__restrict__ qrect,
                                                uint32_t e, uint32_t lane, float4 *r) {
  uint2 p[NCH];
  uint64_t h[NCH];
  load_chunks<NCH>(sxy, ob, oe, lane, p, h);
  if (lane < nk) {
    *r = qrect[e];
    wrect[lane] = rect_key(*r);
  }
  wave_lds_fence();
  return count_rounds<NCH>(wrect, nk, p, h, lane);
}

// A leaf of at most 32 objects: both half-waves hold its objects (lane l
// and l + 32 the same one), and a round tests two subqueries, kk on the
// low half and kk + 1 on the high half.
constexpr uint64_t kLowHalf = 0xffffffffull;

__device__ __forceinline__ uint32_t count_half(uint4 *wrect, uint32_t nk,
                                               const float2 *__restrict__ sxy, uint32_t ob,
                                               uint32_t oe, const float4 *__restrict__ qrect,
                                               uint32_t e, uint32_t lane, float4 *r) {
  const uint32_t half = lane >> 5, i = ob + (lane & 31u);
  const uint64_t h = ballot(i < oe);
  const uint2 p = pos_key(sxy[min(i, oe - 1u)]);
  if (lane < nk) {
    *r = qrect[e];
    wrect[lane] = rect_key(*r);
  }
  wave_lds_fence();
  uint32_t blk = 0;
  for (uint32_t kk = 0; kk < nk; kk += 2) {
    const uint4 rk = wrect[min(kk + half, nk - 1u)];
    uint64_t m = hits(rk, p, h);
    if (kk + 1u >= nk) m &= kLowHalf;  // no second subquery
    const uint32_t lo = (uint32_t)__popcll(m & kLowHalf), hi = (uint32_t)__popcll(m >> 32);
    blk = lane == kk ? lo : (lane == kk + 1u ? hi : blk);
  }
  return blk;
}

// A further block of a long leaf.
template <uint32_t NCH>
__device__ __forceinline__ uint32_t count_block(const uint4 *wrect, uint32_t nk,
                                                const float2 *__restrict__ sxy, uint32_t o0,
                                                uint32_t oe, uint32_t lane) {
  uint2 p[NCH];
  uint64_t h[NCH];
  load_chunks<NCH>(sxy, o0, oe, lane, p, h);
  return count_rounds<NCH>(wrect, nk, p, h, lane);
}

// Eight waves per SIMD (at most 64 registers) hide more of the gathers'
// latency; this kernel fits without spilling registers to memory.
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8)))
k_join_count(const Ctl *ctl, const uint4 *trec, const uint32_t *tleaf, const uint32_t *leaf_sqoff,
             const uint32_t *__restrict__ sq, const float4 *__restrict__ qrect,
             const float2 *__restrict__ sxy, uint32_t *sq_cnt, float *tlog, const uint32_t *lstart,
             const uint32_t *llevel, uint64_t *cu_tests) {
  __shared__ uint4 lrect[kBlock];
  if (!ctl->go_split) return;
  const uint32_t nt = ctl->n_run;
  const uint32_t lane = lane_id();
  const uint32_t nwaves = gridDim.x * kWavesPerBlock;
  const uint32_t w0 =
      __builtin_amdgcn_readfirstlane(blockIdx.x * kWavesPerBlock + threadIdx.x / kWave);
  if (w0 >= nt) return;
  uint4 *wrect = lrect + (threadIdx.x & ~(uint32_t)(kWave - 1));
  const uint32_t *trec32 = (const uint32_t *)trec;
  uint4 rec = rec_read(rec_load(trec32, w0, nt, lane), w0, nt);
  uint4 rn = rec_read(rec_load(trec32, w0 + nwaves, nt, lane), w0 + nwaves, nt);
  uint32_t ea = sq_entry(sq, rec, lane), eb;
  // one step per task: the next task's entries and the record after it are
  // loaded first; the record is read out after this task's own loads have
  // been waited for, so no wait is spent on it.  The entry registers
  // alternate roles, so none is copied (a copy would wait for its load).
  auto step = [&](uint32_t t, const uint32_t e, uint32_t &enx) {
    enx = sq_entry(sq, rn, lane);
    const uint32_t recv = rec_load(trec32, t + 2u * nwaves, nt, lane);
    const uint32_t sb = rec.x, se = rec.y, ob = rec.z, oe = rec.w;
    rec = rn;
    if (sb >= se) {
      rn = rec_read(recv, t + 2u * nwaves, nt);
      return;
    }
    const uint32_t leaf = tlog ? tleaf[t] : 0u;
    const uint64_t clk0 = tlog ? __builtin_amdgcn_s_memrealtime() : 0;
    const uint32_t nk = se - sb;  // at most kTaskSub
    if (cu_tests && lane == 0)
      atomicAdd((unsigned long long *)&cu_tests[cu_slot()], (unsigned long long)nk * (oe - ob));
    float4 r = make_float4(0.f, 0.f, 0.f, 0.f);
    uint32_t cnt = 0;
    wave_lds_fence();
    if (ob < oe) {
      if (oe - ob <= 32u)
        cnt = count_half(wrect, nk, sxy, ob, oe, qrect, e, lane, &r);
      else
        cnt = by_chunks(chunk_count(ob, oe), [&](auto N) {
          return count_first<decltype(N)::value>(wrect, nk, sxy, ob, oe, qrect, e, lane, &r);
        });
      for (uint32_t o0 = ob + (uint32_t)kWave * kJoinRegChunks; o0 < oe;
           o0 += (uint32_t)kWave * kJoinRegChunks)
        cnt += by_chunks(chunk_count(o0, oe), [&](auto N) {
          return count_block<decltype(N)::value>(wrect, nk, sxy, o0, oe, lane);
        });
    } else if (tlog && lane < nk) {
      r = qrect[e];
    }
    rn = rec_read(recv, t + 2u * nwaves, nt);
    if (lane < nk) sq_cnt[sb + lane] = cnt;
    if (tlog) {  // a leaf's record sums its tasks: mean overlap, clock ticks
      const float ovl = wave_sum(lane < nk ? overlap_frac(ctl, lstart, llevel, leaf, r) : 0.0f);
      const uint64_t clk1 = __builtin_amdgcn_s_memrealtime();
      if (lane == 0) {
        const float nsq = (float)(leaf_sqoff[leaf + 1] - leaf_sqoff[leaf]);
        atomicAdd(&tlog[(uint64_t)leaf * 8 + 3], ovl / nsq);
        atomicAdd(&tlog[(uint64_t)leaf * 8 + 4], (float)(clk1 - clk0));
      }
    }
  };
  for (uint32_t t = w0; t < nt; t += 2u * nwaves) {
    step(t, ea, eb);
    if (t + nwaves >= nt) break;
    step(t + nwaves, eb, ea);
  }
}

// Top of the result-offset scan: total result ids, reductions of the
// tick's partials, result capacity check, and the automatic rebuild
// decision for the next tick.
// sqb: the results were appended by the baseline filter, whose global
// counter holds their total (no scan).
__global__ void __launch_bounds__(kChunkBlocks) k_join_top(Ctl *ctl, ScanJobs jobs, uint64_t *part,
                                                           const uint64_t *red, uint64_t cap_res,
                                                           uint32_t policy, uint32_t period,
                                                           uint32_t sqb) {
  __shared__ uint64_t lds[kChunkBlocks / kWave + 1];
  __shared__ uint32_t ldm[kChunkBlocks / kWave + 1];
  const bool ok = ctl->go_split != 0;
  const int t = threadIdx.x;
  // every partial is loaded before the first scan waits on a barrier
  const uint64_t p_res = ok && !sqb ? part[t] : 0u;
  const uint64_t p_covp = red[kRedCovPairs * kChunkBlocks + t];
  const uint64_t p_tests = red[kRedTests * kChunkBlocks + t];
  const uint64_t p_tasks = red[kRedTasks * kChunkBlocks + t];
  const uint32_t p_mx = (uint32_t)red[kRedMaxLeaf * kChunkBlocks + t];
  uint64_t total = 0;
  if (ok && !sqb) {
    part[t] = block_excl_scan<uint64_t, kChunkBlocks>(p_res, lds, &total);
    if (t == 0) job_store(jobs.j[0], job_n(jobs.j[0]), total);
  }
  if (sqb) total = ctl->n_res;
  uint64_t covp, tests, tasks;
  block_excl_scan<uint64_t, kChunkBlocks>(p_covp, lds, &covp);
  block_excl_scan<uint64_t, kChunkBlocks>(p_tests, lds, &tests);
  block_excl_scan<uint64_t, kChunkBlocks>(p_tasks, lds, &tasks);
  const uint32_t mx = block_minmax_1024<true>(p_mx, ldm);
  if (t != 0) return;
  ctl->max_leaf = mx;
  ctl->tests = tests;
  ctl->n_tasks = (uint32_t)tasks;
  if (ok) {
    ctl->n_res = total;
    ctl->cov_pairs = covp;
    if (total > cap_res || (sqb && (ctl->err & kErrOvfRes))) {
      ctl->err |= kErrOvfRes;
      ctl->go_join = 0;
    } else {
      ctl->go_join = 1;
    }
  }
  if (ctl->err & kErrOvfTree) ctl->built = 0;
  const bool leaf_big = mx > 2u * ctl->th_cur;
  const bool moved_out = (uint64_t)ctl->n_outside * 100u > ctl->n_present;
  const bool periodic = ctl->since_build + 1u >= period;
  ctl->want_rebuild = policy == 0u && (leaf_big || moved_out || periodic || !ctl->built);
}

// Subqueries 0..nk-1 against NCH chunks: each hit goes to its subquery's
// next free result slot (woff, advanced in LDS when more objects follow).
template <uint32_t NCH>
__device__ __forceinline__ void write_rounds(const uint4 *wrect, uint64_t *woff, uint32_t nk,
                                             const uint2 *p, const uint64_t *h,
                                             const uint32_t *id, uint32_t *__restrict__ res_ids,
                                             bool more) {
  for (uint32_t kk = 0; kk < nk; ++kk) {
    const uint4 r = wrect[kk];
    uint64_t base = woff[kk];
#pragma unroll
    for (uint32_t c = 0; c < NCH; ++c) {
      const uint64_t m = hits(r, p[c], h[c]);
      if (__builtin_amdgcn_inverse_ballot_w64(m)) res_ids[base + mbcnt(m)] = id[c];
      base += (uint64_t)__popcll(m);
    }
    if (more) woff[kk] = base;  // every lane stores the same value
  }
}

// First block of a task: object loads and the gathers of the subqueries'
// rectangles and result offsets go out together.
template <uint32_t NCH>
__device__ __forceinline__ void write_first(uint4 *wrect, uint64_t *woff, uint32_t nk,
                                            const float2 *__restrict__ sxy,
                                            const uint32_t *__restrict__ sid, uint32_t ob,
                                            uint32_t oe, const float4 *__restrict__ qrect,
                                            const uint64_t *__restrict__ res_off, uint32_t e,
                                            uint32_t sb, uint32_t lane,
                                            uint32_t *__restrict__ res_ids, bool more) {
  uint2 p[NCH];
  uint64_t h[NCH];
  uint32_t id[NCH];
  load_chunks<NCH>(sxy, ob, oe, lane, p, h);
  load_ids<NCH>(sid, ob, oe, lane, id);
  if (lane < nk) {
    const float4 r = qrect[e];
    woff[lane] = res_off[sb + lane];
    wrect[lane] = rect_key(r);
  }
  wave_lds_fence();
  write_rounds<NCH>(wrect, woff, nk, p, h, id, res_ids, more);
}

// Decoding side of count_half: a round writes the hits of subquery kk
// (low half) and kk + 1 (high half), each lane ranked within its half.
__device__ __forceinline__ void write_half(uint4 *wrect, uint64_t *woff, uint32_t nk,
                                           const float2 *__restrict__ sxy,
                                           const uint32_t *__restrict__ sid, uint32_t ob,
                                           uint32_t oe, const float4 *__restrict__ qrect,
                                           const uint64_t *__restrict__ res_off, uint32_t e,
                                           uint32_t sb, uint32_t lane,
                                           uint32_t *__restrict__ res_ids) {
  const uint32_t half = lane >> 5, i = min(ob + (lane & 31u), oe - 1u);
  const uint64_t h = ballot(ob + (lane & 31u) < oe);
  const uint2 p = pos_key(sxy[i]);
  const uint32_t id = sid[i];
  if (lane < nk) {
    const float4 r = qrect[e];
    woff[lane] = res_off[sb + lane];
    wrect[lane] = rect_key(r);
  }
  wave_lds_fence();
  const uint64_t mine = half ? ~kLowHalf : kLowHalf;
  for (uint32_t kk = 0; kk < nk; kk += 2) {
    const uint32_t k = min(kk + half, nk - 1u);
    const uint4 rk = wrect[k];
    const uint64_t base = woff[k];
    uint64_t m = hits(rk, p, h);
    if (kk + 1u >= nk) m &= kLowHalf;
    if (__builtin_amdgcn_inverse_ballot_w64(m)) res_ids[base + mbcnt(m & mine)] = id;
  }
}

template <uint32_t NCH>
__device__ __forceinline__ void write_block(const uint4 *wrect, uint64_t *woff, uint32_t nk,
                                            const float2 *__restrict__ sxy,
                                            const uint32_t *__restrict__ sid, uint32_t o0,
                                            uint32_t oe, uint32_t lane,
                                            uint32_t *__restrict__ res_ids, bool more) {
  uint2 p[NCH];
  uint64_t h[NCH];
  uint32_t id[NCH];
  load_chunks<NCH>(sxy, o0, oe, lane, p, h);
  load_ids<NCH>(sid, o0, oe, lane, id);
  write_rounds<NCH>(wrect, woff, nk, p, h, id, res_ids, more);
}

// Tasks of one object block (at most kJoinRegChunks x 64 objects) produce
// their ids in address order: the runs of a task's subqueries are adjacent,
// and each subquery's hits come chunk by chunk.  Such a task stages its ids
// in the wave's LDS slice and stores them 64 at a time, full and
// consecutive, instead of one partial store per subquery and chunk.
constexpr uint32_t kStage = 1024;  // staged ids per wave

// Stores the staged ids [0, fill) at res_ids[gbase ..): every full 64 (all:
// every one), the rest moved to the front of the slice.
__device__ __forceinline__ void stage_flush(uint32_t *stage, uint32_t &fill, uint64_t &gbase,
                                            uint32_t *__restrict__ res_ids, uint32_t lane,
                                            bool all) {
  wave_lds_fence();
  const uint32_t nfull = fill & ~((uint32_t)kWave - 1u);
  for (uint32_t j = 0; j < nfull; j += (uint32_t)kWave) res_ids[gbase + j + lane] = stage[j + lane];
  const uint32_t rem = fill - nfull;
  if (all) {
    if (lane < rem) res_ids[gbase + nfull + lane] = stage[nfull + lane];
    gbase += fill;
    fill = 0;
    return;
  }
  const uint32_t v = lane < rem ? stage[nfull + lane] : 0u;
  wave_lds_fence();  // every read above is done before the slice is overwritten
  if (lane < rem) stage[lane] = v;
  gbase += nfull;
  fill = rem;
}

template <uint32_t NCH>
__device__ __forceinline__ void stage_rounds(const uint4 *wrect, uint32_t nk, const uint2 *p,
                                             const uint64_t *h, const uint32_t *id,
                                             uint32_t *stage, uint32_t &fill, uint64_t &gbase,
                                             uint32_t *__restrict__ res_ids, uint32_t lane) {
  for (uint32_t kk = 0; kk < nk; ++kk) {
    if (fill > kStage - (uint32_t)kWave * NCH) stage_flush(stage, fill, gbase, res_ids, lane, false);
    const uint4 r = wrect[kk];
#pragma unroll
    for (uint32_t c = 0; c < NCH; ++c) {
      const uint64_t m = hits(r, p[c], h[c]);
      if (__builtin_amdgcn_inverse_ballot_w64(m)) stage[mbcnt(m, fill)] = id[c];
      fill += (uint32_t)__popcll(m);
    }
  }
}

// A one-block task: loads as write_first, ids staged from the task's first
// result offset on.
template <uint32_t NCH>
__device__ __forceinline__ void write_staged(uint4 *wrect, uint32_t nk,
                                             const float2 *__restrict__ sxy,
                                             const uint32_t *__restrict__ sid, uint32_t ob,
                                             uint32_t oe, const float4 *__restrict__ qrect,
                                             const uint64_t *__restrict__ res_off, uint32_t e,
                                             uint32_t sb, uint32_t lane, uint32_t *stage,
                                             uint32_t *__restrict__ res_ids) {
  uint2 p[NCH];
  uint64_t h[NCH];
  uint32_t id[NCH];
  load_chunks<NCH>(sxy, ob, oe, lane, p, h);
  load_ids<NCH>(sid, ob, oe, lane, id);
  uint64_t gbase = res_off[sb];
  if (lane < nk) wrect[lane] = rect_key(qrect[e]);
  wave_lds_fence();
  uint32_t fill = 0;
  stage_rounds<NCH>(wrect, nk, p, h, id, stage, fill, gbase, res_ids, lane);
  stage_flush(stage, fill, gbase, res_ids, lane, true);
}

// write_half with staging: a round stages subquery kk's hits (low half)
// and then kk + 1's (high half).
__device__ __forceinline__ void write_half_staged(uint4 *wrect, uint32_t nk,
                                                  const float2 *__restrict__ sxy,
                                                  const uint32_t *__restrict__ sid, uint32_t ob,
                                                  uint32_t oe, const float4 *__restrict__ qrect,
                                                  const uint64_t *__restrict__ res_off,
                                                  uint32_t e, uint32_t sb, uint32_t lane,
                                                  uint32_t *stage,
                                                  uint32_t *__restrict__ res_ids) {
  const uint32_t half = lane >> 5, i = min(ob + (lane & 31u), oe - 1u);
  const uint64_t h = ballot(ob + (lane & 31u) < oe);
  const uint2 p = pos_key(sxy[i]);
  const uint32_t id = sid[i];
  uint64_t gbase = res_off[sb];
  if (lane < nk) wrect[lane] = rect_key(qrect[e]);
  wave_lds_fence();
  uint32_t fill = 0;
  for (uint32_t kk = 0; kk < nk; kk += 2) {
    if (fill > kStage - (uint32_t)kWave) stage_flush(stage, fill, gbase, res_ids, lane, false);
    const uint4 rk = wrect[min(kk + half, nk - 1u)];
    uint64_t m = hits(rk, p, h);
    if (kk + 1u >= nk) m &= kLowHalf;
    const uint32_t lo = (uint32_t)__popcll(m & kLowHalf);
    if (__builtin_amdgcn_inverse_ballot_w64(m))
      stage[fill + (half ? lo + mbcnt(m & ~kLowHalf) : mbcnt(m & kLowHalf))] = id;
    fill += (uint32_t)__popcll(m);
  }
  stage_flush(stage, fill, gbase, res_ids, lane, true);
}

// The write pass puts the results of the subqueries in subquery order: task
// by task, the runs of a task's subqueries are adjacent, so the pass stores
// its ids as one contiguous stream and reads its offsets in order; a
// query's results are its slots' runs (slot_sq).  Six waves per SIMD (at
// most 80 registers; twelve register chunks need 92 otherwise, five waves):
// the compiler keeps two registers in scratch, and the extra wave per SIMD
// hides more of the stores' latency.
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6)))
k_join_write(Ctl *ctl, const uint4 *trec, const uint32_t *tleaf, const uint32_t *__restrict__ sq,
             const float4 *__restrict__ qrect, const float2 *__restrict__ sxy,
             const uint32_t *__restrict__ sid, const uint64_t *__restrict__ res_off,
             uint32_t *__restrict__ res_ids, uint32_t nq, float *tlog) {
  __shared__ uint4 lrect[kBlock];
  __shared__ uint64_t loff[kBlock];
  __shared__ uint32_t lstage[kWavesPerBlock * kStage];
  const bool go = ctl->go_join != 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->qry_seq += nq;
    ctl->tick += 1;
  }
  if (!go) return;
  const uint32_t nt = ctl->n_run;
  const uint32_t lane = lane_id();
  const uint32_t nwaves = gridDim.x * kWavesPerBlock;
  const uint32_t w0 =
      __builtin_amdgcn_readfirstlane(blockIdx.x * kWavesPerBlock + threadIdx.x / kWave);
  uint4 *wrect = lrect + (threadIdx.x & ~(uint32_t)(kWave - 1));
  uint64_t *woff = loff + (threadIdx.x & ~(uint32_t)(kWave - 1));
  uint32_t *stage = lstage + (threadIdx.x / kWave) * kStage;
  if (w0 >= nt) return;
  const uint32_t *trec32 = (const uint32_t *)trec;
  uint4 rec = rec_read(rec_load(trec32, w0, nt, lane), w0, nt);
  uint4 rn = rec_read(rec_load(trec32, w0 + nwaves, nt, lane), w0 + nwaves, nt);
  uint32_t ea = sq_entry(sq, rec, lane), eb;
  auto step = [&](uint32_t t, const uint32_t e, uint32_t &enx) {
    enx = sq_entry(sq, rn, lane);
    const uint32_t recv = rec_load(trec32, t + 2u * nwaves, nt, lane);
    const uint32_t sb = rec.x, se = rec.y, ob = rec.z, oe = rec.w;
    rec = rn;
    if (sb >= se || ob >= oe) {
      rn = rec_read(recv, t + 2u * nwaves, nt);
      return;
    }
    const uint32_t leaf = tlog ? tleaf[t] : 0u;
    const uint64_t clk0 = tlog ? __builtin_amdgcn_s_memrealtime() : 0;
    const uint32_t nk = se - sb;  // at most kTaskSub
    const uint32_t nch = chunk_count(ob, oe);
    const bool more = ob + (uint32_t)kWave * kJoinRegChunks < oe;
    wave_lds_fence();
    if (oe - ob <= 32u)
      write_half_staged(wrect, nk, sxy, sid, ob, oe, qrect, res_off, e, sb, lane, stage,
                        res_ids);
    else if (!more)
      by_chunks(nch, [&](auto N) {
        write_staged<decltype(N)::value>(wrect, nk, sxy, sid, ob, oe, qrect, res_off, e, sb, lane,
                                         stage, res_ids);
      });
    else
      write_first<kJoinRegChunks>(wrect, woff, nk, sxy, sid, ob, oe, qrect, res_off, e, sb, lane,
                                  res_ids, more);
    rn = rec_read(recv, t + 2u * nwaves, nt);
    for (uint32_t o0 = ob + (uint32_t)kWave * kJoinRegChunks; o0 < oe;
         o0 += (uint32_t)kWave * kJoinRegChunks) {
      const bool more2 = o0 + (uint32_t)kWave * kJoinRegChunks < oe;
      wave_lds_fence();
      by_chunks(chunk_count(o0, oe), [&](auto N) {
        write_block<decltype(N)::value>(wrect, woff, nk, sxy, sid, o0, oe, lane, res_ids, more2);
      });
    }
    if (tlog && lane == 0)
      atomicAdd(&tlog[(uint64_t)leaf * 8 + 5], (float)(__builtin_amdgcn_s_memrealtime() - clk0));
  };
  for (uint32_t t = w0; t < nt; t += 2u * nwaves) {
    step(t, ea, eb);
    if (t + nwaves >= nt) break;
    step(t + nwaves, eb, ea);
  }
}

// --------------------------------------------------------------- results --

// Rebuild by cost, at the end of every tick (rent or buy: keeping the
// quadtree costs the excess of each kept tick over the fastest kept tick
// since the last build; a build costs its tick's excess over that kept
// tick; the next tick builds once the summed excess reaches the cost of a
// build, which spends at most twice the least possible on any sequence of
// growing excesses).  Durations are device time from the index frame's
// decision to this kernel.  Results do not depend on when the quadtree is
// built.
__device__ void rebuild_by_cost(Ctl *ctl) {
  const float d = (float)(__builtin_amdgcn_s_memrealtime() - ctl->t_start);
  if (ctl->rebuild) {
    ctl->d_build = d;
    ctl->d_base = 0.0f;
    ctl->b_cost = -1.0f;
    ctl->excess = 0.0f;
  } else {
    if (ctl->d_base == 0.0f || d < ctl->d_base) ctl->d_base = d;
    if (ctl->b_cost < 0.0f) ctl->b_cost = fmaxf(ctl->d_build - d, 0.0f);
    ctl->excess += d - ctl->d_base;
  }
  ctl->want_rebuild = !ctl->built || (ctl->b_cost >= 0.0f && ctl->excess >= ctl->b_cost);
}

// End of a tick: the control block to the host's pinned mirror (one wave,
// a word per lane), so reading the tick's counters needs no copy command.
__global__ void k_ctl_out(Ctl *ctl, Ctl *host) {
  static_assert(sizeof(Ctl) % 4 == 0, "word copy");
  if (threadIdx.x == 0 && ctl->policy == 3u) rebuild_by_cost(ctl);
  __syncthreads();
  const uint32_t *src = (const uint32_t *)ctl;
  uint32_t *dst = (uint32_t *)host;
  for (uint32_t i = threadIdx.x; i < sizeof(Ctl) / 4; i += blockDim.x) dst[i] = src[i];
}

__global__ void k_counters(const Ctl *ctl, uint64_t *out) {
  const bool ok = ctl->go_join != 0;
  out[0] = ok ? ctl->n_res + ctl->cov_pairs : 0ull;
  out[1] = ok ? ctl->n_res : 0ull;
  out[2] = ok ? ctl->cov_pairs : 0ull;
  out[3] = ctl->n_isect;
  out[4] = ctl->n_cov;
  out[5] = ctl->tests;
  out[6] = ctl->n_tasks;
  out[7] = ctl->err;
}

// ------------------------------------------------------- host launchers --

#define LAUNCH(k, g, b, s, ...) hipLaunchKernelGGL(k, dim3(g), dim3(b), 0, s, __VA_ARGS__)

void launch_ctl_init(Ctl *ctl, uint32_t th, uint32_t ug_split, uint32_t ug_bits, uint32_t policy,
                     hipStream_t s) {
  LAUNCH(k_ctl_init, 1, 1, s, ctl, th, ug_split, ug_bits, policy);
}
void launch_request_build(Ctl *ctl, uint32_t th, hipStream_t s) {
  LAUNCH(k_request_build, 1, 1, s, ctl, th);
}
void launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s) {
  LAUNCH(k_fill_u32, grid_for(n), kBlock, s, p, n, v);
}
void launch_fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s) {
  LAUNCH(k_fill_u64, grid_for(n), kBlock, s, p, n, v);
}

// Writes the selected parts of a (1: updates, 2: queries) into tin.
__global__ void k_tick_in(TickIn a, uint32_t parts, TickIn *tin) {
  if (threadIdx.x != 0) return;
  if (parts & 1u) {
    tin->id = a.id;
    tin->x = a.x;
    tin->y = a.y;
  }
  if (parts & 2u) {
    tin->qid = a.qid;
    tin->xa = a.xa;
    tin->ya = a.ya;
    tin->xb = a.xb;
    tin->yb = a.yb;
  }
}

void launch_tick_in(const Bufs &B, const TickIn &a, uint32_t parts, hipStream_t s) {
  LAUNCH(k_tick_in, 1, kWave, s, a, parts, B.tin);
}

void launch_updates(const Bufs &B, uint32_t m, uint64_t seq_off, hipStream_t s) {
  const unsigned g = grid_for(m);
  LAUNCH(k_upd_stamp, g, kBlock, s, (const TickIn *)B.tin, m, B.N, seq_off, B.ustamp, B.ctl);
  LAUNCH(k_upd_write, g, kBlock, s, (const TickIn *)B.tin, m, B.N, seq_off,
         (const uint64_t *)B.ustamp, (const Ctl *)B.ctl, B.pos);
}


void launch_index(const Bufs &B, uint32_t decision, uint32_t policy, uint64_t upd_total,
                  uint32_t nq, uint32_t key_bits, hipStream_t s) {
  LAUNCH(k_mbr, kChunkBlocks, kBlock, s, (const float2 *)B.pos, B.N,
         (const Ctl *)B.ctl, B.blk, B.red);
  LAUNCH(k_decide, 1, kChunkBlocks, s, B.ctl, B.blk, (const uint64_t *)B.red, B.front[0],
         B.tkhist, decision, policy, upd_total);
  if (decision == 0u && key_bits) {
    // the tree is kept and the host knows the leaf-key width: exactly the
    // passes it needs, starting from the buffer that makes them end in A
    const int passes = (int)((key_bits + 7u) / 8u);
    const bool odd = passes & 1;
    LAUNCH(k_morton, kChunkBlocks, kBlock, s, (const float2 *)B.pos, B.N, tree_of(B), B.ctl,
           (const uint32_t *)B.blk, odd ? B.keyB : B.keyA, odd ? B.valB : B.valA,
           odd ? B.sxy2 : B.sxy, (const TickIn *)B.tin, nq, B.qstamp);
    if (odd)
      radix_sort_pairs(B.keyB, B.valB, B.keyA, B.valA, &B.ctl->n_present, B.N, nullptr, B.hist,
                       B.tot, 0, 8 * passes, s, B.sxy2, B.sxy);
    else
      radix_sort_pairs(B.keyA, B.valA, B.keyB, B.valB, &B.ctl->n_present, B.N, nullptr, B.hist,
                       B.tot, 0, 8 * passes, s, B.sxy, B.sxy2);
    return;
  }
  LAUNCH(k_morton, kChunkBlocks, kBlock, s, (const float2 *)B.pos, B.N, tree_of(B), B.ctl,
         (const uint32_t *)B.blk, B.keyA, B.valA, B.sxy, (const TickIn *)B.tin, nq, B.qstamp);
  radix_sort_pairs(B.keyA, B.valA, B.keyB, B.valB, &B.ctl->n_present, B.N, nullptr, B.hist,
                   B.tot, 0, 32, s, B.sxy, B.sxy2, &B.ctl->sort_skip);
}

void launch_build(const Bufs &B, uint32_t l_max, hipStream_t s) {
  for (uint32_t l = 1; l <= l_max; ++l) {
    // enough waves for a wave per quadrant on the top levels, enough lanes
    // for a lane per quadrant below
    LAUNCH(k_tree_level, grid_for(B.FCAP > kWaveSplitMax * kWave ? B.FCAP : kWaveSplitMax * kWave),
           kBlock, s, B.ctl, l, l_max, (const uint32_t *)B.keyA,
           (const uint4 *)B.front[(l - 1) & 1], B.front[l & 1], B.FCAP, B.lstart, B.llevel,
           B.LCAP);
  }
  LAUNCH(k_tree_done, 1, 1, s, B.ctl, B.LCAP, B.tcap, B.N);
  radix_sort_pairs(B.lstart, B.llevel, B.lstart2, B.llevel2, &B.ctl->n_leaves, B.LCAP,
                   &B.ctl->rebuild, B.hist, B.tot, 0, 32, s);
  LAUNCH(k_nodes_open, grid_for(B.LCAP), kBlock, s, (const Ctl *)B.ctl,
         (const uint32_t *)B.lstart, (const uint32_t *)B.llevel, B.nopen);
  ScanJobs jobs{};
  jobs.j[0] = job_u32(B.nopen, B.node_off, &B.ctl->n_leaves, 0);
  mscan(jobs, 1, B.part, &B.ctl->rebuild, nullptr, s);
  LAUNCH(k_nodes_build, grid_for(B.LCAP), kBlock, s, B.ctl, (const uint32_t *)B.lstart,
         (const uint32_t *)B.llevel, (const uint32_t *)B.node_off, B.nodes, B.NCAP);
  LAUNCH(k_table_build, grid_for(1ull << (2 * B.tcap), 4096), kBlock, s, (const Ctl *)B.ctl,
         (const uint32_t *)B.lstart, (const uint32_t *)B.llevel, (const uint32_t *)B.node_off,
         B.table);
}

void launch_leaves(const Bufs &B, hipStream_t s) {
  // a thread per leaf (binary searches) or per sorted object (one pass)
  LAUNCH(k_leaf_ranges, grid_for(B.LCAP > B.N ? B.LCAP : B.N, 4096), kBlock, s, (const Ctl *)B.ctl,
         (const uint32_t *)B.keyA, (const uint32_t *)B.lstart, B.leaf_beg);
}

const uint32_t *launch_split(const Bufs &B, uint32_t nq, uint32_t covering, hipStream_t s) {
  const TickIn *tin = B.tin;
  const uint32_t *qord = nullptr;
  if (nq >= kQueryOrderMin) {
    LAUNCH(k_qorder_keys, grid_for(nq), kBlock, s, B.ctl, tin, nq, B.qkey, B.qord);
    const bool alt = radix_sort_pairs(B.qkey, B.qord, B.qkey2, B.qord2, &B.ctl->n_qord, nq, nullptr,
                                      B.hist, B.tot, 0, 16, s);
    qord = alt ? B.qord2 : B.qord;
  }
  LAUNCH(k_fill_u64, 4, kBlock, s, B.red + (uint64_t)kRedCovPairs * kChunkBlocks,
         (uint64_t)kChunkBlocks, 0ull);
  LAUNCH(k_q_count, grid_for((uint64_t)nq * kSplitGroup, 8192), kBlock, s, B.ctl, tin, nq, B.N,
         (const uint64_t *)B.qstamp, tree_of(B), (const uint32_t *)B.leaf_beg, B.qrect, B.q_ni,
         B.q_nc, B.qlist, B.slots, covering, qord, B.qpos, B.red);
  ScanJobs jobs{};
  jobs.j[0] = job_u32(B.q_ni, B.q_ioff, nullptr, nq);
  jobs.j[1] = job_u32(B.q_nc, B.q_coff, nullptr, nq);
  mscan_reduce(jobs, 2, B.part, nullptr, s);
  LAUNCH(k_split_top, 1, kChunkBlocks, s, B.ctl, jobs, B.part, B.S, B.C);
  mscan_down(jobs, 2, (const uint64_t *)B.part, nullptr, s);
  // subqueries in slot order: leaf keys in sq_cnt, rectangle indices in
  // slot_sq; the sort by leaf makes the slots as its values, ping-pongs
  // through res_off's memory and ends where it started (values in sq)
  uint32_t *skey = B.sq_cnt, *sval = B.sq, *k1 = (uint32_t *)B.res_off, *v1 = k1 + B.S;
  // 16 queries per block and 4,096 blocks: enough groups in flight to hide
  // a query's three dependent loads (counts, offsets, its list)
  constexpr unsigned kQWriteBlocks = 4096;
  static_assert(kQWriteBlocks % kXcds == 0, "k_q_write sweeps per XCD");
  LAUNCH(k_q_write, kQWriteBlocks, kBlock, s, B.ctl, tin, nq, B.N, (const uint64_t *)B.qstamp,
         tree_of(B), (const uint32_t *)B.leaf_beg, (const float4 *)B.qrect,
         (const uint32_t *)B.q_ioff, (const uint32_t *)B.q_coff, (const uint32_t *)B.q_ni,
         (const uint32_t *)B.q_nc, (const uint32_t *)B.qlist, B.slots, skey, B.slot_sq,
         B.cov_leaf, covering, qord);
  radix_sort_pairs(skey, sval, k1, v1, &B.ctl->n32[0], B.S, &B.ctl->go_split, B.hist, B.tot, 0,
                   32, s, nullptr, nullptr, &B.ctl->sq_skip, true);
  LAUNCH(k_sq_final, (grid_for(B.S, 4096) + kXcds - 1u) / kXcds * kXcds, kBlock, s,
         (const Ctl *)B.ctl, (const uint32_t *)skey,
         (const uint32_t *)sval, B.sq, B.slot_sq, B.leaf_sqoff);
  return qord;
}

void launch_schedule(const Bufs &B, uint32_t reorder, uint32_t l_max, bool learned,
                     hipStream_t s) {
  const bool mlp = reorder && learned;  // the network's keys replace the weight keys
  LAUNCH(k_task_keys, kChunkBlocks, kBlock, s, B.ctl, (const uint32_t *)B.leaf_beg,
         (const uint32_t *)B.leaf_sqoff, (const uint32_t *)B.llevel, l_max, B.tkey, B.vtask,
         B.xbase, B.TCAP, B.red, B.tlog, B.tkhist, reorder, mlp ? 0u : 1u);
  if (mlp) launch_schedule_mlp(B, s);
  LAUNCH(k_task_place, grid_for(B.TCAP, 2048), kBlock, s, B.ctl, (const uint32_t *)B.tkey,
         (const uint2 *)B.vtask, (const uint32_t *)B.leaf_sqoff, (const uint32_t *)B.leaf_beg,
         B.tkhist, B.trec, B.tleaf);
}

void launch_join_count(const Bufs &B, hipStream_t s) {
  LAUNCH(k_join_count, kJoinBlocks, kBlock, s, (const Ctl *)B.ctl, (const uint4 *)B.trec,
         (const uint32_t *)B.tleaf, (const uint32_t *)B.leaf_sqoff, (const uint32_t *)B.sq,
         (const float4 *)B.qrect, (const float2 *)B.sxy, B.sq_cnt,
         B.tlog, (const uint32_t *)B.lstart, (const uint32_t *)B.llevel, B.cu_tests);
}

void launch_join_scan(const Bufs &B, uint64_t cap_res, uint32_t policy, uint32_t period,
                      hipStream_t s) {
  ScanJobs jobs{};
  jobs.j[0] = job_u64(B.sq_cnt, B.res_off, &B.ctl->n32[0], 0);
  mscan_reduce(jobs, 1, B.part, &B.ctl->go_split, s);
  LAUNCH(k_join_top, 1, kChunkBlocks, s, B.ctl, jobs, B.part, (const uint64_t *)B.red, cap_res,
         policy, period, 0u);
  mscan_down(jobs, 1, (const uint64_t *)B.part, &B.ctl->go_split, s);
}

void launch_join_top_sqb(const Bufs &B, uint64_t cap_res, uint32_t policy, uint32_t period,
                         hipStream_t s) {
  ScanJobs jobs{};
  jobs.j[0] = job_u64(B.sq_cnt, B.res_off, &B.ctl->n32[0], 0);
  LAUNCH(k_join_top, 1, kChunkBlocks, s, B.ctl, jobs, B.part, (const uint64_t *)B.red, cap_res,
         policy, period, 1u);
}

void launch_join_write(const Bufs &B, uint32_t nq, hipStream_t s) {
  LAUNCH(k_join_write, kJoinBlocks, kBlock, s, B.ctl, (const uint4 *)B.trec,
         (const uint32_t *)B.tleaf, (const uint32_t *)B.sq, (const float4 *)B.qrect,
         (const float2 *)B.sxy, (const uint32_t *)B.valA, (const uint64_t *)B.res_off, B.res_ids,
         nq, B.tlog);
}

const void *join_write_kernel() { return reinterpret_cast<const void *>(&k_join_write); }

void launch_ctl_out(const Bufs &B, Ctl *host, hipStream_t s) {
  LAUNCH(k_ctl_out, 1, kWave, s, B.ctl, host);
}

void launch_counters(const Bufs &B, uint64_t *out, hipStream_t s) {
  LAUNCH(k_counters, 1, 1, s, (const Ctl *)B.ctl, out);
}

}  // namespace sj
