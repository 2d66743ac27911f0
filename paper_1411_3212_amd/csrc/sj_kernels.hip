// Kernels of the per-tick spatial join (gfx950, wave64).
//
// Pipeline of one tick (paper Section "Query processing pipeline"):
//   updates      last-writer-wins scatter of (id, x, y) into positions by id
//   index        MBR -> frame -> Morton codes -> LDS-staged radix sort ->
//                sorted positions (index creation, Algorithm 1 first steps)
//   build        level-wise PR-quadtree split under the threshold, leaves in
//                Morton order, node table for query traversal (Algorithm 1)
//   leaves       object range of every leaf in the sorted order
//   split        per query: leaves it touches, intersecting / covering;
//                count -> exclusive scan -> write (query indexing)
//   schedule     leaves with intersecting subqueries, heaviest first
//                (task scheduling optimisation)
//   join         per leaf, one wave per 64 objects: ballot of the closed
//                containment test for every intersecting subquery; count
//                pass -> exclusive scan -> write pass of object ids
//                (filtering with bitmaps + decoding, Algorithm 2 and the
//                decoding algorithm)
#include "sj_device.h"
#include "sj_kernels.h"

namespace sj {

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

__global__ void k_ctl_init(Ctl *ctl, uint32_t th) {
  Ctl c;
  uint8_t *b = (uint8_t *)&c;
  for (unsigned i = 0; i < sizeof(Ctl); ++i) b[i] = 0;
  c.th_cur = th;
  c.scale = 65536.0f;
  *ctl = c;
}

__global__ void k_request_build(Ctl *ctl, uint32_t th) {
  ctl->force = 1u;
  if (th) ctl->th_next = th;
}

// --------------------------------------------------------------- updates --
// Tick batching: within a tick the most recent update of an object wins.
// Every update gets a sequence number (monotone over the scene's life);
// an atomic max per object keeps the latest, then only that one is written.

__global__ void __launch_bounds__(kBlock) k_upd_stamp(const uint32_t *id, const float *x,
                                                      const float *y, uint32_t m, uint32_t N,
                                                      uint64_t *stamp, Ctl *ctl) {
  const uint64_t seq = ctl->upd_seq;
  const uint32_t stride = gridDim.x * kBlock;
  const uint32_t mr = (m + kWave - 1) / kWave * kWave;
  for (uint32_t k = blockIdx.x * kBlock + threadIdx.x; k < mr; k += stride) {
    bool bad_id = false, bad_xy = false;
    if (k < m) {
      const uint32_t o = id[k];
      const float xv = x[k], yv = y[k];
      bad_id = o >= N;
      bad_xy = !bad_id && !(isfinite(xv) && isfinite(yv));
      if (!bad_id && !bad_xy) atomicMax((unsigned long long *)&stamp[o], (unsigned long long)(seq + k + 1));
    }
    if (ballot(bad_id | bad_xy)) {
      uint64_t mi = ballot(bad_id), mx = ballot(bad_xy);
      if (lane_id() == 0) atomicOr(&ctl->err_upd, (mi ? kErrUpdId : 0u) | (mx ? kErrUpdCoord : 0u));
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_upd_write(const uint32_t *id, const float *x,
                                                      const float *y, uint32_t m, uint32_t N,
                                                      const uint64_t *stamp, const Ctl *ctl,
                                                      float *px, float *py) {
  const uint64_t seq = ctl->upd_seq;
  for (uint32_t k = blockIdx.x * kBlock + threadIdx.x; k < m; k += gridDim.x * kBlock) {
    const uint32_t o = id[k];
    if (o >= N) continue;
    if (stamp[o] == seq + k + 1) {
      px[o] = x[k];
      py[o] = y[k];
    }
  }
}

__global__ void k_upd_end(Ctl *ctl, uint32_t m) { ctl->upd_seq += m; }

// ----------------------------------------------------------------- index --

__global__ void k_tick_begin(Ctl *ctl) {
  ctl->err = ctl->err_upd;
  ctl->err_upd = 0;
  ctl->mbr[0] = ctl->mbr[1] = 0xffffffffu;
  ctl->mbr[2] = ctl->mbr[3] = 0u;
  ctl->n_present = 0;
  ctl->n_outside = 0;
  ctl->rebuild = 0;
  for (int l = 0; l < kFine + 2; ++l) ctl->fcount[l] = 0;
  ctl->n_tasks = 0;
  ctl->prev_max_leaf = ctl->max_leaf;
  ctl->max_leaf = 0;
  ctl->go_split = 0;
  ctl->go_join = 0;
  ctl->n_isect = ctl->n_cov = ctl->n_res = ctl->cov_pairs = ctl->tests = 0;
}

// MBR of the present objects (position not NaN), present count per block
// of ids (for the order-preserving compaction) and the number of present
// objects outside the current frame.
__global__ void __launch_bounds__(kBlock) k_mbr(const float *px, const float *py, uint32_t N,
                                                Ctl *ctl, uint32_t *blk) {
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
  for (uint64_t i = b0 + threadIdx.x; i < b1; i += kBlock) {
    const float xv = px[i];
    if (xv == xv) {
      const float yv = py[i];
      ++cnt;
      mnx = fminf(mnx, xv);
      mxx = fmaxf(mxx, xv);
      mny = fminf(mny, yv);
      mxy = fmaxf(mxy, yv);
      if (built) {
        const float tx = __fmul_rn(__fsub_rn(xv, x0), sc), ty = __fmul_rn(__fsub_rn(yv, y0), sc);
        out += !(tx >= 0.0f && tx < 65536.0f && ty >= 0.0f && ty < 65536.0f);
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
    blk[blockIdx.x] = cnt;
    if (cnt) {
      atomicMin(&ctl->mbr[0], fenc(mnx));
      atomicMin(&ctl->mbr[1], fenc(mny));
      atomicMax(&ctl->mbr[2], fenc(mxx));
      atomicMax(&ctl->mbr[3], fenc(mxy));
    }
    if (out) atomicAdd(&ctl->n_outside, out);
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

// Exclusive scan of the per-block present counts; rebuild decision; frame.
__global__ void __launch_bounds__(kChunkBlocks) k_decide(Ctl *ctl, uint32_t *blk,
                                                         uint32_t policy, uint32_t period) {
  __shared__ uint32_t lds[kChunkBlocks / kWave + 1];
  uint32_t total;
  uint32_t ex = block_excl_scan<uint32_t, kChunkBlocks>(blk[threadIdx.x], lds, &total);
  blk[threadIdx.x] = ex;
  if (threadIdx.x != 0) return;
  ctl->n_present = total;
  bool r = ctl->force || !ctl->built || policy == 1u;
  if (!r && policy == 0u) {
    r = ctl->since_build + 1 >= period || ctl->prev_max_leaf > 2u * ctl->th_cur ||
        (uint64_t)ctl->n_outside * 100u > total;
  }
  ctl->rebuild = r ? 1u : 0u;
  if (!r) {
    ctl->since_build += 1;
    return;
  }
  if (ctl->th_next) ctl->th_cur = ctl->th_next;
  ctl->th_next = 0;
  ctl->force = 0;
  ctl->built = 1;
  ctl->since_build = 0;
  float x0 = 0.0f, y0 = 0.0f;
  int32_t e = 0;
  if (total) {
    x0 = fdec(ctl->mbr[0]);
    y0 = fdec(ctl->mbr[1]);
    const float w = __fsub_rn(fdec(ctl->mbr[2]), x0), h = __fsub_rn(fdec(ctl->mbr[3]), y0);
    e = frame_exp(w > h ? w : h);
  }
  ctl->x0 = x0;
  ctl->y0 = y0;
  ctl->e = e;
  ctl->scale = __uint_as_float((uint32_t)(127 + kFine - e) << 23);
}

// Morton codes of present objects, compacted in id order.
__global__ void __launch_bounds__(kBlock) k_morton(const float *px, const float *py, uint32_t N,
                                                   const Ctl *ctl, const uint32_t *blk,
                                                   uint32_t *keys, uint32_t *vals) {
  __shared__ uint32_t lds[kWavesPerBlock + 1];
  const uint32_t chunk = (N + gridDim.x - 1) / gridDim.x;
  const uint64_t b0 = (uint64_t)blockIdx.x * chunk;
  const uint64_t b1 = b0 + chunk < N ? b0 + chunk : N;
  const float x0 = ctl->x0, y0 = ctl->y0, sc = ctl->scale;
  uint32_t base = blk[blockIdx.x];
  for (uint64_t t0 = b0; t0 < b1; t0 += kBlock) {
    const uint64_t i = t0 + threadIdx.x;
    const float xv = i < b1 ? px[i] : NAN;
    const bool pres = xv == xv;
    uint32_t tot;
    const uint32_t ex = block_excl_scan<uint32_t, kBlock>(pres ? 1u : 0u, lds, &tot);
    if (pres) {
      const float yv = py[i];
      keys[base + ex] = morton2(cell_of(xv, x0, sc), cell_of(yv, y0, sc));
      vals[base + ex] = (uint32_t)i;
    }
    base += tot;
  }
}

__global__ void __launch_bounds__(kBlock) k_gather(const float *px, const float *py,
                                                   const uint32_t *ids, const Ctl *ctl,
                                                   float2 *sxy) {
  const uint32_t n = ctl->n_present;
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const uint32_t o = ids[i];
    sxy[i] = make_float2(px[o], py[o]);
  }
}

// ----------------------------------------------------------------- build --
// Algorithm 1 on the device: the frontier of level l-1 holds the quadrants
// to split as intervals of the sorted codes; each is cut into its four
// level-l children by binary search; a child with more than th objects
// below l_max joins the next frontier, every other child (empty ones
// included) becomes a leaf.

__global__ void k_tree_init(Ctl *ctl, uint4 *front0) {
  if (!ctl->rebuild) return;
  front0[0] = make_uint4(0u, 0u, ctl->n_present, 0u);
  ctl->fcount[0] = 1;
  ctl->n_leaves = 0;
  ctl->l_deep = 0;
}

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
    bool ovf = false;
    if (valid) {
      for (uint32_t k = 0; k < 4; ++k) {
        const uint32_t cz = zp * 4u + k;
        if ((splitm >> k) & 1u) {
          if (fb < fcap) fout[fb] = make_uint4(cz, bnd[k], bnd[k + 1], 0u);
          else ovf = true;
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
    flag_error(ctl, kErrOvfTree, ovf);
    if (ballot(nleaf != 0) && lane_id() == 0) atomicMax(&ctl->l_deep, l);
  }
}

// The leaf table is sized for the worst case of the smallest threshold, so
// this never fires; if it did, the tick is flagged and no traversal runs.
__global__ void k_tree_done(Ctl *ctl, uint32_t lcap) {
  if (!ctl->rebuild) return;
  if (ctl->n_leaves > lcap) {
    ctl->n_leaves = lcap;
    ctl->err |= kErrOvfTree;
  }
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

__global__ void __launch_bounds__(kBlock) k_nodes_build(Ctl *ctl, const uint32_t *lstart,
                                                        const uint32_t *llevel,
                                                        const uint32_t *node_off, uint4 *nodes,
                                                        uint32_t ncap) {
  if (!ctl->rebuild) return;
  const uint32_t n = ctl->n_leaves;
  for (uint32_t t = blockIdx.x * kBlock + threadIdx.x; t < n; t += gridDim.x * kBlock) {
    const uint32_t s = lstart[t], l = llevel[t], k0 = open_level(s);
    for (uint32_t k = k0; k < l; ++k) {
      const uint32_t idx = node_off[t] + (k - k0);
      const uint32_t p = k == 0 ? 0u : s >> (2u * (kFine - k));
      uint32_t ref[4];
      bool bad = false;
      for (uint32_t c = 0; c < 4; ++c) {
        const uint32_t cs = (p * 4u + c) << (2u * (kFine - k - 1));
        const uint32_t u = lower_bound_u32(lstart, 0u, n, cs);
        if (u >= n || lstart[u] != cs) {
          bad = true;
          ref[c] = kLeafBit;
          continue;
        }
        const uint32_t lu = llevel[u];
        ref[c] = lu == k + 1 ? (kLeafBit | u) : node_off[u] + (k + 1 - open_level(cs));
      }
      if (bad) atomicOr(&ctl->err, kErrOvfTree);
      if (idx < ncap) nodes[idx] = make_uint4(ref[0], ref[1], ref[2], ref[3]);
      else atomicOr(&ctl->err, kErrOvfTree);
    }
  }
}

// ---------------------------------------------------------------- leaves --

__global__ void __launch_bounds__(kBlock) k_leaf_ranges(const Ctl *ctl, const uint32_t *codes,
                                                        const uint32_t *lstart, uint32_t *leaf_beg,
                                                        uint32_t *leaf_nsq) {
  const uint32_t n = ctl->n_leaves, np = ctl->n_present;
  for (uint32_t t = blockIdx.x * kBlock + threadIdx.x; t < n; t += gridDim.x * kBlock) {
    leaf_beg[t] = lower_bound_u32(codes, 0u, np, lstart[t]);
    leaf_nsq[t] = 0u;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) leaf_beg[n] = np;
}

__global__ void __launch_bounds__(kBlock) k_leaf_stats(Ctl *ctl, const uint32_t *leaf_beg,
                                                       const uint32_t *llevel, uint32_t l_max) {
  const uint32_t n = ctl->n_leaves;
  const uint32_t nr = (n + kWave - 1) / kWave * kWave;
  for (uint32_t t = blockIdx.x * kBlock + threadIdx.x; t < nr; t += gridDim.x * kBlock) {
    uint32_t c = 0;
    if (t < n && llevel[t] < l_max) c = leaf_beg[t + 1] - leaf_beg[t];
    c = wave_max(c);
    if (lane_id() == 0 && c) atomicMax(&ctl->max_leaf, c);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && (ctl->err & kErrOvfTree)) ctl->built = 0;
}

// ----------------------------------------------------------------- split --
// Query splitting (mapping function g): the corners are mapped through the
// same cell function as the objects (clamped to the frame); a depth-first
// walk of the node table visits every leaf whose finest-level cell range
// overlaps the query's.  A leaf strictly inside the query's cell range on
// both axes is covering; any other overlapping leaf is intersecting.
// Leaves without objects are skipped (they are inactive).

struct QBox {
  uint32_t i0, i1, j0, j1;
};

template <typename Visit>
__device__ __forceinline__ void walk_leaves(const uint4 *__restrict__ nodes, uint32_t *stack,
                                            const QBox q, Visit &&visit) {
  uint32_t node = 0, depth = 0, pi = 0, pj = 0, c = 0;
  uint4 rec = nodes[0];
  while (true) {
    if (c < 4) {
      const uint32_t ref = c == 0 ? rec.x : c == 1 ? rec.y : c == 2 ? rec.z : rec.w;
      const uint32_t ci = 2u * pi + (c & 1u), cj = 2u * pj + (c >> 1);
      const uint32_t s = (uint32_t)kFine - (depth + 1);
      const uint32_t ilo = ci << s, ihi = ilo + ((1u << s) - 1u);
      const uint32_t jlo = cj << s, jhi = jlo + ((1u << s) - 1u);
      const bool ov = ilo <= q.i1 && q.i0 <= ihi && jlo <= q.j1 && q.j0 <= jhi;
      if (ov && !(ref & kLeafBit) && depth + 1 < (uint32_t)kFine) {
        stack[depth * kBlock] = node;
        ++depth;
        node = ref;
        pi = ci;
        pj = cj;
        c = 0;
        rec = nodes[node];
        continue;
      }
      if (ov) visit(ref & ~kLeafBit, q.i0 < ilo && ihi < q.i1 && q.j0 < jlo && jhi < q.j1);
      ++c;
    } else {
      if (depth == 0) break;
      --depth;
      c = ((pi & 1u) | ((pj & 1u) << 1)) + 1u;
      pi >>= 1;
      pj >>= 1;
      node = stack[depth * kBlock];
      rec = nodes[node];
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_q_stamp(const uint32_t *qid, uint32_t nq, uint32_t N,
                                                    uint64_t *qstamp, Ctl *ctl) {
  const uint64_t seq = ctl->qry_seq;
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

__global__ void __launch_bounds__(kBlock) k_q_count(
    Ctl *ctl, const uint32_t *qid, const float *xa, const float *ya, const float *xb,
    const float *yb, uint32_t nq, uint32_t N, const uint64_t *qstamp, const uint4 *nodes,
    const uint32_t *leaf_beg, float4 *qrect, uint32_t *q_ni, uint32_t *q_nc, uint32_t *leaf_nsq,
    uint32_t covering) {
  __shared__ uint32_t stack[kFine * kBlock];
  const uint64_t seq = ctl->qry_seq;
  const bool tree_ok = !(ctl->err & kErrOvfTree);
  const uint32_t nr = (nq + kWave - 1) / kWave * kWave;
  for (uint32_t k = blockIdx.x * kBlock + threadIdx.x; k < nr; k += gridDim.x * kBlock) {
    bool bad_rect = false;
    uint32_t ni = 0, nc = 0;
    if (k < nq) {
      const float4 r = make_float4(xa[k], ya[k], xb[k], yb[k]);
      qrect[k] = r;
      QBox q;
      if (query_box(ctl, k, qid[k], N, qstamp, seq, r, &q, &bad_rect) && tree_ok) {
        walk_leaves(nodes, stack + threadIdx.x, q, [&](uint32_t leaf, bool cov) {
          if (leaf_beg[leaf + 1] == leaf_beg[leaf]) return;
          if (cov && covering) {
            ++nc;
          } else {
            ++ni;
            atomicAdd(&leaf_nsq[leaf], 1u);
          }
        });
      }
      q_ni[k] = ni;
      q_nc[k] = nc;
    }
    flag_error(ctl, kErrQueryRect, bad_rect);
  }
}

// Capacities of the tick's subqueries.
__global__ void k_split_check(Ctl *ctl, uint64_t cap_sq, uint64_t cap_cov, uint32_t *n32) {
  uint32_t err = 0;
  if (ctl->n_isect > cap_sq) err |= kErrOvfSubq;
  if (ctl->n_cov > cap_cov) err |= kErrOvfCov;
  if (ctl->err & kErrOvfTree) err |= kErrOvfTree;
  ctl->err |= err;
  ctl->go_split = err ? 0u : 1u;
  n32[0] = err ? 0u : (uint32_t)ctl->n_isect;
  n32[1] = err ? 0u : (uint32_t)ctl->n_cov;
}

__global__ void __launch_bounds__(kBlock) k_q_write(
    Ctl *ctl, const uint32_t *qid, uint32_t nq, uint32_t N, const uint64_t *qstamp,
    const uint4 *nodes, const uint32_t *leaf_beg, const float4 *qrect, const uint32_t *q_ioff,
    const uint32_t *q_coff, const uint32_t *leaf_sqoff, uint32_t *leaf_nsq, uint32_t *sq_q,
    uint32_t *sq_s, uint32_t *cov_leaf, uint32_t covering) {
  if (!ctl->go_split) return;
  __shared__ uint32_t stack[kFine * kBlock];
  const uint64_t seq = ctl->qry_seq;
  uint64_t covp = 0;
  for (uint32_t k = blockIdx.x * kBlock + threadIdx.x; k < nq; k += gridDim.x * kBlock) {
    QBox q;
    bool bad_rect;
    if (!query_box(ctl, k, qid[k], N, qstamp, seq, qrect[k], &q, &bad_rect)) continue;
    uint32_t wi = q_ioff[k], wc = q_coff[k];
    walk_leaves(nodes, stack + threadIdx.x, q, [&](uint32_t leaf, bool cov) {
      const uint32_t cnt = leaf_beg[leaf + 1] - leaf_beg[leaf];
      if (cnt == 0) return;
      if (cov && covering) {
        cov_leaf[wc++] = leaf;
        covp += cnt;
      } else {
        const uint32_t slot = leaf_sqoff[leaf] + atomicSub(&leaf_nsq[leaf], 1u) - 1u;
        sq_q[slot] = k;
        sq_s[slot] = wi++;
      }
    });
  }
  covp = wave_sum(covp);
  if (lane_id() == 0 && covp) atomicAdd((unsigned long long *)&ctl->cov_pairs, (unsigned long long)covp);
}

// -------------------------------------------------------------- schedule --
// Tasks = leaves with at least one intersecting subquery, in Morton order;
// with reordering, heaviest first (weight = subqueries x objects), ties in
// leaf order (the sort is stable).

__global__ void __launch_bounds__(kBlock) k_task_flags(const Ctl *ctl, const uint32_t *leaf_sqoff,
                                                       uint32_t *tflag) {
  const uint32_t n = ctl->go_split ? ctl->n_leaves : 0u;
  for (uint32_t t = blockIdx.x * kBlock + threadIdx.x; t < n; t += gridDim.x * kBlock)
    tflag[t] = leaf_sqoff[t + 1] > leaf_sqoff[t] ? 1u : 0u;
}

__global__ void __launch_bounds__(kBlock) k_task_write(Ctl *ctl, const uint32_t *tflag,
                                                       const uint32_t *toff,
                                                       const uint32_t *leaf_beg,
                                                       const uint32_t *leaf_sqoff,
                                                       uint32_t *tasks, uint32_t *tkey) {
  const uint32_t n = ctl->go_split ? ctl->n_leaves : 0u;
  for (uint32_t t = blockIdx.x * kBlock + threadIdx.x; t < n; t += gridDim.x * kBlock) {
    if (!tflag[t]) continue;
    const uint32_t pos = toff[t];
    const uint64_t w =
        (uint64_t)(leaf_sqoff[t + 1] - leaf_sqoff[t]) * (leaf_beg[t + 1] - leaf_beg[t]);
    tasks[pos] = t;
    tkey[pos] = 0xffffffffu - (uint32_t)(w < 0xffffffffull ? w : 0xffffffffull);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl->n_tasks = n ? toff[n] : 0u;
}

// ------------------------------------------------------------------ join --
// One wave per task (leaf).  Objects of the leaf are taken 64 at a time, one
// per lane; intersecting subqueries of the leaf 64 at a time, one per lane,
// and broadcast to the wave one after the other.  The ballot of the closed
// containment test is the subquery's 64-bit bitmap word for those objects:
// its popcount is the count (pass 1), and in pass 2 every lane with its bit
// set writes its object id at the subquery's offset plus the number of set
// bits below it (coalesced, no atomics, no bitmap in memory).

__global__ void __launch_bounds__(kBlock) k_join_count(Ctl *ctl, const uint32_t *tasks,
                                                       const uint32_t *leaf_beg,
                                                       const uint32_t *leaf_sqoff,
                                                       const uint32_t *sq_q, const uint32_t *sq_s,
                                                       const float4 *qrect, const float2 *sxy,
                                                       uint32_t *sq_cnt) {
  if (!ctl->go_split) return;
  const uint32_t nt = ctl->n_tasks;
  const uint32_t lane = lane_id();
  const uint32_t nwaves = gridDim.x * kWavesPerBlock;
  uint64_t tests = 0;
  for (uint32_t t = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; t < nt; t += nwaves) {
    const uint32_t leaf = tasks[t];
    const uint32_t ob = leaf_beg[leaf], oe = leaf_beg[leaf + 1];
    const uint32_t sb = leaf_sqoff[leaf], se = leaf_sqoff[leaf + 1];
    tests += (uint64_t)(oe - ob) * (se - sb);
    for (uint32_t sc = sb; sc < se; sc += kWave) {
      const uint32_t nk = min((uint32_t)kWave, se - sc);
      float4 r = make_float4(0.f, 0.f, 0.f, 0.f);
      uint32_t slot = 0, cnt = 0;
      if (lane < nk) {
        slot = sq_s[sc + lane];
        r = qrect[sq_q[sc + lane]];
      }
      for (uint32_t o = ob; o < oe; o += kWave) {
        const bool has = o + lane < oe;
        const float2 p = has ? sxy[o + lane] : make_float2(0.f, 0.f);
        for (uint32_t kk = 0; kk < nk; ++kk) {
          const float qxa = readlane_f(r.x, kk), qya = readlane_f(r.y, kk);
          const float qxb = readlane_f(r.z, kk), qyb = readlane_f(r.w, kk);
          const bool in = has && qxa <= p.x && p.x <= qxb && qya <= p.y && p.y <= qyb;
          const uint32_t c = (uint32_t)__popcll(ballot(in));
          if (lane == kk) cnt += c;
        }
      }
      if (lane < nk) sq_cnt[slot] = cnt;
    }
  }
  if (lane == 0 && tests) atomicAdd((unsigned long long *)&ctl->tests, (unsigned long long)tests);
}

__global__ void k_join_check(Ctl *ctl, uint64_t cap_res) {
  if (!ctl->go_split) return;
  if (ctl->n_res > cap_res) {
    ctl->err |= kErrOvfRes;
    ctl->go_join = 0;
  } else {
    ctl->go_join = 1;
  }
}

__global__ void __launch_bounds__(kBlock) k_join_write(const Ctl *ctl, const uint32_t *tasks,
                                                       const uint32_t *leaf_beg,
                                                       const uint32_t *leaf_sqoff,
                                                       const uint32_t *sq_q, const uint32_t *sq_s,
                                                       const float4 *qrect, const float2 *sxy,
                                                       const uint32_t *sid,
                                                       const uint64_t *res_off,
                                                       uint32_t *res_ids) {
  if (!ctl->go_join) return;
  const uint32_t nt = ctl->n_tasks;
  const uint32_t lane = lane_id();
  const uint32_t nwaves = gridDim.x * kWavesPerBlock;
  for (uint32_t t = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; t < nt; t += nwaves) {
    const uint32_t leaf = tasks[t];
    const uint32_t ob = leaf_beg[leaf], oe = leaf_beg[leaf + 1];
    const uint32_t sb = leaf_sqoff[leaf], se = leaf_sqoff[leaf + 1];
    for (uint32_t sc = sb; sc < se; sc += kWave) {
      const uint32_t nk = min((uint32_t)kWave, se - sc);
      float4 r = make_float4(0.f, 0.f, 0.f, 0.f);
      uint64_t off = 0;
      if (lane < nk) {
        off = res_off[sq_s[sc + lane]];
        r = qrect[sq_q[sc + lane]];
      }
      for (uint32_t o = ob; o < oe; o += kWave) {
        const bool has = o + lane < oe;
        const float2 p = has ? sxy[o + lane] : make_float2(0.f, 0.f);
        const uint32_t id = has ? sid[o + lane] : 0u;
        for (uint32_t kk = 0; kk < nk; ++kk) {
          const float qxa = readlane_f(r.x, kk), qya = readlane_f(r.y, kk);
          const float qxb = readlane_f(r.z, kk), qyb = readlane_f(r.w, kk);
          const bool in = has && qxa <= p.x && p.x <= qxb && qya <= p.y && p.y <= qyb;
          const uint64_t m = ballot(in);
          const uint64_t base = readlane_u64(off, kk);
          if (in) res_ids[base + mbcnt(m)] = id;
          if (lane == kk) off += (uint64_t)__popcll(m);
        }
      }
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_q_final(Ctl *ctl, uint32_t nq, const uint32_t *q_ioff,
                                                    const uint64_t *res_off, uint64_t *q_roff,
                                                    const uint32_t *n32) {
  const bool ok = ctl->go_join != 0;
  for (uint32_t k = blockIdx.x * kBlock + threadIdx.x; k <= nq; k += gridDim.x * kBlock)
    q_roff[k] = ok ? res_off[k < nq ? q_ioff[k] : n32[0]] : 0ull;
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

__global__ void k_tick_end(Ctl *ctl, uint32_t nq) {
  ctl->qry_seq += nq;
  ctl->tick += 1;
}

// --------------------------------------------------------------- results --

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__global__ void __launch_bounds__(kBlock) k_hash(const Ctl *ctl, uint32_t nq, const uint32_t *qid,
                                                 const uint64_t *q_roff, const uint32_t *res_ids,
                                                 const uint32_t *q_coff, const uint32_t *cov_leaf,
                                                 const uint32_t *leaf_beg, const uint32_t *sid,
                                                 uint64_t *out_cnt, uint64_t *out_hash) {
  const uint32_t lane = lane_id();
  const uint32_t nwaves = gridDim.x * kWavesPerBlock;
  const bool ok = ctl->go_join != 0;
  for (uint32_t k = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; k < nq; k += nwaves) {
    if (!ok) {
      if (lane == 0) out_cnt[k] = out_hash[k] = 0ull;
      continue;
    }
    const uint64_t hi = (uint64_t)qid[k] << 32;
    uint64_t h = 0, c = 0;
    for (uint64_t i = q_roff[k] + lane; i < q_roff[k + 1]; i += kWave) {
      h += mix64(hi | res_ids[i]);
      ++c;
    }
    for (uint32_t e = q_coff[k]; e < q_coff[k + 1]; ++e) {
      const uint32_t leaf = cov_leaf[e];
      for (uint32_t i = leaf_beg[leaf] + lane; i < leaf_beg[leaf + 1]; i += kWave) {
        h += mix64(hi | sid[i]);
        ++c;
      }
    }
    h = wave_sum(h);
    c = wave_sum(c);
    if (lane == 0) {
      out_cnt[k] = c;
      out_hash[k] = h;
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_exp_count(const Ctl *ctl, uint32_t nq,
                                                      const uint64_t *q_roff,
                                                      const uint32_t *q_coff,
                                                      const uint32_t *cov_leaf,
                                                      const uint32_t *leaf_beg, uint32_t *cnt) {
  const bool ok = ctl->go_join != 0;
  for (uint32_t k = blockIdx.x * kBlock + threadIdx.x; k < nq; k += gridDim.x * kBlock) {
    if (!ok) {
      cnt[k] = 0u;
      continue;
    }
    uint64_t c = q_roff[k + 1] - q_roff[k];
    for (uint32_t e = q_coff[k]; e < q_coff[k + 1]; ++e)
      c += leaf_beg[cov_leaf[e] + 1] - leaf_beg[cov_leaf[e]];
    cnt[k] = (uint32_t)c;
  }
}

__global__ void __launch_bounds__(kBlock) k_exp_write(const Ctl *ctl, uint32_t nq,
                                                      const uint64_t *q_roff,
                                                      const uint32_t *res_ids,
                                                      const uint32_t *q_coff,
                                                      const uint32_t *cov_leaf,
                                                      const uint32_t *leaf_beg,
                                                      const uint32_t *sid, const uint64_t *off,
                                                      uint32_t *ids) {
  if (!ctl->go_join) return;
  const uint32_t lane = lane_id();
  const uint32_t nwaves = gridDim.x * kWavesPerBlock;
  for (uint32_t k = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; k < nq; k += nwaves) {
    uint64_t dst = off[k];
    const uint64_t a = q_roff[k], b = q_roff[k + 1];
    for (uint64_t i = a + lane; i < b; i += kWave) ids[dst + (i - a)] = res_ids[i];
    dst += b - a;
    for (uint32_t e = q_coff[k]; e < q_coff[k + 1]; ++e) {
      const uint32_t leaf = cov_leaf[e];
      const uint32_t lb = leaf_beg[leaf], le = leaf_beg[leaf + 1];
      for (uint32_t i = lb + lane; i < le; i += kWave) ids[dst + (i - lb)] = sid[i];
      dst += le - lb;
    }
  }
}

// ------------------------------------------------------- host launchers --

#define LAUNCH(k, g, b, s, ...) hipLaunchKernelGGL(k, dim3(g), dim3(b), 0, s, __VA_ARGS__)

void launch_ctl_init(Ctl *ctl, uint32_t th, hipStream_t s) { LAUNCH(k_ctl_init, 1, 1, s, ctl, th); }
void launch_request_build(Ctl *ctl, uint32_t th, hipStream_t s) {
  LAUNCH(k_request_build, 1, 1, s, ctl, th);
}
void launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s) {
  LAUNCH(k_fill_u32, grid_for(n), kBlock, s, p, n, v);
}
void launch_fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s) {
  LAUNCH(k_fill_u64, grid_for(n), kBlock, s, p, n, v);
}

void launch_updates(const Bufs &B, const uint32_t *id, const float *x, const float *y, uint32_t m,
                    hipStream_t s) {
  const unsigned g = grid_for(m);
  LAUNCH(k_upd_stamp, g, kBlock, s, id, x, y, m, B.N, B.ustamp, B.ctl);
  LAUNCH(k_upd_write, g, kBlock, s, id, x, y, m, B.N, (const uint64_t *)B.ustamp,
         (const Ctl *)B.ctl, B.px, B.py);
  LAUNCH(k_upd_end, 1, 1, s, B.ctl, m);
}

void launch_index(const Bufs &B, uint32_t policy, uint32_t period, hipStream_t s) {
  LAUNCH(k_tick_begin, 1, 1, s, B.ctl);
  LAUNCH(k_mbr, kChunkBlocks, kBlock, s, (const float *)B.px, (const float *)B.py, B.N, B.ctl,
         B.blk);
  LAUNCH(k_decide, 1, kChunkBlocks, s, B.ctl, B.blk, policy, period);
  LAUNCH(k_morton, kChunkBlocks, kBlock, s, (const float *)B.px, (const float *)B.py, B.N,
         (const Ctl *)B.ctl, (const uint32_t *)B.blk, B.keyA, B.valA);
  radix_sort_pairs(B.keyA, B.valA, B.keyB, B.valB, &B.ctl->n_present, nullptr, B.hist, B.tot, 0,
                   32, s);
  LAUNCH(k_gather, grid_for(B.N), kBlock, s, (const float *)B.px, (const float *)B.py,
         (const uint32_t *)B.valA, (const Ctl *)B.ctl, B.sxy);
}

void launch_build(const Bufs &B, uint32_t l_max, hipStream_t s) {
  LAUNCH(k_tree_init, 1, 1, s, B.ctl, B.front[0]);
  for (uint32_t l = 1; l <= l_max; ++l) {
    LAUNCH(k_tree_level, grid_for(B.FCAP), kBlock, s, B.ctl, l, l_max, (const uint32_t *)B.keyA,
           (const uint4 *)B.front[(l - 1) & 1], B.front[l & 1], B.FCAP, B.lstart, B.llevel,
           B.LCAP);
  }
  LAUNCH(k_tree_done, 1, 1, s, B.ctl, B.LCAP);
  radix_sort_pairs(B.lstart, B.llevel, B.lstart2, B.llevel2, &B.ctl->n_leaves, &B.ctl->rebuild,
                   B.hist, B.tot, 0, 32, s);
  LAUNCH(k_nodes_open, grid_for(B.LCAP), kBlock, s, (const Ctl *)B.ctl,
         (const uint32_t *)B.lstart, (const uint32_t *)B.llevel, B.nopen);
  scan_excl<uint32_t>(B.nopen, B.node_off, &B.ctl->n_leaves, 0, B.part, nullptr,
                      &B.ctl->rebuild, s);
  LAUNCH(k_nodes_build, grid_for(B.LCAP), kBlock, s, B.ctl, (const uint32_t *)B.lstart,
         (const uint32_t *)B.llevel, (const uint32_t *)B.node_off, B.nodes, B.NCAP);
}

void launch_leaves(const Bufs &B, uint32_t l_max, hipStream_t s) {
  LAUNCH(k_leaf_ranges, grid_for(B.LCAP), kBlock, s, (const Ctl *)B.ctl,
         (const uint32_t *)B.keyA, (const uint32_t *)B.lstart, B.leaf_beg, B.leaf_nsq);
  LAUNCH(k_leaf_stats, grid_for(B.LCAP), kBlock, s, B.ctl, (const uint32_t *)B.leaf_beg,
         (const uint32_t *)B.llevel, l_max);
}

void launch_split(const Bufs &B, const uint32_t *qid, const float *xa, const float *ya,
                  const float *xb, const float *yb, uint32_t nq, uint32_t covering,
                  hipStream_t s) {
  const unsigned gq = grid_for(nq, 4096);
  LAUNCH(k_q_stamp, gq, kBlock, s, qid, nq, B.N, B.qstamp, B.ctl);
  LAUNCH(k_q_count, gq, kBlock, s, B.ctl, qid, xa, ya, xb, yb, nq, B.N,
         (const uint64_t *)B.qstamp, (const uint4 *)B.nodes, (const uint32_t *)B.leaf_beg,
         B.qrect, B.q_ni, B.q_nc, B.leaf_nsq, covering);
  scan_excl<uint32_t>(B.q_ni, B.q_ioff, nullptr, nq, B.part, &B.ctl->n_isect, nullptr, s);
  scan_excl<uint32_t>(B.q_nc, B.q_coff, nullptr, nq, B.part, &B.ctl->n_cov, nullptr, s);
  scan_excl<uint32_t>(B.leaf_nsq, B.leaf_sqoff, &B.ctl->n_leaves, 0, B.part, nullptr, nullptr, s);
  LAUNCH(k_split_check, 1, 1, s, B.ctl, B.S, B.C, B.n32);
  LAUNCH(k_q_write, gq, kBlock, s, B.ctl, qid, nq, B.N, (const uint64_t *)B.qstamp,
         (const uint4 *)B.nodes, (const uint32_t *)B.leaf_beg, (const float4 *)B.qrect,
         (const uint32_t *)B.q_ioff, (const uint32_t *)B.q_coff, (const uint32_t *)B.leaf_sqoff,
         B.leaf_nsq, B.sq_q, B.sq_s, B.cov_leaf, covering);
}

void launch_schedule(const Bufs &B, uint32_t reorder, hipStream_t s) {
  LAUNCH(k_task_flags, grid_for(B.LCAP), kBlock, s, (const Ctl *)B.ctl,
         (const uint32_t *)B.leaf_sqoff, B.tflag);
  scan_excl<uint32_t>(B.tflag, B.toff, &B.ctl->n_leaves, 0, B.part, nullptr, &B.ctl->go_split,
                      s);
  LAUNCH(k_task_write, grid_for(B.LCAP), kBlock, s, B.ctl, (const uint32_t *)B.tflag,
         (const uint32_t *)B.toff, (const uint32_t *)B.leaf_beg, (const uint32_t *)B.leaf_sqoff,
         B.tasks, B.tkey);
  if (reorder)
    radix_sort_pairs(B.tkey, B.tasks, B.tkey2, B.tasks2, &B.ctl->n_tasks, &B.ctl->go_split,
                     B.hist, B.tot, 0, 32, s);
}

void launch_join_count(const Bufs &B, hipStream_t s) {
  LAUNCH(k_join_count, kJoinBlocks, kBlock, s, B.ctl, (const uint32_t *)B.tasks,
         (const uint32_t *)B.leaf_beg, (const uint32_t *)B.leaf_sqoff, (const uint32_t *)B.sq_q,
         (const uint32_t *)B.sq_s, (const float4 *)B.qrect, (const float2 *)B.sxy, B.sq_cnt);
}

void launch_join_scan(const Bufs &B, uint64_t cap_res, hipStream_t s) {
  scan_excl<uint64_t>(B.sq_cnt, B.res_off, &B.n32[0], 0, B.part, &B.ctl->n_res, &B.ctl->go_split,
                      s);
  LAUNCH(k_join_check, 1, 1, s, B.ctl, cap_res);
}

void launch_join_write(const Bufs &B, hipStream_t s) {
  LAUNCH(k_join_write, kJoinBlocks, kBlock, s, (const Ctl *)B.ctl, (const uint32_t *)B.tasks,
         (const uint32_t *)B.leaf_beg, (const uint32_t *)B.leaf_sqoff, (const uint32_t *)B.sq_q,
         (const uint32_t *)B.sq_s, (const float4 *)B.qrect, (const float2 *)B.sxy,
         (const uint32_t *)B.valA, (const uint64_t *)B.res_off, B.res_ids);
}

void launch_finish(const Bufs &B, uint32_t nq, hipStream_t s) {
  LAUNCH(k_q_final, grid_for(nq + 1, 4096), kBlock, s, B.ctl, nq, (const uint32_t *)B.q_ioff,
         (const uint64_t *)B.res_off, B.q_roff, (const uint32_t *)B.n32);
  LAUNCH(k_tick_end, 1, 1, s, B.ctl, nq);
}

void launch_counters(const Bufs &B, uint64_t *out, hipStream_t s) {
  LAUNCH(k_counters, 1, 1, s, (const Ctl *)B.ctl, out);
}

void launch_hash(const Bufs &B, uint32_t nq, const uint32_t *qid, uint64_t *cnt, uint64_t *hash,
                 hipStream_t s) {
  LAUNCH(k_hash, grid_for((uint64_t)nq * kWave, 4096), kBlock, s, (const Ctl *)B.ctl, nq, qid,
         (const uint64_t *)B.q_roff, (const uint32_t *)B.res_ids, (const uint32_t *)B.q_coff,
         (const uint32_t *)B.cov_leaf, (const uint32_t *)B.leaf_beg, (const uint32_t *)B.valA,
         cnt, hash);
}

void launch_expand(const Bufs &B, uint32_t nq, uint64_t *off, uint32_t *ids, hipStream_t s) {
  LAUNCH(k_exp_write, grid_for((uint64_t)nq * kWave, 4096), kBlock, s, (const Ctl *)B.ctl, nq,
         (const uint64_t *)B.q_roff, (const uint32_t *)B.res_ids, (const uint32_t *)B.q_coff,
         (const uint32_t *)B.cov_leaf, (const uint32_t *)B.leaf_beg, (const uint32_t *)B.valA,
         (const uint64_t *)off, ids);
}

void launch_expand_count(const Bufs &B, uint32_t nq, uint64_t *off, hipStream_t s) {
  LAUNCH(k_exp_count, grid_for(nq, 4096), kBlock, s, (const Ctl *)B.ctl, nq,
         (const uint64_t *)B.q_roff,
         (const uint32_t *)B.q_coff, (const uint32_t *)B.cov_leaf, (const uint32_t *)B.leaf_beg,
         B.q_ni);
  scan_excl<uint64_t>(B.q_ni, off, nullptr, nq, B.part, nullptr, nullptr, s);
}

}  // namespace sj
