// Data-parallel primitives of libsj: chunked multi-array exclusive scans and
// a stable LDS-staged LSD radix sort of (u32 key, u32 value) pairs.
//
// All kernels take their element counts from device memory (or from a host
// value) and an optional gate word: when the gate reads 0 the kernel returns
// at once.  Grids are fixed, so a launch sequence does not depend on sizes
// produced on the device.
#include "sj_device.h"
#include "sj_host.h"

#include <utility>

namespace sj {

__device__ __forceinline__ bool gated(const uint32_t *gate) { return gate && *gate == 0u; }

// Role of a radix pass when the keys fit in *skip bits (a multiple of 8,
// at least 8): the passes below sort; the passes above have a zero digit
// for every key and are identities.  Identities run in pairs as nothing (the
// data returns to the same buffer), and one left over runs as a copy.
enum : int { kPassSort = 0, kPassCopy = 1, kPassNone = 2 };
__device__ __forceinline__ int pass_role(const uint32_t *skip, int shift) {
  if (!skip) return kPassSort;
  const uint32_t np = *skip / 8u, p = (uint32_t)shift / 8u;
  if (p < np) return kPassSort;
  return (p == np && (np & 1u)) ? kPassCopy : kPassNone;
}

// ---------------------------------------------------------------- scans --
// Block b of kChunkBlocks owns the contiguous chunk [b*chunk, (b+1)*chunk)
// of every array.  reduce: chunk sums -> part[job][b]; a single-block "top"
// kernel scans part[job][*] (scan_partials) and stores the totals; down:
// every block scans its chunk with its partial as carry-in.

__global__ void __launch_bounds__(kBlock) k_mscan_reduce(ScanJobs jobs, uint64_t *part,
                                                         const uint32_t *gate) {
  if (gated(gate)) return;
  __shared__ uint64_t lds[kWavesPerBlock];
  const ScanJob &j = jobs.j[blockIdx.y];
  const uint32_t n = job_n(j);
  const uint32_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const uint64_t b0 = (uint64_t)blockIdx.x * chunk;
  const uint64_t b1 = b0 + chunk < n ? b0 + chunk : n;
  // four rows of loads in flight per thread
  uint64_t s = 0;
  for (uint64_t t0 = b0; t0 < b1; t0 += 4u * kBlock) {
    uint32_t v[4];
#pragma unroll
    for (uint32_t r = 0; r < 4u; ++r) {
      const uint64_t i = t0 + r * kBlock + threadIdx.x;
      v[r] = i < b1 ? job_in(j, i) : 0u;
    }
#pragma unroll
    for (uint32_t r = 0; r < 4u; ++r) s += v[r];
  }
  s = wave_sum(s);
  if (lane_id() == 0) lds[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
    for (int w = 0; w < kWavesPerBlock; ++w) t += lds[w];
    part[blockIdx.y * kChunkBlocks + blockIdx.x] = t;
  }
}

__global__ void __launch_bounds__(kBlock) k_mscan_down(ScanJobs jobs, const uint64_t *part,
                                                       const uint32_t *gate) {
  if (gated(gate)) return;
  __shared__ uint64_t lds[kWavesPerBlock + 1];
  const ScanJob &j = jobs.j[blockIdx.y];
  const uint32_t n = job_n(j);
  const uint32_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const uint64_t b0 = (uint64_t)blockIdx.x * chunk;
  const uint64_t b1 = b0 + chunk < n ? b0 + chunk : n;
  uint64_t run = part[blockIdx.y * kChunkBlocks + blockIdx.x];
  // the loads of four rows are issued before the first row is scanned
  for (uint64_t t0 = b0; t0 < b1; t0 += 4u * kBlock) {
    uint32_t v[4];
#pragma unroll
    for (uint32_t r = 0; r < 4u; ++r) {
      const uint64_t i = t0 + r * kBlock + threadIdx.x;
      v[r] = i < b1 ? job_in(j, i) : 0u;
    }
#pragma unroll
    for (uint32_t r = 0; r < 4u; ++r) {
      if (t0 + r * kBlock >= b1) break;  // uniform over the block
      const uint64_t i = t0 + r * kBlock + threadIdx.x;
      uint64_t tot;
      const uint64_t ex = block_excl_scan<uint64_t, kBlock>(v[r], lds, &tot);
      if (i < b1) job_store(j, i, run + ex);
      run += tot;
    }
  }
}

// Generic top: totals to out[n] and optionally to total_out[job].
__global__ void __launch_bounds__(kChunkBlocks) k_mscan_top(ScanJobs jobs, int njobs,
                                                            uint64_t *part, const uint32_t *gate,
                                                            uint64_t *t0, uint64_t *t1,
                                                            uint64_t *t2) {
  if (gated(gate)) return;
  __shared__ uint64_t lds[kChunkBlocks / kWave + 1];
  uint64_t *tout[3] = {t0, t1, t2};
  for (int q = 0; q < njobs; ++q) {
    const uint64_t total = scan_partials(part + q * kChunkBlocks, lds);
    if (threadIdx.x == 0) {
      job_store(jobs.j[q], job_n(jobs.j[q]), total);
      if (tout[q]) *tout[q] = total;
    }
  }
}

void mscan_reduce(const ScanJobs &jobs, int njobs, uint64_t *part, const uint32_t *gate,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_mscan_reduce, dim3(kChunkBlocks, njobs), dim3(kBlock), 0, s, jobs, part,
                     gate);
}

void mscan_down(const ScanJobs &jobs, int njobs, const uint64_t *part, const uint32_t *gate,
                hipStream_t s) {
  hipLaunchKernelGGL(k_mscan_down, dim3(kChunkBlocks, njobs), dim3(kBlock), 0, s, jobs, part,
                     gate);
}

void mscan(const ScanJobs &jobs, int njobs, uint64_t *part, const uint32_t *gate,
           uint64_t *total0, hipStream_t s) {
  mscan_reduce(jobs, njobs, part, gate, s);
  hipLaunchKernelGGL(k_mscan_top, dim3(1), dim3(kChunkBlocks), 0, s, jobs, njobs, part, gate,
                     total0, (uint64_t *)nullptr, (uint64_t *)nullptr);
  mscan_down(jobs, njobs, part, gate, s);
}

ScanJob job_u32(const uint32_t *in, uint32_t *out, const uint32_t *n_dev, uint32_t n_host,
                const uint32_t *in2) {
  return ScanJob{in, in2, out, n_dev, n_host, 0u};
}
ScanJob job_u64(const uint32_t *in, uint64_t *out, const uint32_t *n_dev, uint32_t n_host) {
  return ScanJob{in, nullptr, out, n_dev, n_host, 1u};
}

// ----------------------------------------------------------- radix sort --
// One pass sorts by the 8-bit digit (key >> shift) & 255, stably:
//  hist:    per-block digit histograms, digit-major hist[d * B + b];
//  hscan:   exclusive scan over blocks of every digit, digit totals tot[d];
//  scatter: every block ranks its keys tile by tile (wave ballots give the
//           rank among equal digits of a wave), places the tile in LDS in
//           digit order and writes each digit's run contiguously to its
//           global offset.  A float2 per pair can travel with it (the
//           objects' positions: sorted with their ids, they need no gather
//           by id, which would read one random line per object).
// Passes above the device value *skip only copy or do nothing (pass_role).

__global__ void __launch_bounds__(kBlock) k_rs_hist(const uint32_t *keys, const uint32_t *n_dev,
                                                    const uint32_t *gate, const uint32_t *skip,
                                                    int shift, uint32_t *hist) {
  if (gated(gate) || pass_role(skip, shift) != kPassSort) return;
  __shared__ uint32_t lh[256];
  const uint32_t n = *n_dev;
  const uint32_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const uint64_t b0 = (uint64_t)blockIdx.x * chunk;
  const uint64_t b1 = b0 + chunk < n ? b0 + chunk : n;
  lh[threadIdx.x] = 0;
  __syncthreads();
  // kSortItems rows of loads in flight per thread
  for (uint64_t t0 = b0; t0 < b1; t0 += (uint64_t)kSortItems * kBlock) {
    uint32_t k[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
      const uint64_t i = t0 + (uint64_t)r * kBlock + threadIdx.x;
      k[r] = i < b1 ? keys[i] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kSortItems; ++r)
      if (t0 + (uint64_t)r * kBlock + threadIdx.x < b1) atomicAdd(&lh[(k[r] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[threadIdx.x * kChunkBlocks + blockIdx.x] = lh[threadIdx.x];
}

__global__ void __launch_bounds__(kChunkBlocks) k_rs_hscan(uint32_t *hist, const uint32_t *gate,
                                                           const uint32_t *skip, int shift,
                                                           uint32_t *tot, uint32_t nblk) {
  if (gated(gate) || pass_role(skip, shift) != kPassSort) return;
  __shared__ uint32_t lds[kChunkBlocks / kWave + 1];
  uint32_t *h = hist + blockIdx.x * kChunkBlocks;
  uint32_t total;
  const bool mine = threadIdx.x < nblk;  // histograms of the grid's blocks only
  uint32_t ex = block_excl_scan<uint32_t, kChunkBlocks>(mine ? h[threadIdx.x] : 0u, lds, &total);
  if (mine) h[threadIdx.x] = ex;
  if (threadIdx.x == 0) tot[blockIdx.x] = total;
}

template <bool CARRY>
__global__ void __launch_bounds__(kBlock) k_rs_scatter(const uint32_t *__restrict__ kin,
                                                       const uint32_t *__restrict__ vin,
                                                       uint32_t *__restrict__ kout,
                                                       uint32_t *__restrict__ vout,
                                                       const uint32_t *n_dev, const uint32_t *gate,
                                                       const uint32_t *skip, int shift,
                                                       const uint32_t *hist, const uint32_t *tot,
                                                       const float2 *__restrict__ cin,
                                                       float2 *__restrict__ cout) {
  if (gated(gate)) return;
  const int role = pass_role(skip, shift);
  if (role == kPassNone) return;
  // per (row, wave, digit) counts, then their running offsets (at most a
  // tile, 2,048): 16 bits each, so that four blocks fit a CU's LDS; once
  // the tile's places are known the same memory stages the carried float2s
  constexpr int kCnt = kSortItems * kWavesPerBlock * 256;
  static_assert(kSortTile <= 65535, "tile offsets fit 16 bits");
  static_assert(kCnt * sizeof(uint16_t) >= kSortTile * sizeof(float2), "carry fits the counts");
  __shared__ __align__(16) uint16_t cnt[kCnt];
  float2 *sc = reinterpret_cast<float2 *>(cnt);
  __shared__ uint32_t sk[kSortTile];
  __shared__ uint32_t sv[kSortTile];
  __shared__ uint32_t goff[256], tbase[256], tcnt[256];
  __shared__ uint32_t lds[kWavesPerBlock + 1];

  const uint32_t n = *n_dev;
  const uint32_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const uint64_t b0 = (uint64_t)blockIdx.x * chunk;
  const uint64_t b1 = b0 + chunk < n ? b0 + chunk : n;
  if (b0 >= b1) return;  // uniform per block: no barrier is skipped by part of it
  if (role == kPassCopy) {
    for (uint64_t i = b0 + threadIdx.x; i < b1; i += kBlock) {
      kout[i] = kin[i];
      vout[i] = vin ? vin[i] : (uint32_t)i;
      if (CARRY) cout[i] = cin[i];
    }
    return;
  }
  const int tid = threadIdx.x, w = tid / kWave;
  {
    uint32_t total;
    uint32_t base = block_excl_scan<uint32_t, kBlock>(tot[tid], lds, &total);
    goff[tid] = base + hist[tid * kChunkBlocks + blockIdx.x];
  }
  __syncthreads();
  // without a carried payload, a tile's inputs are loaded while the
  // previous tile is placed and stored, so that waiting for them does not
  // also wait for those stores (with one, the registers for it would cost
  // half the waves)
  constexpr bool kAhead = !CARRY;
  uint32_t nkey[kSortItems], nval[kSortItems];
  float2 ncar[kSortItems];
  auto load_tile = [&](uint64_t t0) {
    const uint32_t tn = (uint32_t)((b1 - t0) < (uint64_t)kSortTile ? (b1 - t0) : kSortTile);
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
      const uint32_t li = r * kBlock + tid;
      const bool valid = li < tn;
      nkey[r] = valid ? kin[t0 + li] : 0u;
      nval[r] = !valid ? 0u : vin ? vin[t0 + li] : (uint32_t)(t0 + li);
      if (CARRY) ncar[r] = valid ? cin[t0 + li] : make_float2(0.f, 0.f);
    }
  };
  if (kAhead) load_tile(b0);
  for (uint64_t t0 = b0; t0 < b1; t0 += kSortTile) {
    const uint32_t tile_n = (uint32_t)((b1 - t0) < (uint64_t)kSortTile ? (b1 - t0) : kSortTile);
    for (int i = tid; i < kCnt; i += kBlock) cnt[i] = 0;
    __syncthreads();
    uint32_t key[kSortItems], val[kSortItems], dig[kSortItems], rank[kSortItems];
    float2 car[kSortItems];
    if (!kAhead) load_tile(t0);
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
      key[r] = nkey[r];
      val[r] = nval[r];
      if (CARRY) car[r] = ncar[r];
    }
    if (kAhead && t0 + kSortTile < b1) load_tile(t0 + kSortTile);
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
      const uint32_t li = r * kBlock + tid;
      const bool valid = li < tile_n;
      dig[r] = (key[r] >> shift) & 255u;
      uint64_t m = ballot(valid);
#pragma unroll
      for (int bit = 0; bit < 8; ++bit) {
        const bool b = (dig[r] >> bit) & 1u;
        const uint64_t bb = ballot(b);
        m &= b ? bb : ~bb;
      }
      rank[r] = mbcnt(m);
      if (valid && rank[r] == 0)
        cnt[(r * kWavesPerBlock + w) * 256 + dig[r]] = (uint16_t)__popcll(m);
    }
    __syncthreads();
    // thread d: exclusive running count of digit d over (sub-tile, wave)
    uint32_t run = 0;
#pragma unroll
    for (int rw = 0; rw < kSortItems * kWavesPerBlock; ++rw) {
      const uint32_t c = cnt[rw * 256 + tid];
      cnt[rw * 256 + tid] = (uint16_t)run;
      run += c;
    }
    {
      uint32_t total;
      uint32_t base = block_excl_scan<uint32_t, kBlock>(run, lds, &total);
      tbase[tid] = base;
      tcnt[tid] = run;
    }
    __syncthreads();
    uint32_t pos[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r)
      pos[r] = tbase[dig[r]] + cnt[(r * kWavesPerBlock + w) * 256 + dig[r]] + rank[r];
    if (CARRY) __syncthreads();  // every count is read before the carry overwrites them
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
      if (r * kBlock + tid < tile_n) {
        sk[pos[r]] = key[r];
        sv[pos[r]] = val[r];
        if (CARRY) sc[pos[r]] = car[r];
      }
    }
    __syncthreads();
    // every item's destination first, then the stores
    uint32_t gdst[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
      const uint32_t i = r * kBlock + tid;
      const bool valid = i < tile_n;
      key[r] = valid ? sk[i] : 0u;
      val[r] = valid ? sv[i] : 0u;
      if (CARRY) car[r] = valid ? sc[i] : make_float2(0.f, 0.f);
      const uint32_t d = (key[r] >> shift) & 255u;
      gdst[r] = valid ? goff[d] + (i - tbase[d]) : 0u;
    }
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
      if (r * kBlock + tid < tile_n) {
        kout[gdst[r]] = key[r];
        vout[gdst[r]] = val[r];
        if (CARRY) cout[gdst[r]] = car[r];
      }
    }
    __syncthreads();
    goff[tid] += tcnt[tid];
    __syncthreads();
  }
}

bool radix_sort_pairs(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1,
                      const uint32_t *n_dev, uint64_t n_cap, const uint32_t *gate,
                      uint32_t *hist, uint32_t *tot, int bit_begin, int bit_end, hipStream_t s,
                      float2 *c0, float2 *c1, const uint32_t *skip, bool iota) {
  // about one tile per block when the count reaches its bound
  uint64_t g = (n_cap + kSortTile - 1) / kSortTile;
  const unsigned nblk = (unsigned)(g < 1 ? 1 : (g > kChunkBlocks ? kChunkBlocks : g));
  uint32_t *ki = k0, *vi = v0, *ko = k1, *vo = v1;
  float2 *ci = c0, *co = c1;
  bool in_alt = false;
  for (int shift = bit_begin; shift < bit_end; shift += 8) {
    hipLaunchKernelGGL(k_rs_hist, dim3(nblk), dim3(kBlock), 0, s, (const uint32_t *)ki,
                       n_dev, gate, skip, shift, hist);
    hipLaunchKernelGGL(k_rs_hscan, dim3(256), dim3(kChunkBlocks), 0, s, hist, gate, skip, shift,
                       tot, nblk);
    // the first pass makes the values when they are the input positions
    const uint32_t *vr = iota && shift == bit_begin ? nullptr : vi;
    if (ci)
      hipLaunchKernelGGL(k_rs_scatter<true>, dim3(nblk), dim3(kBlock), 0, s,
                         (const uint32_t *)ki, vr, ko, vo, n_dev, gate, skip, shift,
                         (const uint32_t *)hist, (const uint32_t *)tot, (const float2 *)ci, co);
    else
      hipLaunchKernelGGL(k_rs_scatter<false>, dim3(nblk), dim3(kBlock), 0, s,
                         (const uint32_t *)ki, vr, ko, vo, n_dev, gate, skip, shift,
                         (const uint32_t *)hist, (const uint32_t *)tot,
                         (const float2 *)nullptr, (float2 *)nullptr);
    std::swap(ki, ko);
    std::swap(vi, vo);
    std::swap(ci, co);
    in_alt = !in_alt;
  }
  // with a key width the writing passes are even in number: back in k0
  return skip ? false : in_alt;
}

}  // namespace sj
