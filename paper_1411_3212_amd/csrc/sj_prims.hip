// Data-parallel primitives of libsj: chunked exclusive scans and a stable
// LDS-staged LSD radix sort of (u32 key, u32 value) pairs.
//
// All kernels take their element count from device memory (or from a host
// value when the device pointer is null) and an optional gate word: when the
// gate reads 0 the kernel returns at once.  The grids are fixed, so a
// sequence of launches does not depend on sizes produced on the device.
#include "sj_device.h"
#include "sj_host.h"

namespace sj {

__device__ __forceinline__ bool gated(const uint32_t *gate) { return gate && *gate == 0u; }
__device__ __forceinline__ uint32_t count_of(const uint32_t *n_dev, uint32_t n_host) {
  return n_dev ? *n_dev : n_host;
}

// ---------------------------------------------------------------- scans --
// Exclusive scan of a u32 array, result type T; out[n] = total.  Block b of
// kChunkBlocks owns the contiguous chunk [b*chunk, (b+1)*chunk).

__global__ void __launch_bounds__(kBlock) k_scan_reduce(const uint32_t *in, const uint32_t *n_dev,
                                                        uint32_t n_host, const uint32_t *gate,
                                                        uint64_t *part) {
  if (gated(gate)) return;
  __shared__ uint64_t lds[kWavesPerBlock];
  const uint32_t n = count_of(n_dev, n_host);
  const uint32_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const uint64_t b0 = (uint64_t)blockIdx.x * chunk;
  const uint64_t b1 = b0 + chunk < n ? b0 + chunk : n;
  uint64_t s = 0;
  for (uint64_t i = b0 + threadIdx.x; i < b1; i += kBlock) s += in[i];
  s = wave_sum(s);
  if (lane_id() == 0) lds[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
    for (int w = 0; w < kWavesPerBlock; ++w) t += lds[w];
    part[blockIdx.x] = t;
  }
}

template <typename T>
__global__ void __launch_bounds__(kChunkBlocks) k_scan_top(uint64_t *part, T *out,
                                                           const uint32_t *n_dev, uint32_t n_host,
                                                           const uint32_t *gate,
                                                           uint64_t *total_out) {
  if (gated(gate)) return;
  __shared__ uint64_t lds[kChunkBlocks / kWave + 1];
  uint64_t total;
  uint64_t v = part[threadIdx.x];
  uint64_t ex = block_excl_scan<uint64_t, kChunkBlocks>(v, lds, &total);
  part[threadIdx.x] = ex;
  if (threadIdx.x == 0) {
    out[count_of(n_dev, n_host)] = (T)total;
    if (total_out) *total_out = total;
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_scan_down(const uint32_t *in, T *out,
                                                      const uint32_t *n_dev, uint32_t n_host,
                                                      const uint32_t *gate, const uint64_t *part) {
  if (gated(gate)) return;
  __shared__ uint64_t lds[kWavesPerBlock + 1];
  const uint32_t n = count_of(n_dev, n_host);
  const uint32_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const uint64_t b0 = (uint64_t)blockIdx.x * chunk;
  const uint64_t b1 = b0 + chunk < n ? b0 + chunk : n;
  uint64_t run = part[blockIdx.x];
  for (uint64_t t0 = b0; t0 < b1; t0 += kBlock) {
    const uint64_t i = t0 + threadIdx.x;
    uint64_t v = i < b1 ? in[i] : 0;
    uint64_t tot;
    uint64_t ex = block_excl_scan<uint64_t, kBlock>(v, lds, &tot);
    if (i < b1) out[i] = (T)(run + ex);
    run += tot;
  }
}

template <typename T>
void scan_excl(const uint32_t *in, T *out, const uint32_t *n_dev, uint32_t n_host,
               uint64_t *part, uint64_t *total_out, const uint32_t *gate, hipStream_t s) {
  hipLaunchKernelGGL(k_scan_reduce, dim3(kChunkBlocks), dim3(kBlock), 0, s, in, n_dev, n_host,
                     gate, part);
  hipLaunchKernelGGL(k_scan_top<T>, dim3(1), dim3(kChunkBlocks), 0, s, part, out, n_dev, n_host,
                     gate, total_out);
  hipLaunchKernelGGL(k_scan_down<T>, dim3(kChunkBlocks), dim3(kBlock), 0, s, in, out, n_dev,
                     n_host, gate, (const uint64_t *)part);
}

template void scan_excl<uint32_t>(const uint32_t *, uint32_t *, const uint32_t *, uint32_t,
                                  uint64_t *, uint64_t *, const uint32_t *, hipStream_t);
template void scan_excl<uint64_t>(const uint32_t *, uint64_t *, const uint32_t *, uint32_t,
                                  uint64_t *, uint64_t *, const uint32_t *, hipStream_t);

// ----------------------------------------------------------- radix sort --
// One pass sorts by the 8-bit digit (key >> shift) & 255, stably:
//  hist:    per-block digit histograms, digit-major hist[d * B + b];
//  hscan:   exclusive scan over blocks of every digit, digit totals tot[d];
//  scatter: every block ranks its keys tile by tile (wave ballots give the
//           rank among equal digits of a wave), places the tile in LDS in
//           digit order and writes each digit's run contiguously to its
//           global offset.

__global__ void __launch_bounds__(kBlock) k_rs_hist(const uint32_t *keys, const uint32_t *n_dev,
                                                    const uint32_t *gate, int shift,
                                                    uint32_t *hist) {
  if (gated(gate)) return;
  __shared__ uint32_t lh[256];
  const uint32_t n = *n_dev;
  const uint32_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const uint64_t b0 = (uint64_t)blockIdx.x * chunk;
  const uint64_t b1 = b0 + chunk < n ? b0 + chunk : n;
  lh[threadIdx.x] = 0;
  __syncthreads();
  for (uint64_t i = b0 + threadIdx.x; i < b1; i += kBlock) atomicAdd(&lh[(keys[i] >> shift) & 255u], 1u);
  __syncthreads();
  hist[threadIdx.x * kChunkBlocks + blockIdx.x] = lh[threadIdx.x];
}

__global__ void __launch_bounds__(kChunkBlocks) k_rs_hscan(uint32_t *hist, const uint32_t *gate,
                                                           uint32_t *tot) {
  if (gated(gate)) return;
  __shared__ uint32_t lds[kChunkBlocks / kWave + 1];
  uint32_t *h = hist + blockIdx.x * kChunkBlocks;
  uint32_t total;
  uint32_t ex = block_excl_scan<uint32_t, kChunkBlocks>(h[threadIdx.x], lds, &total);
  h[threadIdx.x] = ex;
  if (threadIdx.x == 0) tot[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kBlock) k_rs_scatter(const uint32_t *__restrict__ kin,
                                                       const uint32_t *__restrict__ vin,
                                                       uint32_t *__restrict__ kout,
                                                       uint32_t *__restrict__ vout,
                                                       const uint32_t *n_dev, const uint32_t *gate,
                                                       int shift, const uint32_t *hist,
                                                       const uint32_t *tot) {
  if (gated(gate)) return;
  __shared__ uint32_t cnt[kSortItems * kWavesPerBlock * 256];
  __shared__ uint32_t sk[kSortTile];
  __shared__ uint32_t sv[kSortTile];
  __shared__ uint32_t goff[256], tbase[256], tcnt[256];
  __shared__ uint32_t lds[kWavesPerBlock + 1];

  const uint32_t n = *n_dev;
  const uint32_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const uint64_t b0 = (uint64_t)blockIdx.x * chunk;
  const uint64_t b1 = b0 + chunk < n ? b0 + chunk : n;
  const int tid = threadIdx.x, w = tid / kWave;
  {
    uint32_t total;
    uint32_t base = block_excl_scan<uint32_t, kBlock>(tot[tid], lds, &total);
    goff[tid] = base + hist[tid * kChunkBlocks + blockIdx.x];
  }
  __syncthreads();
  for (uint64_t t0 = b0; t0 < b1; t0 += kSortTile) {
    const uint32_t tile_n = (uint32_t)((b1 - t0) < (uint64_t)kSortTile ? (b1 - t0) : kSortTile);
    for (int i = tid; i < kSortItems * kWavesPerBlock * 256; i += kBlock) cnt[i] = 0;
    __syncthreads();
    uint32_t key[kSortItems], val[kSortItems], dig[kSortItems], rank[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
      const uint32_t li = r * kBlock + tid;
      const bool valid = li < tile_n;
      key[r] = valid ? kin[t0 + li] : 0u;
      val[r] = valid ? vin[t0 + li] : 0u;
      dig[r] = (key[r] >> shift) & 255u;
      uint64_t m = ballot(valid);
#pragma unroll
      for (int bit = 0; bit < 8; ++bit) {
        const bool b = (dig[r] >> bit) & 1u;
        const uint64_t bb = ballot(b);
        m &= b ? bb : ~bb;
      }
      rank[r] = mbcnt(m);
      if (valid && rank[r] == 0) cnt[(r * kWavesPerBlock + w) * 256 + dig[r]] = (uint32_t)__popcll(m);
    }
    __syncthreads();
    // thread d: exclusive running count of digit d over (sub-tile, wave)
    uint32_t run = 0;
#pragma unroll
    for (int rw = 0; rw < kSortItems * kWavesPerBlock; ++rw) {
      uint32_t c = cnt[rw * 256 + tid];
      cnt[rw * 256 + tid] = run;
      run += c;
    }
    {
      uint32_t total;
      uint32_t base = block_excl_scan<uint32_t, kBlock>(run, lds, &total);
      tbase[tid] = base;
      tcnt[tid] = run;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
      const uint32_t li = r * kBlock + tid;
      if (li < tile_n) {
        const uint32_t pos = tbase[dig[r]] + cnt[(r * kWavesPerBlock + w) * 256 + dig[r]] + rank[r];
        sk[pos] = key[r];
        sv[pos] = val[r];
      }
    }
    __syncthreads();
    for (uint32_t i = tid; i < tile_n; i += kBlock) {
      const uint32_t k = sk[i];
      const uint32_t d = (k >> shift) & 255u;
      const uint32_t g = goff[d] + (i - tbase[d]);
      kout[g] = k;
      vout[g] = sv[i];
    }
    __syncthreads();
    goff[tid] += tcnt[tid];
    __syncthreads();
  }
}

void radix_sort_pairs(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1,
                      const uint32_t *n_dev, const uint32_t *gate, uint32_t *hist, uint32_t *tot,
                      int bit_begin, int bit_end, hipStream_t s) {
  uint32_t *ki = k0, *vi = v0, *ko = k1, *vo = v1;
  for (int shift = bit_begin; shift < bit_end; shift += 8) {
    hipLaunchKernelGGL(k_rs_hist, dim3(kChunkBlocks), dim3(kBlock), 0, s, (const uint32_t *)ki,
                       n_dev, gate, shift, hist);
    hipLaunchKernelGGL(k_rs_hscan, dim3(256), dim3(kChunkBlocks), 0, s, hist, gate, tot);
    hipLaunchKernelGGL(k_rs_scatter, dim3(kChunkBlocks), dim3(kBlock), 0, s,
                       (const uint32_t *)ki, (const uint32_t *)vi, ko, vo, n_dev, gate, shift,
                       (const uint32_t *)hist, (const uint32_t *)tot);
    uint32_t *t = ki;
    ki = ko;
    ko = t;
    t = vi;
    vi = vo;
    vo = t;
  }
}

}  // namespace sj
