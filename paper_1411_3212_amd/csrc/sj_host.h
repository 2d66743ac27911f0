// Host-side launch helpers shared by the translation units of libsj.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sj_device.h"

namespace sj {

ScanJob job_u32(const uint32_t *in, uint32_t *out, const uint32_t *n_dev, uint32_t n_host,
                const uint32_t *in2 = nullptr);
ScanJob job_u64(const uint32_t *in, uint64_t *out, const uint32_t *n_dev, uint32_t n_host);

// Exclusive scans of up to kMaxScanJobs arrays (out[n] = total).  The full
// form runs reduce, a generic single-block top and down; callers with extra
// per-tick bookkeeping launch their own top kernel between mscan_reduce and
// mscan_down (the top must call scan_partials on part[q * kChunkBlocks]).
// part: kMaxScanJobs * kChunkBlocks u64.  Skipped when *gate == 0.
void mscan(const ScanJobs &jobs, int njobs, uint64_t *part, const uint32_t *gate,
           uint64_t *total0, hipStream_t s);
void mscan_reduce(const ScanJobs &jobs, int njobs, uint64_t *part, const uint32_t *gate,
                  hipStream_t s);
void mscan_down(const ScanJobs &jobs, int njobs, const uint64_t *part, const uint32_t *gate,
                hipStream_t s);

// Stable LSD radix sort of n = *n_dev <= n_cap (key, value) pairs over key bits
// [bit_begin, bit_end) in steps of 8.  Passes alternate between (k0, v0)
// and (k1, v1); returns true if the result is in (k1, v1).  If c0 and c1
// are set, a float2 per pair travels with it, between c0 and c1 like the
// values.  skip (device, optional; then bit_end - bit_begin = 32): the keys
// fit in *skip bits, the passes above have nothing to sort and the result
// is in (k0, v0).  iota: the values are the pairs' input positions (v0 is
// not read, only written).  hist: 256 * kChunkBlocks u32, tot: 256 u32.
// Skipped when *gate == 0.
bool radix_sort_pairs(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1,
                      const uint32_t *n_dev, uint64_t n_cap, const uint32_t *gate,
                      uint32_t *hist, uint32_t *tot, int bit_begin, int bit_end, hipStream_t s,
                      float2 *c0 = nullptr, float2 *c1 = nullptr,
                      const uint32_t *skip = nullptr, bool iota = false);

inline unsigned grid_for(uint64_t n, unsigned cap = 2048) {
  uint64_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  return (unsigned)(g < cap ? g : cap);
}

}  // namespace sj
