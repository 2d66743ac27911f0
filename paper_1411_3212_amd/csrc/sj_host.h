// Host-side launch helpers shared by the translation units of libsj.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sj {

// Exclusive scan of in[0..n) (n = *n_dev, or n_host when n_dev is null)
// into out[0..n]; out[n] and *total_out (if non-null) get the total.
// part: kChunkBlocks u64 of scratch.  Skipped when *gate == 0.
template <typename T>
void scan_excl(const uint32_t *in, T *out, const uint32_t *n_dev, uint32_t n_host,
               uint64_t *part, uint64_t *total_out, const uint32_t *gate, hipStream_t s);

// Stable LSD radix sort of n = *n_dev (key, value) pairs over key bits
// [bit_begin, bit_end) in steps of 8.  Passes alternate between (k0, v0)
// and (k1, v1); with an even number of passes the result is in (k0, v0).
// hist: 256 * kChunkBlocks u32, tot: 256 u32.  Skipped when *gate == 0.
void radix_sort_pairs(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1,
                      const uint32_t *n_dev, const uint32_t *gate, uint32_t *hist, uint32_t *tot,
                      int bit_begin, int bit_end, hipStream_t s);

inline unsigned grid_for(uint64_t n, unsigned cap = 2048) {
  uint64_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  return (unsigned)(g < cap ? g : cap);
}

}  // namespace sj
