// The PR-quadtree as the device traversals see it (shared by the kernels of
// the tick and of the k-nearest-neighbour queries).
#pragma once

#include "sj_device.h"
#include "sj_kernels.h"

namespace sj {

// Start-table entry of a leaf: flag, level - 1 (4 bits), leaf index (27 bits).
constexpr uint32_t kLeafIdxBits = 27;
constexpr uint32_t kLeafIdxMask = (1u << kLeafIdxBits) - 1u;

// The quadtree as the traversals see it: node table (4 child references,
// kLeafBit marks a leaf), start table at level tlev, leaf starts and levels.
struct Tree {
  const uint4 *nodes;
  const uint32_t *table;
  const uint32_t *lstart, *llevel;
  uint32_t tlev;
};

// Leaf containing the finest-level code `code`: its start-table cell gives
// the leaf, or the internal node at level tlev to descend from (one child
// reference per level, at most kFine - tlev of them).
__device__ __forceinline__ uint32_t table_entry(const Tree &tr, uint32_t code) {
  return tr.table[code >> (2u * (kFine - tr.tlev))];
}
// The descent from table entry e (split from the table load so that a
// thread can issue several table loads before it waits for one).
__device__ __forceinline__ uint32_t leaf_from(const Tree &tr, uint32_t e, uint32_t code) {
  if (e & kLeafBit) return e & kLeafIdxMask;
  uint32_t node = e;
  for (uint32_t k = tr.tlev; k < (uint32_t)kFine; ++k) {
    const uint32_t q = (code >> (2u * (kFine - k - 1u))) & 3u;
    const uint4 nd = tr.nodes[node];
    const uint32_t r = q == 0u ? nd.x : q == 1u ? nd.y : q == 2u ? nd.z : nd.w;
    if (r & kLeafBit) return r & ~kLeafBit;
    node = r;
  }
  return 0u;  // not reached: every level-16 cell lies in a leaf
}
__device__ __forceinline__ uint32_t leaf_of(const Tree &tr, uint32_t code) {
  return leaf_from(tr, table_entry(tr, code), code);
}

// The scene's quadtree arrays (tlev is read from the control block by the
// kernels).
inline Tree tree_of(const Bufs &B) {
  return Tree{(const uint4 *)B.nodes, (const uint32_t *)B.table, (const uint32_t *)B.lstart,
              (const uint32_t *)B.llevel, 0u};
}

}  // namespace sj
