// Device-side definitions shared by the kernels of libsj (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sj {

constexpr int kWave = 64;
constexpr int kBlock = 256;               // threads per block of most kernels
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kChunkBlocks = 1024;        // blocks of chunked scans / sorts
constexpr int kFine = 16;                 // bits per axis of the finest grid
constexpr uint32_t kLeafBit = 0x80000000u; // child reference: leaf index
constexpr int kSortItems = 8;             // keys per thread per sort tile
constexpr int kSortTile = kBlock * kSortItems;
constexpr uint32_t kTaskSub = 64;         // intersecting subqueries per join task

// Error bits latched on the device.
enum : uint32_t {
  kErrUpdId = 1u << 0,
  kErrUpdCoord = 1u << 1,
  kErrQueryId = 1u << 2,
  kErrQueryRect = 1u << 3,
  kErrOvfSubq = 1u << 4,
  kErrOvfCov = 1u << 5,
  kErrOvfRes = 1u << 6,
  kErrOvfTree = 1u << 7,
};
constexpr uint32_t kErrOverflow = kErrOvfSubq | kErrOvfCov | kErrOvfRes | kErrOvfTree;

// Scene control block in device memory.  Kernels read the per-tick sizes
// from here, so that the launch sequence of a tick does not depend on
// values produced on the device (and can be captured in a graph).
struct Ctl {
  // index frame: square of side 2^e anchored at (x0, y0)
  float x0, y0;
  int32_t e;
  float scale;            // 2^(16 - e)
  uint32_t built;
  uint32_t th_cur;        // threshold of the current quadtree
  uint32_t th_next;       // threshold requested for the next build (0: keep)
  uint32_t force;         // build requested by the host
  uint32_t rebuild;       // the current tick builds the quadtree
  uint32_t sort_skip;     // radix passes from this shift on only copy (keys are below 2^it)
  uint32_t want_rebuild;  // automatic policy: build on the next tick
  uint32_t since_build;   // ticks since the last build
  uint32_t tick;
  uint32_t n_present;
  uint32_t n_outside;     // present objects outside the frame
  uint32_t n_leaves, l_deep, tlev;
  uint32_t fcount[kFine + 2];  // frontier sizes per level of the build
  uint32_t n_tasks;       // leaves with join work
  uint32_t n_entries;     // join tasks: one per leaf + one per further kTaskSub subqueries
  uint32_t n_run;         // join tasks with work, in run order in the task records
  uint32_t n_qord;        // queries put in spatial order
  uint32_t exp_bad;       // an expansion selected a query index >= nq
  uint32_t ug_split;      // uniform-grid index: columns (and rows) of the frame; 0: quadtree
  uint32_t ug_bits;       // bits per axis of the grid cells' Morton codes
  uint32_t sq_skip;       // radix digits of the subqueries' leaf keys (multiple of 8)
  uint32_t max_leaf;
  uint32_t n_knn_fb;      // kNN queries of the tick listed for the fallback scan
  uint32_t err_upd;       // errors of updates since the last tick
  uint32_t err;           // errors of the current tick (includes err_upd)
  uint32_t go_split;      // subquery/covering capacities respected
  uint32_t go_join;       // result capacity respected
  uint32_t n32[2];        // intersecting / covering subqueries as u32
  uint64_t n_isect, n_cov, n_res, cov_pairs, tests;
  uint64_t upd_seq, qry_seq;
  // rebuild by cost (SJ_REBUILD_COST): device clock (100 MHz) at the start
  // of the tick; durations of the last build tick and of the fastest kept
  // tick since; the build's extra cost over it (< 0: not known yet); the
  // summed excess of the kept ticks over the fastest one
  uint64_t t_start;
  uint32_t policy;
  float d_build, d_base, b_cost, excess;
  uint32_t pad_cost;
};

// Input arrays of a tick.  Kernels read them from this block in device
// memory, written on the stream just before the tick, so that a captured
// tick does not depend on where its caller keeps its inputs.
struct TickIn {
  const uint32_t *id;  // updates: object ids, positions
  const float *x, *y;
  const uint32_t *qid;  // queries: issuing object, rectangle corners
  const float *xa, *ya, *xb, *yb;
};

// Slots of the per-block partial reductions (red[slot * kChunkBlocks + b]).
enum : int {
  kRedMinX = 0, kRedMinY, kRedMaxX, kRedMaxY, kRedOutside,
  kRedCovPairs, kRedTests, kRedMaxLeaf, kRedTasks, kRedCost, kRedCostMax, kRedSlots
};

__device__ __forceinline__ uint32_t fenc(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float fdec(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

// SplitMix64's output function (the pair-set hash of a result set adds it
// over the pairs (qid << 32) | id).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// Per-CU work counters: the slot of the compute unit running the wave, from
// its hardware id registers (HW_ID: CU, shader array and shader engine;
// XCC_ID: the accelerator complex die).  Distinct CUs get distinct slots
// below kCuSlots.
constexpr uint32_t kCuSlots = 4096;
__device__ __forceinline__ uint32_t cu_slot() {
  const uint32_t hw = __builtin_amdgcn_s_getreg((31 << 11) | 4);    // HW_REG_HW_ID, 32 bits
  const uint32_t xcc = __builtin_amdgcn_s_getreg((31 << 11) | 20);  // HW_REG_XCC_ID, 32 bits
  const uint32_t cu = (hw >> 8) & 0xfu, sh = (hw >> 12) & 1u, se = (hw >> 13) & 7u;
  return ((xcc & 0xfu) << 8) | (se << 5) | (sh << 4) | cu;
}

// Column (or row) of the uniform grid holding finest-level cell `fine`:
// the frame's 2^16 finest cells are cut into s runs of floor or ceil of
// 2^16 / s cells (monotone, exact integer arithmetic).
__device__ __forceinline__ uint32_t ug_col(uint32_t fine, uint32_t s) {
  return (uint32_t)(((uint64_t)fine * s) >> 16);
}

// Finest-level cell index of a coordinate: one binary32 subtraction, an
// exact multiplication by a power of two, truncation, clamping.  Monotone,
// and the same function for objects and query corners.
__device__ __forceinline__ uint32_t cell_of(float v, float v0, float scale) {
  float d = __fsub_rn(v, v0);
  float t = __fmul_rn(d, scale);
  if (!(t >= 0.0f)) return 0u;
  if (t >= 65536.0f) return 65535u;
  return (uint32_t)t;
}

__device__ __forceinline__ uint32_t spread16(uint32_t x) {
  x &= 0xffffu;
  x = (x | (x << 8)) & 0x00ff00ffu;
  x = (x | (x << 4)) & 0x0f0f0f0fu;
  x = (x | (x << 2)) & 0x33333333u;
  x = (x | (x << 1)) & 0x55555555u;
  return x;
}
__device__ __forceinline__ uint32_t morton2(uint32_t i, uint32_t j) {
  return spread16(i) | (spread16(j) << 1);
}

// Inverse of spread16: the even bits of x.
__device__ __forceinline__ uint32_t compact16(uint32_t x) {
  x &= 0x55555555u;
  x = (x | (x >> 1)) & 0x33333333u;
  x = (x | (x >> 2)) & 0x0f0f0f0fu;
  x = (x | (x >> 4)) & 0x00ff00ffu;
  x = (x | (x >> 8)) & 0x0000ffffu;
  return x;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Number of set bits of m below the calling lane, plus acc (the count
// instructions add it for free).
__device__ __forceinline__ uint32_t mbcnt(uint64_t m, uint32_t acc = 0u) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, acc));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int readlane_i(int v, int l) {
  return __builtin_amdgcn_readlane(v, l);
}
__device__ __forceinline__ float readlane_f(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int l) {
  uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    T y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  return x;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}

template <typename T>
__device__ __forceinline__ T wave_max(T x) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    T y = __shfl_xor(x, o, kWave);
    x = y > x ? y : x;
  }
  return x;
}

// Exclusive scan over a block of NT threads; lds must hold NT/64 + 1
// elements.  Returns the exclusive prefix; *total gets the block sum.
template <typename T, int NT>
__device__ __forceinline__ T block_excl_scan(T v, T *lds, T *total) {
  constexpr int NW = NT / kWave;
  const int lane = lane_id(), w = threadIdx.x / kWave;
  T inc = wave_incl_scan(v);
  if (lane == kWave - 1) lds[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    T s = 0;
    for (int i = 0; i < NW; ++i) {
      T t = lds[i];
      lds[i] = s;
      s += t;
    }
    lds[NW] = s;
  }
  __syncthreads();
  T r = inc - v + lds[w];
  *total = lds[NW];
  __syncthreads();
  return r;
}

// Wave-aggregated append: each lane asks for `want` slots of a counter;
// one atomic per wave.  Returns the lane's first slot.
__device__ __forceinline__ uint32_t wave_append(uint32_t *counter, uint32_t want) {
  uint32_t inc = wave_incl_scan(want);
  uint32_t tot = (uint32_t)readlane_i((int)inc, kWave - 1);
  uint32_t base = 0;
  if (lane_id() == 0 && tot) base = atomicAdd(counter, tot);
  base = (uint32_t)readlane_i((int)base, 0);
  return base + inc - want;
}

// Work-groups go to the GPU's XCDs in turn, and each XCD has its own L2.
// A sweep gives XCD x the x-th contiguous eighth of n items and walks it
// with all of that XCD's work-groups together (unit u of `per_block` units
// in a block takes items first, first + stride, ... below end), so items
// processed at the same time are neighbours held by one L2.  The grid must
// be a multiple of kXcds.
constexpr uint32_t kXcds = 8;

struct Sweep {
  uint32_t first, end, stride;
};

__device__ __forceinline__ Sweep xcd_sweep(uint32_t n, uint32_t per_block, uint32_t u) {
  const uint32_t x = blockIdx.x % kXcds, bx = blockIdx.x / kXcds, per_x = gridDim.x / kXcds;
  const uint32_t span = (n + kXcds - 1u) / kXcds;
  const uint64_t lo = (uint64_t)x * span;
  const uint32_t end = (uint32_t)min(lo + span, (uint64_t)n);
  const uint64_t first = lo + (uint64_t)bx * per_block + u;
  return Sweep{(uint32_t)min(first, (uint64_t)end), end, per_x * per_block};
}

__device__ __forceinline__ void flag_error(Ctl *ctl, uint32_t bits, bool cond) {
  uint64_t m = ballot(cond);
  if (m && lane_id() == (uint32_t)(__ffsll((unsigned long long)m) - 1)) atomicOr(&ctl->err, bits);
}

__device__ __forceinline__ uint32_t lower_bound_u32(const uint32_t *a, uint32_t lo, uint32_t hi,
                                                    uint32_t key) {
  while (lo < hi) {
    uint32_t mid = lo + ((hi - lo) >> 1);
    if (a[mid] < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// One array of a multi-array exclusive scan: in[0..n) -> out[0..n], out[n]
// = total; out is u32 or u64.  Up to kMaxScanJobs arrays are scanned by one
// launch of each scan kernel (blockIdx.y selects the array).
constexpr int kMaxScanJobs = 3;
struct ScanJob {
  const uint32_t *in;
  const uint32_t *in2;    // optional second input, added element-wise
  void *out;
  const uint32_t *n_dev;  // element count in device memory, or
  uint32_t n_host;        // this value when n_dev is null
  uint32_t out64;
};
struct ScanJobs {
  ScanJob j[kMaxScanJobs];
};

__device__ __forceinline__ uint32_t job_n(const ScanJob &j) { return j.n_dev ? *j.n_dev : j.n_host; }
__device__ __forceinline__ uint32_t job_in(const ScanJob &j, uint64_t i) {
  return j.in2 ? j.in[i] + j.in2[i] : j.in[i];
}
__device__ __forceinline__ void job_store(const ScanJob &j, uint64_t i, uint64_t v) {
  if (j.out64)
    ((uint64_t *)j.out)[i] = v;
  else
    ((uint32_t *)j.out)[i] = (uint32_t)v;
}

// In a block of kChunkBlocks threads: exclusive scan of the per-block
// partials part[0..kChunkBlocks) in place; returns the total.
__device__ __forceinline__ uint64_t scan_partials(uint64_t *part, uint64_t *lds) {
  uint64_t total;
  const uint64_t v = part[threadIdx.x];
  const uint64_t ex = block_excl_scan<uint64_t, kChunkBlocks>(v, lds, &total);
  part[threadIdx.x] = ex;
  return total;
}

// Fraction of the area of leaf `leaf` (level l, first finest cell st) that
// rectangle r covers, clamped to [0, 1]: the overlap feature of the cost
// model (timing log and threshold tuner).
__device__ __forceinline__ float overlap_frac(const Ctl *ctl, const uint32_t *lstart,
                                              const uint32_t *llevel, uint32_t leaf, float4 r) {
  const uint32_t st = lstart[leaf], l = llevel[leaf];
  const float inv = 1.0f / ctl->scale, size = (float)(1u << (kFine - l)) * inv;
  const float x0 = ctl->x0 + (float)compact16(st) * inv;
  const float y0 = ctl->y0 + (float)compact16(st >> 1) * inv;
  const float w = fminf(r.z, x0 + size) - fmaxf(r.x, x0);
  const float h = fminf(r.w, y0 + size) - fmaxf(r.y, y0);
  return (w > 0.0f && h > 0.0f) ? fminf(1.0f, (w / size) * (h / size)) : 0.0f;
}

// Threshold tuner state (device memory): the installed cost model and the
// outcome of the last tuning.
constexpr int kMaxCand = 8;
struct TuneState {
  uint16_t w[4548];          // BF16 MLP parameters (4545 used)
  float coef[6];             // cost = c0 * sum exp(mlp) + c1 |Q_I| + c2 |Q_C| + c3 leaves
                             //        + c4 * max exp(mlp) + c5 * sort passes * objects
  uint32_t n_cand;
  uint32_t cand[kMaxCand];   // candidate thresholds
  float cost[kMaxCand];      // predicted cost per candidate (inf: infeasible)
  float msum[kMaxCand];      // sum over active leaves of exp(mlp) per candidate
  float mmax[kMaxCand];      // largest exp(mlp) of an active leaf per candidate
  uint32_t err_saved;        // tick errors before the trial builds
  uint32_t th_before;        // threshold before the tuning
  uint32_t chosen, n_tunes, tuned_tick;
};

}  // namespace sj
