// C ABI of libsj (declared in include/sj.h): scene lifecycle, workspace
// layout, and the host side of the tick pipeline.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stddef.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <new>

#include "sj.h"
#include "sj_device.h"
#include "sj_kernels.h"
#include "sj_scene.h"

using sj::Bufs;
using sj::Ctl;

struct GraphSlot {
  hipGraphExec_t exec;   // the whole tick, or its part before the join write pass
  hipGraphExec_t exec2;  // the join write pass, when a profiled tick is two launches
  bool valid;
  bool split;            // exec2 is launched after exec, between the timing events
  uint32_t m, nq, key_bits;
  uint32_t t_lo, t_hi;   // candidates a tuning tick tries
};

struct sj_scene {
  sj_config cfg;
  Bufs B;
  uint8_t *ws;
  size_t ws_bytes;
  hipStream_t stream;
  int device;
  uint32_t th, l_max, period;
  uint32_t last_nq;
  const uint32_t *last_qid;
  bool ticked;
  bool prof;
  bool known;          // host_ctl reflects the device state after the last tick
  bool mirror;         // the last enqueued work ends with a tick's copy of ctl to pin_ctl
  bool events_valid;   // phase events were recorded for the last tick
  bool join_events;    // only the join write pass was timed (graph tick)
  GraphSlot graphs[4]; // captured ticks per decision (keep, build, device, build + tune)
  hipStream_t cap_stream;  // private stream graphs are captured on
  bool force_pending;  // sj_build_index since the last tick
  uint64_t upd_pending;  // updates enqueued since the last tick
  bool upd_open;  // an update event interval is open since the last tick
  hipEvent_t ev[SJ_PH_COUNT + 2];
  hipEvent_t ev_u0, ev_u1;
  Ctl host_ctl;
  Ctl *pin_ctl = nullptr;  // pinned landing buffer of its copies from the device
  bool cm_set;          // a cost model is installed (sj_set_cost_model)
  uint32_t n_cand;      // its candidate thresholds (ascending)
  uint32_t cand[8];
  uint32_t tune_every;  // host-decided builds between two tunings
  uint32_t since_tune;  // host-decided builds since the last tuning
  bool tuned;           // a tuning has been enqueued
  char err[256];
};

static char g_create_err[256] = "";

namespace {

struct Derived {
  uint32_t N, Q, th, th_min, l_max, period, slots, tcap, tune_every, ug, ug_bits;
  bool log, sqb, cu;
  uint64_t S, C, R;
  uint32_t LCAP, NCAP, FCAP;
};

int derive(const sj_config *cfg, Derived *d, char *msg, size_t msz) {
  if (!cfg) {
    snprintf(msg, msz, "null config");
    return SJ_EINVAL;
  }
  d->N = cfg->capacity_objects;
  d->Q = cfg->capacity_queries;
  if (d->N == 0 || d->N > 0x7fffffffu) {
    snprintf(msg, msz, "capacity_objects must be in 1..2^31-1");
    return SJ_EINVAL;
  }
  if (d->Q == 0 || d->Q > 0x7fffffffu) {
    snprintf(msg, msz, "capacity_queries must be in 1..2^31-1");
    return SJ_EINVAL;
  }
  d->S = cfg->capacity_subqueries ? cfg->capacity_subqueries : 32ull * d->Q;
  d->C = cfg->capacity_covering ? cfg->capacity_covering : 32ull * d->Q;
  d->R = cfg->capacity_results ? cfg->capacity_results : 256ull * d->Q;
  if (d->S >= 0xffffffffull || d->C >= 0xffffffffull) {
    snprintf(msg, msz, "subquery and covering capacities must be below 2^32-1");
    return SJ_EINVAL;
  }
  d->th = cfg->th_quad ? cfg->th_quad : 64u;
  d->th_min = cfg->th_min ? cfg->th_min : d->th;
  if (d->th_min > d->th) {
    snprintf(msg, msz, "th_min must not exceed th_quad");
    return SJ_EINVAL;
  }
  d->l_max = cfg->l_max ? cfg->l_max : 16u;
  if (d->l_max > 16u) {
    snprintf(msg, msz, "l_max must be in 1..16");
    return SJ_EINVAL;
  }
  d->period = cfg->rebuild_period ? cfg->rebuild_period : 32u;
  d->slots = cfg->split_slots ? cfg->split_slots : 32u;
  d->log = (cfg->flags & SJ_TIMING_LOG) != 0;
  d->sqb = (cfg->flags & SJ_ATOMIC_RESULTS) != 0;
  d->cu = (cfg->flags & SJ_CU_COUNTERS) != 0;
  d->tune_every = cfg->tune_every ? cfg->tune_every : 8u;
  if (d->slots > 4096u) {
    snprintf(msg, msz, "split_slots must be at most 4096");
    return SJ_EINVAL;
  }
  if (cfg->rebuild_policy > SJ_REBUILD_COST) {
    snprintf(msg, msz, "unknown rebuild policy");
    return SJ_EINVAL;
  }
  d->ug = 0;
  d->ug_bits = 0;
  if (cfg->flags & SJ_UNIFORM_GRID) {
    if (cfg->grid_split < 1u || cfg->grid_split > 4096u) {
      snprintf(msg, msz, "grid_split must be in 1..4096");
      return SJ_EINVAL;
    }
    if (cfg->flags & (SJ_THRESH_MLP | SJ_SCHEDULE_MLP | SJ_TIMING_LOG)) {
      snprintf(msg, msz, "the uniform grid takes no cost model and no timing log");
      return SJ_EINVAL;
    }
    d->ug = cfg->grid_split;
    while ((1u << d->ug_bits) < d->ug) ++d->ug_bits;
  }
  // Split nodes at level l are disjoint and hold more than th_min objects
  // each, and there are at most 4^l of them: bound the tree by that.
  const uint64_t per = (uint64_t)d->N / ((uint64_t)d->th_min + 1u);
  uint64_t splits = 1, fmax = 1, p4 = 1;
  for (uint32_t l = 1; l < d->l_max; ++l) {
    p4 *= 4u;
    const uint64_t c = p4 < per ? p4 : per;
    splits += c;
    if (c > fmax) fmax = c;
  }
  const uint64_t leaves = 3u * splits + 1u;
  if (leaves >= (1ull << 27)) {
    snprintf(msg, msz, "quadtree bound above 2^27 leaves: raise th_min");
    return SJ_EINVAL;
  }
  // Start-table level cap: about four levels below the depth of a uniform
  // tree with th_min objects per leaf, within [4, 12] and l_max.
  uint32_t lu = 0;
  for (uint64_t c = 1; c < per; c *= 4u) ++lu;
  d->tcap = lu + 4u < 4u ? 4u : (lu + 4u > 12u ? 12u : lu + 4u);
  if (d->tcap > d->l_max) d->tcap = d->l_max;
  d->LCAP = (uint32_t)leaves;
  if (d->ug && (1u << (2u * d->ug_bits)) > d->LCAP) d->LCAP = 1u << (2u * d->ug_bits);
  d->NCAP = (uint32_t)splits;
  d->FCAP = (uint32_t)fmax;
  return SJ_OK;
}

struct Carver {
  uint8_t *base;
  size_t off = 0;
  template <typename T>
  T *take(uint64_t count) {
    off = (off + 255u) & ~(size_t)255u;
    T *p = base ? (T *)(base + off) : nullptr;
    off += (size_t)count * sizeof(T);
    return p;
  }
};

size_t carve(const Derived &d, uint8_t *base, Bufs *B) {
  Carver c{base};
  Bufs b{};
  const uint64_t N = d.N, Q = d.Q, L = d.LCAP;
  b.ctl = c.take<Ctl>(1);
  b.tin = c.take<sj::TickIn>(1);
  b.pos = c.take<float2>(N);
  b.ustamp = c.take<uint64_t>(N);
  b.qstamp = c.take<uint64_t>(N);
  b.keyA = c.take<uint32_t>(N);
  b.valA = c.take<uint32_t>(N);
  b.keyB = c.take<uint32_t>(N);
  b.valB = c.take<uint32_t>(N);
  b.sxy = c.take<float2>(N);
  b.sxy2 = c.take<float2>(N);
  b.blk = c.take<uint32_t>(sj::kChunkBlocks);
  b.red = c.take<uint64_t>((uint64_t)sj::kRedSlots * sj::kChunkBlocks);
  b.part = c.take<uint64_t>((uint64_t)sj::kMaxScanJobs * sj::kChunkBlocks);
  b.hist = c.take<uint32_t>(256u * sj::kChunkBlocks);
  b.tot = c.take<uint32_t>(256);
  b.front[0] = c.take<uint4>(d.FCAP);
  b.front[1] = c.take<uint4>(d.FCAP);
  b.lstart = c.take<uint32_t>(L);
  b.llevel = c.take<uint32_t>(L);
  b.lstart2 = c.take<uint32_t>(L);
  b.llevel2 = c.take<uint32_t>(L);
  b.nopen = c.take<uint32_t>(L);
  b.node_off = c.take<uint32_t>(L + 1);
  b.nodes = c.take<uint4>(d.NCAP);
  b.table = c.take<uint32_t>(1ull << (2 * d.tcap));
  b.leaf_beg = c.take<uint32_t>(L + 1);
  b.leaf_sqoff = c.take<uint32_t>(L + 1);
  // join tasks: one per leaf and one per further kTaskSub subqueries of a leaf
  const uint64_t T = (uint64_t)L + d.S / sj::kTaskSub + 1u;
  b.tkey = c.take<uint32_t>(T);
  b.tkhist = c.take<uint32_t>(512);
  b.qkey = c.take<uint32_t>(Q);
  b.qord = c.take<uint32_t>(Q);
  b.qkey2 = c.take<uint32_t>(Q);
  b.qord2 = c.take<uint32_t>(Q);
  b.vtask = c.take<uint2>(T - L);
  b.xbase = c.take<uint32_t>(L);
  b.trec = c.take<uint4>(T);
  b.tleaf = c.take<uint32_t>(T);
  b.TCAP = (uint32_t)T;
  b.qrect = c.take<float4>(Q);
  b.q_ni = c.take<uint32_t>(Q);
  b.q_nc = c.take<uint32_t>(Q);
  b.q_ioff = c.take<uint32_t>(Q + 1);
  b.q_coff = c.take<uint32_t>(Q + 1);
  b.qpos = c.take<uint32_t>(Q);
  b.qlist = c.take<uint32_t>(Q * d.slots);
  b.sq = c.take<uint32_t>(d.S);
  b.slot_sq = c.take<uint32_t>(d.S);
  b.sq_cnt = c.take<uint32_t>(d.S);
  b.res_off = c.take<uint64_t>(d.S + 1);
  b.cov_leaf = c.take<uint32_t>(d.C);
  b.res_ids = c.take<uint32_t>(d.R);
  b.tlog = d.log ? c.take<float>((uint64_t)L * 8) : nullptr;
  b.pairs = d.sqb ? c.take<uint2>(d.R) : nullptr;
  b.cu_tests = d.cu ? c.take<uint64_t>(sj::kCuSlots) : nullptr;
  b.tune = c.take<sj::TuneState>(1);
  b.kq_rect = c.take<float>(4 * Q);
  b.kq_fb = c.take<uint32_t>(Q);
  b.N = d.N;
  b.Q = d.Q;
  b.LCAP = d.LCAP;
  b.NCAP = d.NCAP;
  b.FCAP = d.FCAP;
  b.slots = d.slots;
  b.tcap = d.tcap;
  b.S = d.S;
  b.C = d.C;
  b.R = d.R;
  if (B) *B = b;
  return (c.off + 255u) & ~(size_t)255u;
}

int fail(sj_scene *s, int code, const char *what) {
  if (s) snprintf(s->err, sizeof s->err, "%s", what);
  return code;
}

int hip_fail(sj_scene *s, hipError_t e, const char *where) {
  char buf[256];
  snprintf(buf, sizeof buf, "%s: %s", where, hipGetErrorString(e));
  return fail(s, SJ_EDEVICE, buf);
}

int status_of(sj_scene *s, uint32_t bits) {
  if (bits & sj::kErrOverflow) {
    char buf[256];
    snprintf(buf, sizeof buf, "capacity exceeded (flags 0x%x): subqueries %llu covering %llu "
             "result ids %llu", bits, (unsigned long long)s->host_ctl.n_isect,
             (unsigned long long)s->host_ctl.n_cov, (unsigned long long)s->host_ctl.n_res);
    return fail(s, SJ_EOVERFLOW, buf);
  }
  if (bits & (sj::kErrUpdId | sj::kErrQueryId))
    return fail(s, SJ_EINVAL, "object id >= capacity_objects in an update or a query");
  if (bits & (sj::kErrUpdCoord | sj::kErrQueryRect))
    return fail(s, SJ_EDATA, "non-finite coordinate or inverted query rectangle (ignored)");
  return SJ_OK;
}

int sync_ctl(sj_scene *s) {
  hipError_t e = hipSuccess;
  if (!s->mirror) {
    e = hipMemcpyAsync(s->pin_ctl, s->B.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "hipMemcpyAsync");
  }
  e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "hipStreamSynchronize");
  s->host_ctl = *s->pin_ctl;
  s->known = true;
  return SJ_OK;
}

int check_tick_args(sj_scene *s, const uint32_t *d_qid, const float *d_xa, const float *d_ya,
                    const float *d_xb, const float *d_yb, uint32_t nq) {
  if (nq > s->B.Q) return fail(s, SJ_EINVAL, "run_tick: nq above capacity_queries");
  if (nq && (!d_qid || !d_xa || !d_ya || !d_xb || !d_yb || ((uintptr_t)d_qid & 3u) ||
             ((uintptr_t)d_xa & 3u) || ((uintptr_t)d_ya & 3u) || ((uintptr_t)d_xb & 3u) ||
             ((uintptr_t)d_yb & 3u)))
    return fail(s, SJ_EINVAL, "run_tick: null or misaligned pointer");
  return SJ_OK;
}

// Rebuild decision: when the host has seen the device state after the last
// tick it decides (and launches the build kernels only if needed);
// otherwise the device decides and the build kernels are launched gated.
uint32_t host_decision(const sj_scene *s) {
  if (s->cfg.flags & SJ_UNIFORM_GRID) return 1u;  // the grid is materialised every tick
  if (!s->known) return 2u;
  const Ctl &c = s->host_ctl;
  const uint32_t policy = s->cfg.rebuild_policy;
  const bool r = s->force_pending || !c.built || policy == SJ_REBUILD_ALWAYS ||
                 ((policy == SJ_REBUILD_AUTO || policy == SJ_REBUILD_COST) && c.want_rebuild);
  return r ? 1u : 0u;
}

// Width of the leaf keys of a tick that keeps the quadtree, when the host
// has read the scene's state (0: the device decides).
uint32_t key_bits(const sj_scene *s, uint32_t decision) {
  if (decision != 0u || !s->known) return 0u;
  const uint32_t nl = s->host_ctl.n_leaves;
  uint32_t bits = 0;
  while (bits < 32u && (nl - 1u) >> bits) ++bits;
  return bits < 8u ? 8u : bits;
}

// Whether a tick with this rebuild decision tunes the threshold first: the
// first build decided on the host and every tune_every-th after it.
bool want_tune(const sj_scene *s, uint32_t decision) {
  return s->cm_set && (s->cfg.flags & SJ_THRESH_MLP) && decision == 1u &&
         (!s->tuned || s->since_tune + 1u >= s->tune_every);
}

// Candidates [lo, hi) a tuning build tries: all of them the first time;
// afterwards those within a factor of two of the current threshold (the
// best threshold moves with the distribution, which drifts between two
// tunings; the small thresholds, whose trial splits cost the most, are
// tried again only when the choice comes close to them).
void tune_window(const sj_scene *s, uint32_t *lo, uint32_t *hi) {
  *lo = 0;
  *hi = s->n_cand;
  if (!s->tuned) return;
  const uint64_t th = s->host_ctl.th_cur;
  uint32_t a = 0, b = s->n_cand;
  while (a < s->n_cand && 2ull * s->cand[a] < th) ++a;
  while (b > a && s->cand[b - 1] > 2ull * th) --b;
  if (a < b) {
    *lo = a;
    *hi = b;
  }
}

void count_build(sj_scene *s, uint32_t decision, bool tune) {
  if (decision != 1u) return;
  if (tune) {
    s->tuned = true;
    s->since_tune = 0;
  } else {
    s->since_tune += 1;
  }
}

// A tick of k-nearest-neighbour queries: query points, k, outputs.
struct KnnArgs {
  const float *qx, *qy;
  uint32_t k;
  uint32_t *out_id;
  float *out_d2;
};

// part: 0 the whole tick; 1 up to the result-offset scan; 2 the join write.
// The tick's query arrays are those last written to the scene's input block
// (for a kNN tick: the candidate squares, written by the radius kernel).
void enqueue_tick(sj_scene *s, uint32_t nq, uint32_t decision, uint64_t upd_total, bool events,
                  int part = 0, bool tune = false, const KnnArgs *knn = nullptr) {
  const hipStream_t st = s->stream;
  const uint32_t flags = s->cfg.flags;
  const uint32_t policy = s->cfg.rebuild_policy;
  auto rec = [&](int i) {
    if (events) (void)hipEventRecord(s->ev[i], st);
  };
  const bool sqb = (flags & SJ_ATOMIC_RESULTS) != 0;
  if (part == 2) {
    if (!sqb) sj::launch_join_write(s->B, nq, st);
    sj::launch_ctl_out(s->B, s->pin_ctl, st);
    return;
  }
  if (s->B.cu_tests) sj::launch_fill_u64(s->B.cu_tests, sj::kCuSlots, 0ull, st);
  rec(0);
  sj::launch_index(s->B, decision, policy, upd_total, nq, key_bits(s, decision), st);
  rec(1);
  if (tune) {
    uint32_t lo, hi;
    tune_window(s, &lo, &hi);
    sj::launch_tune(s->B, lo, hi, s->l_max, nq, (flags & SJ_COVERING) ? 1u : 0u, st);
  }
  if (decision != 0u && !(flags & SJ_UNIFORM_GRID)) sj::launch_build(s->B, s->l_max, st);
  rec(2);
  sj::launch_leaves(s->B, st);
  if (knn) sj::launch_knn_radius(s->B, knn->qx, knn->qy, nq, knn->k, st);
  rec(3);
  const uint32_t *qord = sj::launch_split(s->B, nq, (flags & SJ_COVERING) ? 1u : 0u, st);
  rec(4);
  const bool learned = (flags & SJ_SCHEDULE_MLP) && s->cm_set;
  sj::launch_schedule(s->B, (flags & SJ_REORDER) ? 1u : 0u, s->l_max, learned, st);
  rec(5);
  if (sqb) {
    // the baseline filter appends every result (timed as the count phase),
    // then the tick's totals
    sj::launch_join_sqb(s->B, nq, qord, st);
    rec(6);
    sj::launch_join_top_sqb(s->B, s->B.R, policy, s->period, st);
  } else {
    sj::launch_join_count(s->B, st);
    rec(6);
    sj::launch_join_scan(s->B, s->B.R, policy, s->period, st);
  }
  rec(7);
  if (part == 1) return;
  if (!sqb) sj::launch_join_write(s->B, nq, st);
  rec(8);
  if (knn) sj::launch_knn_select(s->B, knn->qx, knn->qy, nq, knn->k, knn->out_id, knn->out_d2, st);
  rec(9);
  sj::launch_ctl_out(s->B, s->pin_ctl, st);
  s->events_valid = events;
  s->join_events = false;
}

void after_tick(sj_scene *s, const uint32_t *d_qid, uint32_t nq) {
  s->upd_pending = 0;
  s->force_pending = false;
  s->known = false;
  s->mirror = true;
  s->last_nq = nq;
  s->last_qid = d_qid;
  s->ticked = true;
}

}  // namespace

extern "C" {

size_t sj_workspace_bytes(const sj_config *cfg) {
  Derived d;
  char msg[256];
  if (derive(cfg, &d, msg, sizeof msg) != SJ_OK) return 0;
  return carve(d, nullptr, nullptr);
}

int sj_scene_create(const sj_config *cfg, void *d_workspace, size_t ws_bytes, hipStream_t stream,
                    sj_scene **out) {
  if (!out) return SJ_EINVAL;
  *out = nullptr;
  Derived d;
  int rc = derive(cfg, &d, g_create_err, sizeof g_create_err);
  if (rc != SJ_OK) return rc;
  const size_t need = carve(d, nullptr, nullptr);
  if (!d_workspace || ((uintptr_t)d_workspace & 255u)) {
    snprintf(g_create_err, sizeof g_create_err, "workspace must be a 256-byte aligned device pointer");
    return SJ_EINVAL;
  }
  if (ws_bytes < need) {
    snprintf(g_create_err, sizeof g_create_err, "workspace has %zu bytes, needs %zu", ws_bytes,
             need);
    return SJ_ENOSPACE;
  }
  sj_scene *s = new (std::nothrow) sj_scene();
  if (!s) return SJ_EINVAL;
  s->cfg = *cfg;
  s->ws = (uint8_t *)d_workspace;
  s->ws_bytes = ws_bytes;
  s->stream = stream;
  s->th = d.th;
  s->l_max = d.l_max;
  s->period = d.period;
  s->prof = (cfg->flags & SJ_PROFILE) != 0;
  s->tune_every = d.tune_every;
  s->known = true;  // host_ctl is zero: not built, the first tick builds
  (void)hipGetDevice(&s->device);
  if (hipHostMalloc((void **)&s->pin_ctl, sizeof(Ctl), hipHostMallocDefault) != hipSuccess) {
    snprintf(g_create_err, sizeof g_create_err, "hipHostMalloc failed");
    delete s;
    return SJ_EDEVICE;
  }
  carve(d, s->ws, &s->B);
  if (s->prof) {
    bool ok = true;
    for (auto &ev : s->ev) ok = ok && hipEventCreate(&ev) == hipSuccess;
    ok = ok && hipEventCreate(&s->ev_u0) == hipSuccess;
    ok = ok && hipEventCreate(&s->ev_u1) == hipSuccess;
    if (!ok) {
      snprintf(g_create_err, sizeof g_create_err, "hipEventCreate failed");
      (void)hipHostFree(s->pin_ctl);
      delete s;
      return SJ_EDEVICE;
    }
  }
  sj::launch_ctl_init(s->B.ctl, d.th, d.ug, d.ug_bits, cfg->rebuild_policy, stream);
  sj::launch_fill_u32((uint32_t *)s->B.pos, 2ull * d.N, 0x7fc00000u, stream);  // NaN: no position
  sj::launch_fill_u64(s->B.ustamp, d.N, 0ull, stream);
  sj::launch_fill_u64(s->B.qstamp, d.N, 0ull, stream);
  sj::launch_fill_u32((uint32_t *)s->B.tune, sizeof(sj::TuneState) / 4, 0u, stream);
  sj::launch_fill_u32((uint32_t *)s->B.tin, sizeof(sj::TickIn) / 4, 0u, stream);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    snprintf(g_create_err, sizeof g_create_err, "kernel launch: %s", hipGetErrorString(e));
    (void)hipHostFree(s->pin_ctl);
    delete s;
    return SJ_EDEVICE;
  }
  *out = s;
  return SJ_OK;
}

int sj_scene_destroy(sj_scene *s) {
  if (!s) return SJ_EINVAL;
  for (auto &g : s->graphs) {
    if (!g.valid) continue;
    (void)hipGraphExecDestroy(g.exec);
    if (g.split) (void)hipGraphExecDestroy(g.exec2);
  }
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  if (s->prof) {
    for (auto &e : s->ev) (void)hipEventDestroy(e);
    (void)hipEventDestroy(s->ev_u0);
    (void)hipEventDestroy(s->ev_u1);
  }
  (void)hipHostFree(s->pin_ctl);
  delete s;
  return SJ_OK;
}

int sj_apply_updates(sj_scene *s, const uint32_t *d_id, const float *d_x, const float *d_y,
                     uint32_t m) {
  if (!s) return SJ_EINVAL;
  if (m == 0) return SJ_OK;
  if (!d_id || !d_x || !d_y || ((uintptr_t)d_id & 3u) || ((uintptr_t)d_x & 3u) ||
      ((uintptr_t)d_y & 3u))
    return fail(s, SJ_EINVAL, "apply_updates: null or misaligned pointer");
  if (s->prof && !s->upd_open) {
    (void)hipEventRecord(s->ev_u0, s->stream);
    s->upd_open = true;
  }
  s->mirror = false;  // the control block changes after the last tick's copy
  sj::TickIn in{};
  in.id = d_id;
  in.x = d_x;
  in.y = d_y;
  sj::launch_tick_in(s->B, in, 1u, s->stream);
  sj::launch_updates(s->B, m, s->upd_pending, s->stream);
  s->upd_pending += m;
  if (s->prof) (void)hipEventRecord(s->ev_u1, s->stream);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SJ_OK : hip_fail(s, e, "apply_updates launch");
}

int sj_build_index(sj_scene *s, uint32_t th) {
  if (!s) return SJ_EINVAL;
  const uint32_t th_min = s->cfg.th_min ? s->cfg.th_min : s->th;
  if (th && th < th_min) return fail(s, SJ_EINVAL, "build_index: th below th_min");
  s->mirror = false;
  sj::launch_request_build(s->B.ctl, th, s->stream);
  s->force_pending = true;
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SJ_OK : hip_fail(s, e, "build_index launch");
}

int sj_run_tick(sj_scene *s, const uint32_t *d_qid, const float *d_xa, const float *d_ya,
                const float *d_xb, const float *d_yb, uint32_t nq) {
  if (!s) return SJ_EINVAL;
  int rc = check_tick_args(s, d_qid, d_xa, d_ya, d_xb, d_yb, nq);
  if (rc != SJ_OK) return rc;
  const uint32_t decision = host_decision(s);
  const bool tune = want_tune(s, decision);
  sj::TickIn in{};
  in.qid = d_qid;
  in.xa = d_xa;
  in.ya = d_ya;
  in.xb = d_xb;
  in.yb = d_yb;
  sj::launch_tick_in(s->B, in, 2u, s->stream);
  enqueue_tick(s, nq, decision, s->upd_pending, s->prof, 0, tune);
  count_build(s, decision, tune);
  after_tick(s, d_qid, nq);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SJ_OK : hip_fail(s, e, "run_tick launch");
}

int sj_run_knn(sj_scene *s, const uint32_t *d_qid, const float *d_qx, const float *d_qy,
               uint32_t nq, uint32_t k, uint32_t *d_out_id, float *d_out_d2) {
  if (!s) return SJ_EINVAL;
  if (k < 1u || k > SJ_KNN_MAX) return fail(s, SJ_EINVAL, "run_knn: k must be in 1..64");
  if (s->cfg.flags & (SJ_UNIFORM_GRID | SJ_ATOMIC_RESULTS))
    return fail(s, SJ_EINVAL, "run_knn: needs the quadtree and the lock-free join");
  if (nq > s->B.Q) return fail(s, SJ_EINVAL, "run_knn: nq above capacity_queries");
  if (nq && (!d_qid || !d_qx || !d_qy || !d_out_id || !d_out_d2 || ((uintptr_t)d_qid & 3u) ||
             ((uintptr_t)d_qx & 3u) || ((uintptr_t)d_qy & 3u) || ((uintptr_t)d_out_id & 3u) ||
             ((uintptr_t)d_out_d2 & 3u)))
    return fail(s, SJ_EINVAL, "run_knn: null or misaligned pointer");
  const uint32_t decision = host_decision(s);
  sj::TickIn in{};
  in.qid = d_qid;
  const uint64_t Q = s->B.Q;
  in.xa = s->B.kq_rect;
  in.ya = s->B.kq_rect + Q;
  in.xb = s->B.kq_rect + 2 * Q;
  in.yb = s->B.kq_rect + 3 * Q;
  sj::launch_tick_in(s->B, in, 2u, s->stream);
  const KnnArgs a{d_qx, d_qy, k, d_out_id, d_out_d2};
  enqueue_tick(s, nq, decision, s->upd_pending, s->prof, 0, false, &a);
  count_build(s, decision, false);
  after_tick(s, d_qid, nq);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(s, e, "run_knn launch");
  const int rc = sync_ctl(s);
  if (rc != SJ_OK) return rc;
  return status_of(s, s->host_ctl.err);
}

// Event record nodes e0 -> (join write kernel node) -> e1 in a captured
// tick: the kernel node's incoming edges move to e0, its outgoing edges to
// e1.  False (graph possibly edited) if the node or an edit is refused.
static bool time_join_node(hipGraph_t graph, hipEvent_t e0, hipEvent_t e1) {
  size_t n = 0;
  if (hipGraphGetNodes(graph, nullptr, &n) != hipSuccess || n == 0) return false;
  hipGraphNode_t *nodes = new (std::nothrow) hipGraphNode_t[n];
  if (!nodes) return false;
  hipGraphNode_t kw = nullptr;
  if (hipGraphGetNodes(graph, nodes, &n) == hipSuccess) {
    for (size_t i = 0; i < n && !kw; ++i) {
      hipGraphNodeType t;
      hipKernelNodeParams kp;
      if (hipGraphNodeGetType(nodes[i], &t) != hipSuccess || t != hipGraphNodeTypeKernel) continue;
      if (hipGraphKernelNodeGetParams(nodes[i], &kp) != hipSuccess) continue;
      if (kp.func == sj::join_write_kernel()) kw = nodes[i];
    }
  }
  delete[] nodes;
  if (!kw) return false;
  size_t np = 0, ns = 0;
  if (hipGraphNodeGetDependencies(kw, nullptr, &np) != hipSuccess ||
      hipGraphNodeGetDependentNodes(kw, nullptr, &ns) != hipSuccess || np > 8 || ns > 8)
    return false;
  hipGraphNode_t pre[8], suc[8], a, b;
  if ((np && hipGraphNodeGetDependencies(kw, pre, &np) != hipSuccess) ||
      (ns && hipGraphNodeGetDependentNodes(kw, suc, &ns) != hipSuccess))
    return false;
  for (size_t i = 0; i < np; ++i)
    if (hipGraphRemoveDependencies(graph, &pre[i], &kw, 1) != hipSuccess) return false;
  for (size_t i = 0; i < ns; ++i)
    if (hipGraphRemoveDependencies(graph, &kw, &suc[i], 1) != hipSuccess) return false;
  if (hipGraphAddEventRecordNode(&a, graph, np ? pre : nullptr, np, e0) != hipSuccess) return false;
  if (hipGraphAddDependencies(graph, &a, &kw, 1) != hipSuccess) return false;
  if (hipGraphAddEventRecordNode(&b, graph, &kw, 1, e1) != hipSuccess) return false;
  for (size_t i = 0; i < ns; ++i)
    if (hipGraphAddDependencies(graph, &b, &suc[i], 1) != hipSuccess) return false;
  return true;
}

int sj_tick_graph(sj_scene *s, const uint32_t *d_id, const float *d_x, const float *d_y,
                  uint32_t m, const uint32_t *d_qid, const float *d_xa, const float *d_ya,
                  const float *d_xb, const float *d_yb, uint32_t nq) {
  if (!s) return SJ_EINVAL;
  if (m && (!d_id || !d_x || !d_y || ((uintptr_t)d_id & 3u) || ((uintptr_t)d_x & 3u) ||
            ((uintptr_t)d_y & 3u)))
    return fail(s, SJ_EINVAL, "tick_graph: null or misaligned update pointer");
  int rc = check_tick_args(s, d_qid, d_xa, d_ya, d_xb, d_yb, nq);
  if (rc != SJ_OK) return rc;
  if (s->upd_pending) {
    // updates already enqueued for this tick: their sequence numbers are
    // not those a graph would replay, so run this tick eagerly
    rc = sj_apply_updates(s, d_id, d_x, d_y, m);
    return rc != SJ_OK ? rc : sj_run_tick(s, d_qid, d_xa, d_ya, d_xb, d_yb, nq);
  }
  const uint32_t decision = host_decision(s);
  const bool tune = want_tune(s, decision);
  GraphSlot &g = s->graphs[tune ? 3u : decision];
  const uint32_t kb = key_bits(s, decision);
  uint32_t t_lo = 0, t_hi = 0;
  if (tune) tune_window(s, &t_lo, &t_hi);
  if (!(g.valid && g.m == m && g.nq == nq && g.key_bits == kb && g.t_lo == t_lo &&
        g.t_hi == t_hi)) {
    if (g.valid) {
      (void)hipGraphExecDestroy(g.exec);
      if (g.split) (void)hipGraphExecDestroy(g.exec2);
      g.valid = false;
    }
    // capture on a private stream (the caller's may be the null stream,
    // which cannot be captured); the graph is launched on the scene's stream.
    // Profiled scenes capture the join write pass as a graph of its own and
    // time it with events recorded around it.
    if (!s->cap_stream) {
      hipError_t e = hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking);
      if (e != hipSuccess) return hip_fail(s, e, "hipStreamCreate");
    }
    const hipStream_t user = s->stream;
    auto capture = [&](int part, hipGraph_t *out) -> int {
      hipError_t e = hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return hip_fail(s, e, "hipStreamBeginCapture");
      s->stream = s->cap_stream;
      if (part != 2 && m) sj::launch_updates(s->B, m, 0, s->stream);
      enqueue_tick(s, nq, decision, m, false, part, tune);
      s->stream = user;
      e = hipStreamEndCapture(s->cap_stream, out);
      return e == hipSuccess ? SJ_OK : hip_fail(s, e, "hipStreamEndCapture");
    };
    auto instantiate = [&](hipGraph_t graph, hipGraphExec_t *out) -> int {
      hipError_t e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
      return e == hipSuccess ? SJ_OK : hip_fail(s, e, "hipGraphInstantiate");
    };
    g.split = false;
    if (!s->prof) {
      hipGraph_t graph;
      rc = capture(0, &graph);
      if (rc != SJ_OK) return rc;
      rc = instantiate(graph, &g.exec);
      (void)hipGraphDestroy(graph);
      if (rc != SJ_OK) return rc;
    } else {
      // one launch: the captured tick with event nodes inserted right
      // around its join write node; else the tick up to the join write pass
      // and the pass as child graphs with event nodes between them; else two
      // launches with the events recorded between them
      {
        hipGraph_t graph;
        rc = capture(0, &graph);
        if (rc != SJ_OK) return rc;
        const bool ok = time_join_node(graph, s->ev[7], s->ev[8]) &&
                        hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0) == hipSuccess;
        (void)hipGraphDestroy(graph);
        (void)hipGetLastError();  // a refused edit is not an error of the tick
        if (ok) goto captured;
      }
      hipGraph_t g1, g2, top = nullptr;
      rc = capture(1, &g1);
      if (rc != SJ_OK) return rc;
      rc = capture(2, &g2);
      if (rc != SJ_OK) {
        (void)hipGraphDestroy(g1);
        return rc;
      }
      hipGraphNode_t n1, e1, n2, e2;
      bool ok = hipGraphCreate(&top, 0) == hipSuccess;
      ok = ok && hipGraphAddChildGraphNode(&n1, top, nullptr, 0, g1) == hipSuccess;
      ok = ok && hipGraphAddEventRecordNode(&e1, top, &n1, 1, s->ev[7]) == hipSuccess;
      ok = ok && hipGraphAddChildGraphNode(&n2, top, &e1, 1, g2) == hipSuccess;
      ok = ok && hipGraphAddEventRecordNode(&e2, top, &n2, 1, s->ev[8]) == hipSuccess;
      ok = ok && hipGraphInstantiate(&g.exec, top, nullptr, nullptr, 0) == hipSuccess;
      if (top) (void)hipGraphDestroy(top);
      (void)hipGetLastError();  // a refused node is not an error of the tick
      if (!ok) {
        g.split = true;
        rc = instantiate(g1, &g.exec);
        if (rc == SJ_OK) {
          rc = instantiate(g2, &g.exec2);
          if (rc != SJ_OK) (void)hipGraphExecDestroy(g.exec);
        }
      }
      (void)hipGraphDestroy(g1);
      (void)hipGraphDestroy(g2);
      if (rc != SJ_OK) return rc;
    }
  captured:
    g.valid = true;
    g.m = m;
    g.nq = nq;
    g.key_bits = kb;
    g.t_lo = t_lo;
    g.t_hi = t_hi;
  }
  // the graph reads this tick's arrays from the scene's input block
  const sj::TickIn in{d_id, d_x, d_y, d_qid, d_xa, d_ya, d_xb, d_yb};
  sj::launch_tick_in(s->B, in, 3u, s->stream);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipGraphLaunch(g.exec, s->stream);
  if (e == hipSuccess && g.split) {
    e = hipEventRecord(s->ev[7], s->stream);
    if (e == hipSuccess) e = hipGraphLaunch(g.exec2, s->stream);
    if (e == hipSuccess) e = hipEventRecord(s->ev[8], s->stream);
  }
  if (e != hipSuccess) return hip_fail(s, e, "hipGraphLaunch");
  count_build(s, decision, tune);
  after_tick(s, d_qid, nq);
  s->events_valid = false;
  s->join_events = s->prof;
  s->upd_open = false;
  return SJ_OK;
}

int sj_tick_counters(sj_scene *s, uint64_t *d_out) {
  if (!s || !d_out || ((uintptr_t)d_out & 7u)) return SJ_EINVAL;
  sj::launch_counters(s->B, d_out, s->stream);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SJ_OK : hip_fail(s, e, "tick_counters launch");
}

int sj_stats(sj_scene *s, sj_tick_stats *out) {
  if (!s || !out) return SJ_EINVAL;
  int rc = sync_ctl(s);
  if (rc != SJ_OK) return rc;
  const Ctl &c = s->host_ctl;
  memset(out, 0, sizeof *out);
  out->n_present = c.n_present;
  out->n_leaves = c.n_leaves;
  out->n_nodes = (c.n_leaves > 0) ? (c.n_leaves - 1) / 3 : 0;
  out->l_deep = c.l_deep;
  out->th = c.th_cur;
  out->rebuilt = c.rebuild;
  out->n_tasks = c.n_tasks;
  out->max_leaf = c.max_leaf;
  out->n_isect = c.n_isect;
  out->n_cov = c.n_cov;
  out->n_isect_ids = c.n_res;
  out->cov_pairs = c.cov_pairs;
  out->tests = c.tests;
  out->error_bits = c.err;
  out->tick = c.tick;
  out->knn_fallback = c.n_knn_fb;
  return s->ticked ? status_of(s, c.err) : SJ_OK;
}

int sj_fetch_results(sj_scene *s, sj_results *out) {
  if (!s || !out) return SJ_EINVAL;
  if (!s->ticked) return fail(s, SJ_ESTATE, "fetch_results before run_tick");
  int rc = sync_ctl(s);
  if (rc != SJ_OK) return rc;
  const Ctl &c = s->host_ctl;
  memset(out, 0, sizeof *out);
  const bool ok = c.go_join != 0;
  out->nq = s->last_nq;
  out->n_leaves = c.n_leaves;
  out->n_isect_ids = ok ? c.n_res : 0;
  out->n_cov_entries = ok ? c.n_cov : 0;
  out->total_pairs = ok ? c.n_res + c.cov_pairs : 0;
  out->n_runs = ok && !s->B.pairs ? c.n_isect : 0;
  out->n_pairs = ok && s->B.pairs ? c.n_res : 0;
  out->d_pairs = (const uint32_t *)s->B.pairs;
  out->d_isect_slot_off = s->B.q_ioff;
  out->d_slot_run = s->B.slot_sq;
  out->d_run_off = s->B.res_off;
  out->d_isect_id = s->B.res_ids;
  out->d_cov_off = s->B.q_coff;
  out->d_query_pos = s->B.qpos;
  out->d_cov_leaf = s->B.cov_leaf;
  out->d_leaf_beg = s->B.leaf_beg;
  out->d_sorted_id = s->B.valA;
  out->n_present = c.n_present;
  out->n_tasks = c.n_tasks;
  out->n_subqueries = c.n_isect;
  out->cov_pairs = ok ? c.cov_pairs : 0;
  out->tests = c.tests;
  out->error_bits = c.err;
  return status_of(s, c.err);
}

int sj_result_hashes(sj_scene *s, uint64_t *d_count, uint64_t *d_hash) {
  if (!s || !d_count || !d_hash) return SJ_EINVAL;
  if (!s->ticked) return fail(s, SJ_ESTATE, "result_hashes before run_tick");
  sj::launch_hash(s->B, s->last_nq, s->last_qid, d_count, d_hash, s->stream);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SJ_OK : hip_fail(s, e, "result_hashes launch");
}

int sj_expand_results(sj_scene *s, const uint32_t *d_sel, uint32_t n_sel, uint32_t flags,
                      uint64_t *d_off, uint32_t *d_ids, uint64_t ids_cap, uint64_t *n_pairs) {
  if (!s) return SJ_EINVAL;
  if (!s->ticked) return fail(s, SJ_ESTATE, "expand_results before run_tick");
  if (flags & ~(uint32_t)SJ_SORTED) return fail(s, SJ_EINVAL, "expand_results: unknown flags");
  if (d_sel && s->B.pairs)
    return fail(s, SJ_EINVAL, "expand_results: no selection with appended pairs (SJ_ATOMIC_RESULTS)");
  if (d_sel && (((uintptr_t)d_sel & 3u) || !d_off || ((uintptr_t)d_off & 7u) ||
                n_sel > s->B.Q))
    return fail(s, SJ_EINVAL,
                "expand_results: a selection needs aligned d_sel and d_off, n_sel <= "
                "capacity_queries");
  int rc = sync_ctl(s);
  if (rc != SJ_OK) return rc;
  const Ctl &c = s->host_ctl;
  rc = status_of(s, c.err);
  if (rc == SJ_EOVERFLOW) return rc;
  const uint32_t n = d_sel ? n_sel : s->last_nq;
  uint64_t total = c.go_join ? c.n_res + c.cov_pairs : 0;
  if (d_sel) {
    // sizes of the selected lists: counted and scanned into d_off, the total
    // and the index check read back
    uint32_t *bad = &s->B.ctl->exp_bad;
    sj::launch_fill_u32(bad, 1, 0u, s->stream);
    sj::launch_expand_count(s->B, s->last_nq, d_sel, n, d_off, bad, s->stream);
    uint32_t hbad = 0;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
      e = hipMemcpyAsync(&total, d_off + n, sizeof total, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(&hbad, bad, sizeof hbad, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "expand_results count");
    if (hbad) return fail(s, SJ_EINVAL, "expand_results: selected query index >= nq");
  }
  if (n_pairs) *n_pairs = total;
  if (!d_ids) return rc;
  if (!d_off || ((uintptr_t)d_off & 7u) || ((uintptr_t)d_ids & 3u) || ids_cap < total)
    return fail(s, SJ_EINVAL, "expand_results: missing, misaligned or too small buffer");
  if (!d_sel) sj::launch_expand_count(s->B, s->last_nq, nullptr, n, d_off, &s->B.ctl->exp_bad,
                                      s->stream);
  sj::launch_expand(s->B, s->last_nq, d_sel, n, d_off, d_ids, (flags & SJ_SORTED) != 0,
                    s->stream);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(s, e, "expand_results launch");
  e = hipStreamSynchronize(s->stream);
  return e == hipSuccess ? rc : hip_fail(s, e, "expand_results sync");
}

int sj_phase_times(sj_scene *s, float *ms, int n) {
  if (!s || !ms || n < 0) return SJ_EINVAL;
  if (!s->prof) return fail(s, SJ_ESTATE, "scene created without SJ_PROFILE");
  if (!s->events_valid && !s->join_events) return fail(s, SJ_ESTATE, "no tick timed yet");
  hipError_t e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "phase_times sync");
  float t[SJ_PH_COUNT] = {0};
  auto elapsed = [&](float *out, hipEvent_t a, hipEvent_t b) {
    hipError_t r = hipEventElapsedTime(out, a, b);
    if (r != hipSuccess) {
      (void)hipGetLastError();  // do not leave a sticky error for other callers
      if (e == hipSuccess) e = r;
      *out = 0.0f;
    }
  };
  if (s->join_events) {
    // graph tick: only the join write pass is bracketed by events
    elapsed(&t[SJ_PH_JOIN_WRITE], s->ev[7], s->ev[8]);
  } else {
    if (s->upd_open) elapsed(&t[SJ_PH_UPDATES], s->ev_u0, s->ev_u1);
    // events 0..9 bracket: index, build, leaves, split, schedule, join count,
    // join scan, join write, finish (counted with the join scan)
    float d[9];
    for (int i = 0; i < 9; ++i) elapsed(&d[i], s->ev[i], s->ev[i + 1]);
    t[SJ_PH_INDEX] = d[0];
    t[SJ_PH_BUILD] = d[1];
    t[SJ_PH_LEAVES] = d[2];
    t[SJ_PH_SPLIT] = d[3];
    t[SJ_PH_SCHEDULE] = d[4];
    t[SJ_PH_JOIN_COUNT] = d[5];
    t[SJ_PH_JOIN_SCAN] = d[6] + d[8];
    t[SJ_PH_JOIN_WRITE] = d[7];
  }
  for (int i = 0; i < n && i < SJ_PH_COUNT; ++i) ms[i] = t[i];
  s->upd_open = false;
  return e == hipSuccess ? SJ_OK : hip_fail(s, e, "hipEventElapsedTime");
}

int sj_set_cost_model(sj_scene *s, const uint16_t *d_w, const float coef[SJ_COST_TERMS],
                      const uint32_t *cand,
                      uint32_t n_cand) {
  if (!s || !d_w || !coef || !cand) return SJ_EINVAL;
  if (s->cfg.flags & SJ_UNIFORM_GRID)
    return fail(s, SJ_EINVAL, "set_cost_model: the uniform grid has no threshold to tune");
  if (n_cand == 0 || n_cand > (uint32_t)sj::kMaxCand)
    return fail(s, SJ_EINVAL, "set_cost_model: n_cand must be in 1..8");
  const uint32_t th_min = s->cfg.th_min ? s->cfg.th_min : s->th;
  for (uint32_t c = 0; c < n_cand; ++c) {
    if (cand[c] < th_min || cand[c] == 0)
      return fail(s, SJ_EINVAL, "set_cost_model: candidate below th_min");
    if (c && cand[c] <= cand[c - 1])
      return fail(s, SJ_EINVAL, "set_cost_model: candidates must be ascending");
  }
  struct {
    float coef[SJ_COST_TERMS];
    uint32_t n_cand;
    uint32_t cand[sj::kMaxCand];
  } h{};
  for (int i = 0; i < SJ_COST_TERMS; ++i) h.coef[i] = coef[i];
  h.n_cand = n_cand;
  for (uint32_t c = 0; c < n_cand; ++c) h.cand[c] = cand[c];
  static_assert(offsetof(sj::TuneState, n_cand) ==
                    offsetof(sj::TuneState, coef) + 4 * SJ_COST_TERMS, "layout");
  static_assert(offsetof(sj::TuneState, cand) == offsetof(sj::TuneState, n_cand) + 4, "layout");
  sj::TuneState *ts = s->B.tune;
  hipError_t e = hipMemcpyAsync(ts->w, d_w, 4545 * sizeof(uint16_t), hipMemcpyDeviceToDevice,
                                s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ts->coef, &h, sizeof h, hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "set_cost_model copy");
  s->cm_set = true;
  s->n_cand = n_cand;
  for (uint32_t c = 0; c < n_cand; ++c) s->cand[c] = cand[c];
  s->tuned = false;
  s->since_tune = 0;
  for (GraphSlot &g : s->graphs) {  // captured with the previous model state
    if (!g.valid) continue;
    (void)hipGraphExecDestroy(g.exec);
    if (g.split) (void)hipGraphExecDestroy(g.exec2);
    g.valid = false;
  }
  return SJ_OK;
}

int sj_tune_info_get(sj_scene *s, sj_tune_info *out) {
  if (!s || !out) return SJ_EINVAL;
  sj::TuneState h;
  hipError_t e = hipMemcpyAsync(&h, s->B.tune, sizeof h, hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "tune_info copy");
  memset(out, 0, sizeof *out);
  out->n_cand = h.n_cand < (uint32_t)sj::kMaxCand ? h.n_cand : (uint32_t)sj::kMaxCand;
  for (uint32_t c = 0; c < out->n_cand; ++c) {
    out->cand[c] = h.cand[c];
    out->cost[c] = h.cost[c];
    out->mlp_sum[c] = h.msum[c];
    out->mlp_max[c] = h.mmax[c];
  }
  out->chosen = h.chosen;
  out->n_tunes = h.n_tunes;
  out->tuned_tick = h.tuned_tick;
  return SJ_OK;
}

int sj_timing_log(sj_scene *s, sj_timing_view *out) {
  if (!s || !out) return SJ_EINVAL;
  if (!s->B.tlog) return fail(s, SJ_ESTATE, "scene created without SJ_TIMING_LOG");
  int rc = sync_ctl(s);
  if (rc != SJ_OK) return rc;
  int khz = 0;
  hipError_t e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, s->device);
  if (e != hipSuccess) return hip_fail(s, e, "wall clock rate");
  out->n_leaves = s->host_ctl.n_leaves;
  out->clock_mhz = (float)khz / 1000.0f;
  out->d_records = s->B.tlog;
  return SJ_OK;
}

int sj_index_view_get(sj_scene *s, sj_index_view *out) {
  if (!s || !out) return SJ_EINVAL;
  int rc = sync_ctl(s);
  if (rc != SJ_OK) return rc;
  const Ctl &c = s->host_ctl;
  memset(out, 0, sizeof *out);
  out->n_present = c.n_present;
  out->n_leaves = c.n_leaves;
  out->l_deep = c.l_deep;
  out->x0 = c.x0;
  out->y0 = c.y0;
  out->e = c.e;
  out->d_codes = s->B.keyA;
  out->d_ids = s->B.valA;
  out->d_leaf_start = s->B.lstart;
  out->d_leaf_level = s->B.llevel;
  out->d_leaf_beg = s->B.leaf_beg;
  out->d_pos = (const float *)s->B.pos;
  return SJ_OK;
}

int sj_cu_counters(sj_scene *s, uint64_t *out, uint32_t n) {
  if (!s || !out || n == 0 || n > sj::kCuSlots) return SJ_EINVAL;
  if (!s->B.cu_tests) return fail(s, SJ_ESTATE, "scene created without SJ_CU_COUNTERS");
  hipError_t e = hipMemcpyAsync(out, s->B.cu_tests, (size_t)n * sizeof(uint64_t),
                                hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  return e == hipSuccess ? SJ_OK : hip_fail(s, e, "cu_counters copy");
}

const char *sj_last_error(const sj_scene *s) { return s ? s->err : g_create_err; }


}  // extern "C"

int sj_scene_ctl_to_host_async(sj_scene *s, Ctl *h_ctl) {
  hipError_t e = hipMemcpyAsync(h_ctl, s->B.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s->stream);
  return e == hipSuccess ? SJ_OK : hip_fail(s, e, "control block copy");
}

void sj_scene_ctl_from_host(sj_scene *s, const Ctl *h_ctl) {
  memcpy(&s->host_ctl, h_ctl, sizeof(Ctl));
  s->known = true;
}

int sj_scene_status(sj_scene *s) { return status_of(s, s->host_ctl.err); }

int sj_scene_positions_copy(sj_scene *s, void *h_pos, int to_host) {
  const size_t bytes = (size_t)s->B.N * sizeof(float2);
  hipError_t e = to_host ? hipMemcpyAsync(h_pos, s->B.pos, bytes, hipMemcpyDeviceToHost, s->stream)
                         : hipMemcpyAsync(s->B.pos, h_pos, bytes, hipMemcpyHostToDevice, s->stream);
  return e == hipSuccess ? SJ_OK : hip_fail(s, e, "positions copy");
}

void sj_set_global_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_create_err, sizeof g_create_err, fmt, ap);
  va_end(ap);
}
