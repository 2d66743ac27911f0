// Tick-serving runtime: many scenes, one device, continuous batching.
//
// A resident scene holds a workspace and two sets of output slots carved
// from a caller-provided device pool (first-fit allocator, 256-byte blocks,
// freed blocks coalesce), and has its own stream.  Tick requests (device
// input buffers, read in place by the tick, so they stay valid until it is
// retired) queue per scene in arrival order.  sj_server_poll retires
// finished ticks and starts queued ones: a request starts when its scene has
// no tick in flight and fewer than `max_running` ticks run; ticks of
// different scenes overlap on the device.  A tick is: the scene's captured
// graph (updates + join) on the request's arrays, per-query counts and
// pair-set hashes and the tick counters into the output slots, an
// asynchronous copy of the control block to pinned host memory (so the
// quadtree decision of the next tick is known on the host), an event.
//
// Eviction: an idle scene can leave the device.  Its state that results
// depend on, the last-known position of every object (Definition 1 reads
// nothing else), is copied to pinned host memory, with its configuration
// and current leaf threshold; its pool memory is returned.  When a request
// of a scene that is not resident comes up in arrival order, the poll
// admits it again (a new workspace, the positions copied back; its next
// tick builds a quadtree), evicting least recently used idle scenes that
// the server manages when the pool is full.  A scene that waits for memory
// holds back the admission of scenes behind it, not the ticks of resident
// scenes.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <chrono>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "sj.h"
#include "sj_device.h"
#include "sj_scene.h"

using sj::Ctl;

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// First-fit allocator over [base, base + size): a sorted map of free ranges.
struct PoolAlloc {
  uint8_t *base = nullptr;
  size_t size = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  size_t used = 0;

  void init(void *b, size_t n) {
    base = (uint8_t *)b;
    size = n & ~(kAlign - 1);
    free_.clear();
    if (size) free_[0] = size;
    used = 0;
  }
  void *alloc(size_t n) {
    n = align_up(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const size_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > n) free_[off + n] = len - n;
      used += n;
      return base + off;
    }
    return nullptr;
  }
  void release(void *p, size_t n) {
    n = align_up(n);
    size_t off = (size_t)((uint8_t *)p - base);
    used -= n;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + n == next->first) {
      n += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += n;
        return;
      }
    }
    free_[off] = n;
  }
};

struct Request {
  uint64_t tag;
  uint64_t *record;
  bool digest;
  const uint32_t *id;
  const float *x, *y;
  uint32_t m;
  const uint32_t *qid;
  const float *xa, *ya, *xb, *yb;
  uint32_t nq;
};

struct ServedScene {
  bool live = false;      // registered (admitted, or added to be admitted on demand)
  bool resident = false;  // holds pool memory and a scene object
  bool managed = false;   // the poll may evict it when idle
  sj_config cfg{};        // as admitted; th_quad follows the scene's threshold
  sj_scene *scene = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  uint8_t *mem = nullptr;
  size_t mem_bytes = 0;
  uint32_t max_updates = 0, max_queries = 0;
  // output slots, two sets used by alternate ticks: the set of a finished
  // tick stays valid while the scene's next tick runs
  uint64_t *o_cnt[2], *o_hash[2], *o_counters[2];
  uint32_t parity = 0;
  Ctl *h_ctl = nullptr;  // pinned copy of the control block
  std::deque<Request> queue;
  bool running = false;
  Request cur{};
  bool has_result = false;
  Request last{};
  int status = SJ_OK;
  float2 *snap = nullptr;  // pinned host positions of an evicted scene
  bool has_snap = false;
  uint64_t last_use = 0;   // server clock at its last admission or retired tick
  uint64_t retired_poll = 0;  // the poll that retired its last tick
};

// Tick record: the 8 tick counters, then the digest of the tick's results:
// sum of the per-query pair-set hashes and sum of the result sizes (mod 2^64).
__global__ void k_record_init(const uint64_t *counters, uint64_t *record) {
  for (int i = 0; i < 8; ++i) record[i] = counters[i];
  record[8] = 0;
  record[9] = 0;
}

__global__ void __launch_bounds__(256) k_record_digest(const uint64_t *cnt, const uint64_t *hash,
                                                       uint32_t nq, uint64_t *record) {
  __shared__ uint64_t sh[4], sc[4];
  uint64_t h = 0, c = 0;
  for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < nq; i += gridDim.x * 256) {
    h += hash[i];
    c += cnt[i];
  }
  h = sj::wave_sum(h);
  c = sj::wave_sum(c);
  if ((threadIdx.x & 63) == 0) {
    sh[threadIdx.x / 64] = h;
    sc[threadIdx.x / 64] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    h = sh[0] + sh[1] + sh[2] + sh[3];
    c = sc[0] + sc[1] + sc[2] + sc[3];
    atomicAdd((unsigned long long *)&record[8], (unsigned long long)h);
    atomicAdd((unsigned long long *)&record[9], (unsigned long long)c);
  }
}

}  // namespace

struct sj_server {
  PoolAlloc pool;
  uint32_t max_running = 4;
  uint32_t running = 0;
  uint64_t clock = 0;
  uint64_t polls = 0;
  uint32_t admissions = 0, evictions = 0;
  std::vector<ServedScene> scenes;
  std::deque<std::pair<uint32_t, uint64_t>> order;  // (scene, tag) in arrival order
  char err[256] = "";
};

static int srv_fail(sj_server *s, int code, const char *msg) {
  snprintf(s->err, sizeof s->err, "%s", msg);
  return code;
}

static char g_server_err[256] = "";

extern "C" {

int sj_server_create(void *d_pool, size_t pool_bytes, uint32_t max_running, sj_server **out) {
  if (!out || !d_pool || ((uintptr_t)d_pool & (kAlign - 1)) || pool_bytes < kAlign) {
    snprintf(g_server_err, sizeof g_server_err, "server: bad pool");
    return SJ_EINVAL;
  }
  sj_server *s = new (std::nothrow) sj_server();
  if (!s) return SJ_EINVAL;
  s->pool.init(d_pool, pool_bytes);
  s->max_running = max_running ? max_running : 4;
  *out = s;
  return SJ_OK;
}

int sj_server_destroy(sj_server *s) {
  if (!s) return SJ_EINVAL;
  for (auto &sc : s->scenes) {
    if (!sc.live) continue;
    if (sc.stream) (void)hipStreamSynchronize(sc.stream);
    if (sc.resident) sj_scene_destroy(sc.scene);
    if (sc.done) (void)hipEventDestroy(sc.done);
    if (sc.stream) (void)hipStreamDestroy(sc.stream);
    if (sc.h_ctl) (void)hipHostFree(sc.h_ctl);
    if (sc.snap) (void)hipHostFree(sc.snap);
  }
  delete s;
  return SJ_OK;
}

size_t sj_server_scene_bytes(const sj_config *cfg, uint32_t max_updates) {
  (void)max_updates;  // updates are read where the caller keeps them
  const size_t ws = sj_workspace_bytes(cfg);
  if (!ws) return 0;
  const size_t Q = cfg->capacity_queries;
  return align_up(ws) + 4 * align_up(8 * Q) + 2 * align_up(64);
}

// A registered scene's stream, completion event and pinned control block
// (kept while it is evicted).
static int scene_handles(ServedScene &sc) {
  hipError_t e = hipStreamCreateWithFlags(&sc.stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&sc.done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipHostMalloc((void **)&sc.h_ctl, sizeof(Ctl), hipHostMallocDefault);
  if (e == hipSuccess) return SJ_OK;
  if (sc.done) (void)hipEventDestroy(sc.done);
  if (sc.stream) (void)hipStreamDestroy(sc.stream);
  sc.done = nullptr;
  sc.stream = nullptr;
  return SJ_EDEVICE;
}

// Pool memory, output slots and a scene object for a registered scene, with
// the positions of its snapshot copied back (ordered before its next tick
// on its stream).  SJ_ENOSPACE: the pool has no room now.
static int make_resident(sj_server *s, ServedScene &sc) {
  const size_t need = sj_server_scene_bytes(&sc.cfg, sc.max_updates);
  if (!need) return srv_fail(s, SJ_EINVAL, "admit: invalid scene configuration");
  uint8_t *mem = (uint8_t *)s->pool.alloc(need);
  if (!mem) return SJ_ENOSPACE;
  const size_t ws = align_up(sj_workspace_bytes(&sc.cfg));
  uint8_t *p = mem + ws;
  auto take = [&](size_t bytes) {
    uint8_t *r = p;
    p += align_up(bytes);
    return r;
  };
  const size_t Q = sc.cfg.capacity_queries;
  for (int b = 0; b < 2; ++b) {
    sc.o_cnt[b] = (uint64_t *)take(8 * Q);
    sc.o_hash[b] = (uint64_t *)take(8 * Q);
    sc.o_counters[b] = (uint64_t *)take(64);
  }
  int rc = sj_scene_create(&sc.cfg, mem, ws, sc.stream, &sc.scene);
  if (rc == SJ_OK && sc.has_snap) rc = sj_scene_positions_copy(sc.scene, sc.snap, 0);
  if (rc != SJ_OK) {
    srv_fail(s, rc, sc.scene ? sj_last_error(sc.scene) : sj_last_error(nullptr));
    if (sc.scene) sj_scene_destroy(sc.scene);
    sc.scene = nullptr;
    s->pool.release(mem, need);
    return rc;
  }
  sc.mem = mem;
  sc.mem_bytes = need;
  sc.parity = 0;
  sc.resident = true;
  sc.last_use = ++s->clock;
  s->admissions += 1;
  return SJ_OK;
}

// Moves an idle resident scene to host memory: positions, configuration and
// the threshold of its current quadtree; returns its pool memory.
static int evict_scene(sj_server *s, ServedScene &sc) {
  const size_t bytes = (size_t)sc.cfg.capacity_objects * sizeof(float2);
  if (!sc.snap && hipHostMalloc((void **)&sc.snap, bytes, hipHostMallocDefault) != hipSuccess) {
    sc.snap = nullptr;
    return srv_fail(s, SJ_EDEVICE, "evict: pinned snapshot allocation failed");
  }
  sj_tick_stats st{};
  const int rs = sj_stats(sc.scene, &st);  // synchronises the scene's stream
  if (rs == SJ_EDEVICE) return srv_fail(s, rs, sj_last_error(sc.scene));
  int rc = sj_scene_positions_copy(sc.scene, sc.snap, 1);
  if (rc == SJ_OK && hipStreamSynchronize(sc.stream) != hipSuccess) rc = SJ_EDEVICE;
  if (rc != SJ_OK) return srv_fail(s, rc, "evict: positions copy failed");
  // keep the threshold (the workspace stays sized for the same smallest one)
  if (!sc.cfg.th_min) sc.cfg.th_min = sc.cfg.th_quad ? sc.cfg.th_quad : 64u;
  if (st.th >= sc.cfg.th_min) sc.cfg.th_quad = st.th;
  sj_scene_destroy(sc.scene);
  sc.scene = nullptr;
  s->pool.release(sc.mem, sc.mem_bytes);
  sc.mem = nullptr;
  sc.resident = false;
  sc.has_snap = true;
  s->evictions += 1;
  return SJ_OK;
}

// Registers a scene slot; resident: admit it now (SJ_ENOSPACE if it does
// not fit), else it is admitted when its first request comes up.
static int register_scene(sj_server *s, const sj_config *cfg, uint32_t max_updates, bool resident,
                          uint32_t *scene_id) {
  if (!s || !cfg || !scene_id) return SJ_EINVAL;
  const size_t need = sj_server_scene_bytes(cfg, max_updates);
  if (!need) return srv_fail(s, SJ_EINVAL, "admit: invalid scene configuration");
  if (need > s->pool.size)
    return srv_fail(s, SJ_ENOSPACE, "admit: the scene is larger than the whole pool");
  ServedScene sc;
  sc.cfg = *cfg;
  sc.max_updates = max_updates;
  sc.max_queries = cfg->capacity_queries;
  sc.managed = !resident;
  if (scene_handles(sc) != SJ_OK)
    return srv_fail(s, SJ_EDEVICE, "admit: stream/event/pinned allocation failed");
  if (resident) {
    const int rc = make_resident(s, sc);
    if (rc != SJ_OK) {
      (void)hipEventDestroy(sc.done);
      (void)hipStreamDestroy(sc.stream);
      (void)hipHostFree(sc.h_ctl);
      return rc == SJ_ENOSPACE ? srv_fail(s, rc, "admit: the scene does not fit in the pool now")
                               : rc;
    }
  }
  sc.live = true;
  uint32_t id = 0;
  while (id < s->scenes.size() && s->scenes[id].live) ++id;
  if (id == s->scenes.size()) s->scenes.emplace_back();
  s->scenes[id] = sc;
  *scene_id = id;
  return SJ_OK;
}

int sj_server_admit(sj_server *s, const sj_config *cfg, uint32_t max_updates, uint32_t *scene_id) {
  return register_scene(s, cfg, max_updates, true, scene_id);
}

int sj_server_add(sj_server *s, const sj_config *cfg, uint32_t max_updates, uint32_t *scene_id) {
  return register_scene(s, cfg, max_updates, false, scene_id);
}

int sj_server_evict(sj_server *s, uint32_t id) {
  if (!s || id >= s->scenes.size() || !s->scenes[id].live) return SJ_EINVAL;
  ServedScene &sc = s->scenes[id];
  if (!sc.resident) return srv_fail(s, SJ_ESTATE, "evict: the scene is not resident");
  if (sc.running) return srv_fail(s, SJ_ESTATE, "evict: a tick of the scene is running");
  return evict_scene(s, sc);
}

int sj_server_retire(sj_server *s, uint32_t id) {
  if (!s || id >= s->scenes.size() || !s->scenes[id].live) return SJ_EINVAL;
  ServedScene &sc = s->scenes[id];
  if (sc.running || !sc.queue.empty()) return srv_fail(s, SJ_ESTATE, "retire: ticks pending");
  (void)hipStreamSynchronize(sc.stream);
  if (sc.resident) {
    sj_scene_destroy(sc.scene);
    s->pool.release(sc.mem, sc.mem_bytes);
  }
  (void)hipEventDestroy(sc.done);
  (void)hipStreamDestroy(sc.stream);
  (void)hipHostFree(sc.h_ctl);
  if (sc.snap) (void)hipHostFree(sc.snap);
  sc = ServedScene();
  return SJ_OK;
}

int sj_server_submit(sj_server *s, uint32_t id, const uint32_t *d_id, const float *d_x,
                     const float *d_y, uint32_t m, const uint32_t *d_qid, const float *d_xa,
                     const float *d_ya, const float *d_xb, const float *d_yb, uint32_t nq,
                     uint64_t tag, uint64_t *d_record, uint32_t flags) {
  if (!s || id >= s->scenes.size() || !s->scenes[id].live) return SJ_EINVAL;
  ServedScene &sc = s->scenes[id];
  if (m > sc.max_updates || nq > sc.max_queries)
    return srv_fail(s, SJ_EINVAL, "submit: more updates or queries than the scene admits");
  if ((m && (!d_id || !d_x || !d_y)) || (nq && (!d_qid || !d_xa || !d_ya || !d_xb || !d_yb)))
    return srv_fail(s, SJ_EINVAL, "submit: null input");
  const uintptr_t mis = (uintptr_t)d_id | (uintptr_t)d_x | (uintptr_t)d_y | (uintptr_t)d_qid |
                        (uintptr_t)d_xa | (uintptr_t)d_ya | (uintptr_t)d_xb | (uintptr_t)d_yb;
  if (mis & 3u) return srv_fail(s, SJ_EINVAL, "submit: misaligned input");
  if ((uintptr_t)d_record & 7u) return srv_fail(s, SJ_EINVAL, "submit: misaligned record");
  if (flags & ~(uint32_t)SJ_SERVE_DIGEST) return srv_fail(s, SJ_EINVAL, "submit: unknown flags");
  const bool digest = (flags & SJ_SERVE_DIGEST) != 0;
  sc.queue.push_back(
      Request{tag, d_record, digest, d_id, d_x, d_y, m, d_qid, d_xa, d_ya, d_xb, d_yb, nq});
  s->order.emplace_back(id, tag);
  return SJ_OK;
}

static int start_tick(sj_server *s, uint32_t id) {
  ServedScene &sc = s->scenes[id];
  Request r = sc.queue.front();
  sc.queue.pop_front();
  // the graph reads the request's arrays, which stay valid until the tick
  // is retired
  int rc = sj_tick_graph(sc.scene, r.id, r.x, r.y, r.m, r.qid, r.xa, r.ya, r.xb, r.yb, r.nq);
  const uint32_t b = sc.parity;
  if (rc == SJ_OK && r.digest) rc = sj_result_hashes(sc.scene, sc.o_cnt[b], sc.o_hash[b]);
  if (rc == SJ_OK) rc = sj_tick_counters(sc.scene, sc.o_counters[b]);
  if (rc == SJ_OK && r.record) {
    hipLaunchKernelGGL(k_record_init, dim3(1), dim3(1), 0, sc.stream,
                       (const uint64_t *)sc.o_counters[b], r.record);
    if (r.digest) {
      const unsigned g = (unsigned)((r.nq + 1023) / 1024 < 256 ? (r.nq + 1023) / 1024 : 256);
      hipLaunchKernelGGL(k_record_digest, dim3(g ? g : 1), dim3(256), 0, sc.stream,
                         (const uint64_t *)sc.o_cnt[b], (const uint64_t *)sc.o_hash[b], r.nq,
                         r.record);
    }
  }
  if (rc == SJ_OK) rc = sj_scene_ctl_to_host_async(sc.scene, sc.h_ctl);
  hipError_t e = hipEventRecord(sc.done, sc.stream);
  if (rc == SJ_OK && e != hipSuccess) rc = SJ_EDEVICE;
  sc.cur = r;
  sc.running = true;
  sc.status = rc;
  s->running += 1;
  return rc;
}

// Retires finished ticks (up to cap reported) and starts queued ones, in
// arrival order, admitting scenes that are not resident (and evicting the
// least recently used idle managed scenes to make room).
int sj_server_poll(sj_server *s, sj_served *done, uint32_t cap, uint32_t *n_done) {
  if (!s || !n_done) return SJ_EINVAL;
  *n_done = 0;
  const uint64_t poll = ++s->polls;
  for (uint32_t id = 0; id < s->scenes.size(); ++id) {
    ServedScene &sc = s->scenes[id];
    if (!sc.live || !sc.running) continue;
    if (*n_done >= cap) break;
    const hipError_t q = hipEventQuery(sc.done);
    if (q == hipErrorNotReady) continue;
    sc.running = false;
    s->running -= 1;
    sc.last_use = ++s->clock;
    sc.retired_poll = poll;
    int st = sc.status;
    if (q != hipSuccess) st = SJ_EDEVICE;
    if (st == SJ_OK) {
      sj_scene_ctl_from_host(sc.scene, sc.h_ctl);
      st = sj_scene_status(sc.scene);
    }
    sj_served &d = done[(*n_done)++];
    d.tag = sc.cur.tag;
    d.scene_id = id;
    d.status = st;
    d.nq = sc.cur.nq;
    d.d_count = sc.cur.digest ? sc.o_cnt[sc.parity] : nullptr;
    d.d_hash = sc.cur.digest ? sc.o_hash[sc.parity] : nullptr;
    d.d_counters = sc.o_counters[sc.parity];
    sc.parity ^= 1u;
  }
  // start queued requests in arrival order
  bool blocked = false;  // a scene earlier in the order waits for pool memory
  for (auto it = s->order.begin(); it != s->order.end() && s->running < s->max_running;) {
    const uint32_t id = it->first;
    ServedScene &sc = s->scenes[id];
    if (!sc.live) {
      it = s->order.erase(it);
      continue;
    }
    if (sc.running || sc.queue.empty() || sc.queue.front().tag != it->second) {
      ++it;
      continue;
    }
    if (!sc.resident) {
      if (blocked) {
        ++it;
        continue;
      }
      int rc = make_resident(s, sc);
      while (rc == SJ_ENOSPACE) {
        uint32_t victim = UINT32_MAX;
        for (uint32_t v = 0; v < s->scenes.size(); ++v) {
          const ServedScene &o = s->scenes[v];
          // a tick retired by this poll keeps its outputs for the caller
          if (v == id || !o.live || !o.resident || !o.managed || o.running || !o.queue.empty() ||
              o.retired_poll == poll)
            continue;
          if (victim == UINT32_MAX || o.last_use < s->scenes[victim].last_use) victim = v;
        }
        if (victim == UINT32_MAX) break;
        rc = evict_scene(s, s->scenes[victim]);
        if (rc != SJ_OK) return rc;
        rc = make_resident(s, sc);
      }
      if (rc == SJ_ENOSPACE) {
        blocked = true;
        ++it;
        continue;
      }
      if (rc != SJ_OK) return rc;
    }
    start_tick(s, id);
    it = s->order.erase(it);
  }
  return SJ_OK;
}

int sj_server_info(const sj_server *s, sj_server_stats *out) {
  if (!s || !out) return SJ_EINVAL;
  memset(out, 0, sizeof *out);
  out->pool_bytes = s->pool.size;
  out->pool_used = s->pool.used;
  out->running = s->running;
  uint32_t live = 0, queued = 0, resident = 0;
  for (const auto &sc : s->scenes) {
    if (!sc.live) continue;
    ++live;
    resident += sc.resident ? 1u : 0u;
    queued += (uint32_t)sc.queue.size();
  }
  out->scenes = live;
  out->queued = queued;
  out->resident = resident;
  out->admissions = s->admissions;
  out->evictions = s->evictions;
  return SJ_OK;
}

int sj_server_scene(sj_server *s, uint32_t id, sj_scene **out) {
  if (!s || !out || id >= s->scenes.size() || !s->scenes[id].live) return SJ_EINVAL;
  if (!s->scenes[id].resident) return srv_fail(s, SJ_ESTATE, "scene: not resident (evicted)");
  *out = s->scenes[id].scene;
  return SJ_OK;
}

const char *sj_server_last_error(const sj_server *s) { return s ? s->err : g_server_err; }

}  // extern "C"
