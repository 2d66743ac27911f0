"""Tick serving of many independent scenes on one GPU (continuous batching).

Each scene is a moving-object set with its own tick stream.  Tick requests
arrive as a Poisson process per scene.  A scene's memory comes from the
server's device pool (an HBM budget).  With eviction (the default), every
scene is registered up front and the server admits it when one of its
requests comes up, evicting idle scenes (their positions to host memory,
least recently used first) when the pool is full; a scene admitted again
gives the same results.  Without it, a scene is admitted when it fits and
keeps its memory until its last request is served.  Resident scenes' ticks
run on their own streams and overlap on the device (sj_server_*).

The latency of a tick request is its completion time minus its arrival time,
so it includes the waits for admission and for a running slot as well as
the processing.  These are the latency definitions of the paper's
"Quality of Service" section: latency = queueing + processing, and a tick's
latency is that of its slowest query.  All queries of a tick arrive with it.

    python -m paper_1411_3212_amd.serving [--scenes 16] [--requests 2000] ...
prints one JSON line with p50/p99 tick latency, ticks/s and pairs/s.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time
from collections import defaultdict, deque
from dataclasses import dataclass, field

import numpy as np

from . import workloads
from .binding import Scene, Server, make_config


@dataclass
class SceneSpec:
    index: int
    wl: workloads.Workload
    cfg: object
    max_updates: int
    ticks: list = field(default_factory=list)  # (packed device buffer, m, nq)


def scene_capacities(wl: workloads.Workload, th: int = 64, covering: bool = True) -> dict:
    """Per-tick capacities with headroom.  Without covering leaves every
    pair is written as an id, so the result capacity is four times larger."""
    kind = wl.params.get("kind", wl.name)
    rate = float(wl.params.get("query_rate", 0.1 if kind == "hotspot" else 0.5))
    q = max(1, int(round(rate * wl.n)))
    slots = 0  # the library's default list length
    if kind == "hotspot":  # denser hotspots hold more leaves and results per query
        per = dict(sub=48, cov=48, res=512) if wl.n <= 2_000_000 else \
            dict(sub=160, cov=160, res=2048)
        if wl.n > 2_000_000:
            slots = 64  # queries in the dense cores overlap more than 32 leaves
    else:
        per = dict(sub=16, cov=16, res=96)
    res = per["res"] * (1 if covering else 4)
    return dict(nq=q, th=th, capacity_subqueries=per["sub"] * q,
                capacity_covering=per["cov"] * q, capacity_results=res * q,
                split_slots=slots)


def make_specs(n_scenes: int = 16, seed: int = 5, nmin: float = 1e5, nmax: float = 8e6,
               th: int = 64) -> list:
    """Scene sizes log-uniform in [nmin, nmax]; even scenes use the hotspot
    generator, odd scenes the segment generator, seeded 500 + scene."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.floor(np.exp(rng.uniform(math.log(nmin), math.log(nmax), n_scenes))).astype(int)
    specs = []
    for s, n in enumerate(sizes):
        name = "hotspot" if s % 2 == 0 else "segments"
        wl = workloads.make(name, n=int(n), seed=500 + s)
        cap = scene_capacities(wl, th)
        cfg = make_config(int(n), cap["nq"], th=th, capacity_subqueries=cap["capacity_subqueries"],
                          capacity_covering=cap["capacity_covering"],
                          capacity_results=cap["capacity_results"])
        specs.append(SceneSpec(s, wl, cfg, int(n)))
    return specs


def pack_ticks(wl: workloads.Workload, torch) -> list:
    """Every tick of a workload in a packed device buffer [ids x y | qid xa
    ya xb yb] (4-byte words): a list of (buffer, updates, queries)."""
    out = []
    for t in wl.ticks():
        host = np.concatenate([t.ids.view(np.int32), t.x.view(np.int32), t.y.view(np.int32),
                               t.qid.view(np.int32), t.xa.view(np.int32), t.ya.view(np.int32),
                               t.xb.view(np.int32), t.yb.view(np.int32)])
        out.append((torch.from_numpy(host).cuda(), len(t.ids), t.nq))
    torch.cuda.synchronize()
    return out


def upload(specs: list, n_ticks: int, torch) -> None:
    """Generates n_ticks ticks per scene into packed device buffers."""
    for sp in specs:
        sp.wl.n_ticks = n_ticks
        sp.ticks = pack_ticks(sp.wl, torch)


def tick_views(buf, m, nq, torch):
    sizes = (m, m, m, nq, nq, nq, nq, nq)
    out, o = [], 0
    for i, n in enumerate(sizes):
        v = buf[o:o + n]
        out.append(v if i in (0, 3) else v.view(torch.float32))
        o += n
    return out


def poisson_requests(n_scenes: int, n_requests: int, rate_per_scene: float, n_ticks: int,
                     seed: int = 55) -> list:
    """(arrival s, scene, tick index) for n_requests requests: Poisson
    arrivals per scene; a scene's k-th request replays its tick k mod
    n_ticks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    per = [n_requests // n_scenes + (1 if s < n_requests % n_scenes else 0)
           for s in range(n_scenes)]
    reqs = []
    for s in range(n_scenes):
        t = np.cumsum(rng.exponential(1.0 / rate_per_scene, per[s]))
        reqs += [(float(t[k]), s, k % n_ticks) for k in range(per[s])]
    reqs.sort()
    return reqs


def serve(specs: list, requests: list, pool_bytes: int, max_running: int, torch,
          keep_arrays: bool = False, digest: bool = False, evict: bool = True) -> dict:
    """Runs the requests in real time through a server.  Returns latencies,
    per-request counters and, with digest (implied by keep_arrays),
    per-request digests (sum of per-query pair-set hashes mod 2^64, pair
    count) and, with keep_arrays, the per-query count and hash arrays.  The
    digest reads every result, so it is for checking runs.  evict: scenes
    are admitted on demand and evicted when idle (sj_server_add); else each
    is admitted when it fits and retired after its last request."""
    digest = digest or keep_arrays
    srv = Server(pool_bytes, max_running)
    for s_ in {s for _, s, _ in requests}:
        need = srv.scene_bytes(specs[s_].cfg, specs[s_].max_updates)
        if need > srv.pool.numel():
            srv.close()
            raise ValueError(f"scene {s_} needs {need} bytes, more than the whole pool")
    n_req = len(requests)
    remaining = defaultdict(int)
    for _, s, _ in requests:
        remaining[s] += 1
    waiting = []  # scenes with requests but not admitted, in order of first arrival
    sid_of, scene_of = {}, {}
    pending = defaultdict(deque)
    arrival, lat = {}, {}
    arrays = {}
    admitted_at, retired_at = {}, {}
    nxt, done = 0, 0
    history = torch.zeros((max(n_req, 1), 16), dtype=torch.int64, device="cuda")
    if evict:  # every scene registered; the server admits and evicts
        for s_ in sorted(remaining):
            sid_of[s_] = srv.add(specs[s_].cfg, specs[s_].max_updates)
            scene_of[sid_of[s_]] = s_
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while done < n_req:
        now = time.perf_counter() - t0
        while nxt < n_req and requests[nxt][0] <= now:
            ta, s, k = requests[nxt]
            arrival[nxt] = ta
            pending[s].append((nxt, k))
            if s not in sid_of and s not in waiting:
                waiting.append(s)
            nxt += 1
        for s in list(waiting):
            sid = srv.admit(specs[s].cfg, specs[s].max_updates)
            if sid is None:
                continue
            waiting.remove(s)
            sid_of[s] = sid
            scene_of[sid] = s
            admitted_at[s] = time.perf_counter() - t0
        for s, dq in pending.items():
            if s not in sid_of:
                continue
            while dq:
                tag, k = dq.popleft()
                buf, m, nq = specs[s].ticks[k]
                srv.submit(sid_of[s], tag, *tick_views(buf, m, nq, torch), record=history[tag],
                           digest=digest)
        fin = srv.poll()
        tnow = time.perf_counter() - t0
        for sid, tag, status, nq, pc, ph, pk in fin:
            assert status == 0, f"tick {tag} of scene {scene_of[sid]} failed: {status}"
            s = scene_of[sid]
            lat[tag] = tnow - arrival[tag]
            if keep_arrays:  # synchronous copies: tests only
                off = srv.pool.data_ptr()
                cnt = srv.pool[pc - off:pc - off + 8 * nq].view(torch.int64)
                hsh = srv.pool[ph - off:ph - off + 8 * nq].view(torch.int64)
                arrays[tag] = (cnt.cpu().numpy().view(np.uint64), hsh.cpu().numpy().view(np.uint64))
            done += 1
            remaining[s] -= 1
            if remaining[s] == 0 and not evict:
                srv.retire(sid)
                del sid_of[s]
                retired_at[s] = time.perf_counter() - t0
        if not fin and nxt < n_req and srv.info()["running"] == 0 and not any(pending.values()):
            time.sleep(max(0.0, min(requests[nxt][0] - (time.perf_counter() - t0), 0.001)))
    makespan = time.perf_counter() - t0
    torch.cuda.synchronize()
    info = srv.info()
    hist = history.cpu().numpy().view(np.uint64)
    ctr = {t: tuple(int(v) for v in hist[t, :8]) for t in range(n_req)}
    dig = {t: (int(hist[t, 8]), int(hist[t, 9])) for t in range(n_req)}
    srv.close()
    lats = np.array([lat[t] for t in range(n_req)]) * 1e3
    pairs = sum(c[0] for c in ctr.values())
    return dict(latency_ms=lats, counters=ctr, digest=dig, arrays=arrays, makespan_s=makespan,
                pairs=pairs, admitted_at=admitted_at, retired_at=retired_at,
                admissions=info["admissions"], evictions=info["evictions"])


def serve_alone(spec: SceneSpec, tick_seq: list, torch, keep_arrays: bool = False) -> list:
    """The same ticks of one scene, alone, through a plain Scene and the
    graph path: [(digest, arrays)] per tick of tick_seq."""
    cap = spec.cfg
    sc = Scene(cap.capacity_objects, cap.capacity_queries, th=cap.th_quad,
               capacity_subqueries=cap.capacity_subqueries,
               capacity_covering=cap.capacity_covering, capacity_results=cap.capacity_results)
    out = []
    for k in tick_seq:
        buf, m, nq = spec.ticks[k]
        sc.tick_graph(*tick_views(buf, m, nq, torch))
        cnt, h = sc.hashes()
        d = (int(h.sum().item()) & (2**64 - 1), int(cnt.sum().item()))
        a = (cnt.cpu().numpy().view(np.uint64), h.cpu().numpy().view(np.uint64)) if keep_arrays else None
        out.append((d, a))
    sc.close()
    return out


def solo_service_ms(specs: list, torch, reps: int = 3) -> list:
    """Median time of one tick of each scene run alone (graph path, synchronised)."""
    res = []
    for sp in specs:
        cap = sp.cfg
        sc = Scene(cap.capacity_objects, cap.capacity_queries, th=cap.th_quad,
                   capacity_subqueries=cap.capacity_subqueries,
                   capacity_covering=cap.capacity_covering, capacity_results=cap.capacity_results)
        prep = [sc.prepare_tick(*tick_views(buf, m, nq, torch)) for buf, m, nq in sp.ticks]
        ts = []
        for r in range(reps + 2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sc.tick_graph(prep[r % len(sp.ticks)])
            sc.fetch()
            ts.append(time.perf_counter() - t0)
        res.append(float(np.median(ts[2:])) * 1e3)
        sc.close()
    return res


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--scenes", type=int, default=16)
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--ticks", type=int, default=4, help="distinct ticks generated per scene")
    ap.add_argument("--nmin", type=float, default=1e5)
    ap.add_argument("--nmax", type=float, default=8e6)
    ap.add_argument("--load", type=float, default=0.7, help="offered load / solo capacity")
    ap.add_argument("--budget-frac", type=float, default=0.5,
                    help="pool = this fraction of the free HBM (capped at --budget-gib)")
    ap.add_argument("--budget-gib", type=float, default=0.0)
    ap.add_argument("--max-running", type=int, default=4)
    ap.add_argument("--digest", action="store_true",
                    help="also hash every tick's result set (a checking run: reads all results)")
    ap.add_argument("--no-evict", action="store_true",
                    help="admit a scene when it fits and keep it until its last request")
    args = ap.parse_args(argv)
    import torch
    specs = make_specs(args.scenes, nmin=args.nmin, nmax=args.nmax)
    t = time.perf_counter()
    upload(specs, args.ticks, torch)
    gen_s = time.perf_counter() - t
    solo = solo_service_ms(specs, torch)
    cap_ticks_s = 1e3 / float(np.mean(solo))
    rate = args.load * cap_ticks_s / args.scenes
    reqs = poisson_requests(args.scenes, args.requests, rate, args.ticks)
    free, _ = torch.cuda.mem_get_info()
    pool = int(args.budget_frac * free)
    if args.budget_gib:
        pool = min(pool, int(args.budget_gib * 2**30))
    srv_probe = Server(1 << 20)
    need = [srv_probe.scene_bytes(sp.cfg, sp.max_updates) for sp in specs]
    srv_probe.close()
    r = serve(specs, reqs, pool, args.max_running, torch, digest=args.digest,
              evict=not args.no_evict)
    lat = r["latency_ms"]
    out = {
        "metric": "tick serving: p50/p99 tick latency, ticks/s, result pairs/s",
        "scenes": args.scenes, "requests": len(reqs),
        "objects": [sp.wl.n for sp in specs],
        "offered_ticks_per_s": rate * args.scenes, "solo_tick_ms": solo,
        "p50_tick_ms": float(np.percentile(lat, 50)), "p99_tick_ms": float(np.percentile(lat, 99)),
        "mean_tick_ms": float(lat.mean()),
        "ticks_per_s": len(reqs) / r["makespan_s"], "pairs_per_s": r["pairs"] / r["makespan_s"],
        "pool_gib": pool / 2**30, "scene_gib_total": sum(need) / 2**30,
        "max_running": args.max_running, "digest": args.digest, "generation_s": gen_s,
        "evict": not args.no_evict, "admissions": r["admissions"], "evictions": r["evictions"],
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
