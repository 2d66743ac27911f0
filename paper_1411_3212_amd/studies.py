"""The paper's design studies, measured on this implementation (one GPU).

``s1``   lock-free join (count, scan, write) against the baseline filter
         that appends results through atomics (UG_Baseline, Algorithm SQB),
         on the uniform grid and on the quadtree (study S1).
``s3``   heaviest-first task order on and off, with the per-CU imbalance of
         the filtering pass: (max - min) / max of the containment tests done
         by each compute unit, averaged over ticks (study S3).
``s4``   uniform-grid split-factor sweep: per-phase device times, subqueries
         and tick time for every split factor, beside the quadtree (study S4).

Every configuration runs the same ticks; the per-query result sizes and
pair-set hashes of every tick are compared with the first configuration's.

    python -m paper_1411_3212_amd.studies s4 --workload hotspot --splits 50,95,110,150,300
prints one JSON line per study.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import workloads
from .binding import PHASES, Scene


def _capacities(wl, th=64):
    from .serving import scene_capacities
    c = scene_capacities(wl, th)
    c.pop("nq")
    return c


def _ticks(wl, torch):
    out = []
    for t in wl.ticks():
        f = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a).view(dt)).cuda()
        out.append((f(t.ids, np.int32), f(t.x, np.float32), f(t.y, np.float32),
                    f(t.qid, np.int32), f(t.xa, np.float32), f(t.ya, np.float32),
                    f(t.xb, np.float32), f(t.yb, np.float32)))
    torch.cuda.synchronize()
    return out


def run_config(wl, ticks, nq, torch, warm=2, cu=False, **kw):
    """Eager ticks on a profiled scene: per-phase device times and counters
    averaged over the timed ticks, wall time per tick, per-query hashes of
    every timed tick, and (cu) the per-CU imbalance."""
    cap = _capacities(wl, kw.get("th", 64))
    cap.update(kw)
    sc = Scene(wl.n, nq, profile=True, cu_counters=cu, **cap)
    ph = {k: 0.0 for k in PHASES}
    wall, hashes, imb, stats = 0.0, [], [], []
    n = 0
    for i, t in enumerate(ticks):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sc.apply_updates(t[0], t[1], t[2])
        sc.run_tick(*t[3:])
        sc.fetch()
        dt = time.perf_counter() - t0
        if i < warm:
            continue
        n += 1
        wall += dt
        p = sc.phase_times()
        for k in PHASES:
            ph[k] += p[k]
        s = sc.stats()
        stats.append({k: s[k] for k in ("n_isect", "n_cov", "n_isect_ids", "cov_pairs", "tests",
                                         "n_tasks", "n_leaves")})
        if cu:
            c = sc.cu_counters()
            c = c[c > 0].astype(np.float64)
            imb.append(float((c.max() - c.min()) / c.max()) if len(c) else 0.0)
        cnt, h = sc.hashes()
        hashes.append((cnt.clone(), h.clone()))
    sc.close()
    out = {"ms_per_tick": 1e3 * wall / n,
           "phase_ms": {k: round(v / n, 4) for k, v in ph.items()},
           "device_ms": round(sum(ph.values()) / n, 4)}
    for k in stats[0]:
        out[k] = float(np.mean([s[k] for s in stats]))
    if cu:
        out["cu_imbalance"] = float(np.mean(imb))
    return out, hashes


def _same(a, b, torch):
    return all(torch.equal(x[0], y[0]) and torch.equal(x[1], y[1]) for x, y in zip(a, b))


def study(name, configs, wl_name, n_ticks, torch, n=None, cu=False):
    wl = workloads.make(wl_name, n_ticks=n_ticks, **({"n": n} if n else {}))
    ticks = _ticks(wl, torch)
    nq = max(int(t[3].numel()) for t in ticks)
    res, ref = {}, None
    for label, kw in configs:
        r, h = run_config(wl, ticks, nq, torch, cu=cu, **kw)
        if ref is None:
            ref = h
        r["identical_results"] = _same(ref, h, torch)
        res[label] = r
        print(json.dumps({"study": name, "config": label, **r}), flush=True)
    return {"study": name, "workload": wl_name, "objects": wl.n, "queries_per_tick": nq,
            "ticks": n_ticks, "results": res}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("study", choices=["s1", "s3", "s4"])
    ap.add_argument("--workload", default="hotspot", choices=sorted(workloads.WORKLOADS))
    ap.add_argument("--n", type=int, default=0, help="objects (default: the workload's)")
    ap.add_argument("--ticks", type=int, default=6)
    ap.add_argument("--th", type=int, default=64)
    ap.add_argument("--splits", default="25,50,75,95,110,150,200,300")
    ap.add_argument("--grid", type=int, default=110, help="split factor of s1's uniform grid")
    args = ap.parse_args(argv)
    import torch
    th = args.th
    if args.study == "s1":
        configs = [("UG lock-free", dict(grid_split=args.grid)),
                   ("UG baseline (atomics)", dict(grid_split=args.grid, atomic_results=True)),
                   (f"QUAD th {th} lock-free", dict(th=th)),
                   (f"QUAD th {th} baseline (atomics)", dict(th=th, atomic_results=True))]
        out = study("s1", configs, args.workload, args.ticks, torch, args.n or None)
    elif args.study == "s3":
        configs = [(f"QUAD th {th} reorder", dict(th=th)),
                   (f"QUAD th {th} no reorder", dict(th=th, reorder=False)),
                   (f"UG {args.grid} reorder", dict(grid_split=args.grid)),
                   (f"UG {args.grid} no reorder", dict(grid_split=args.grid, reorder=False))]
        out = study("s3", configs, args.workload, args.ticks, torch, args.n or None, cu=True)
    else:
        configs = [(f"QUAD th {th}", dict(th=th))]
        configs += [(f"UG {s}", dict(grid_split=int(s))) for s in args.splits.split(",")]
        out = study("s4", configs, args.workload, args.ticks, torch, args.n or None)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
