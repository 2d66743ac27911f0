"""Learned cost model of the leaf threshold: data, training and evaluation.

The paper fixes the leaf threshold th_quad by hand after a sweep
(Experimental evaluation, S5).  Here a small network predicts the join time
of a quadtree leaf from (log2(1 + objects), log2(1 + intersecting
subqueries), level / 16, mean overlap of the subqueries with the leaf), and
the library's threshold tuner (SJ_THRESH_MLP) adds terms linear in the
subqueries and leaves (the complexity terms of the Computational Complexity
section) to choose the cheapest candidate threshold when it builds.

    python -m paper_1411_3212_amd.costmodel train [--out FILE]
        logs per-leaf join timings (SJ_TIMING_LOG) of hotspot (1M objects)
        and segment (4M objects) ticks at every candidate threshold, trains
        the network on the GPU with the library's forward, gradient and Adam
        kernels, fits the linear terms on the measured tick phases, and
        writes the model as JSON.
    python -m paper_1411_3212_amd.costmodel compare [--workload NAME]
        runs the same ticks with the fixed threshold and with the learned
        one (graph launches) and prints ticks/s, p50/p99 tick latency and
        whether every tick's result set is the same.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import sys
import time
from pathlib import Path

import numpy as np

from . import binding, serving, workloads
from .binding import PHASES, Scene

CAND = (32, 64, 128, 256, 384, 512, 768, 1024)
MODEL_PATH = Path(__file__).resolve().parent / "data" / "cost_model.json"
# tick phases whose time depends on the threshold (the sort of the ticks
# that keep the tree through its leaf keys; the build is amortised over the
# rebuild period and left out)
COST_PHASES = ("index", "leaves", "split", "schedule", "join_count", "join_scan", "join_write")
TRAIN_SETS = (("hotspot", 20), ("segments", 20))  # 2 x 8 thresholds x 17 logged ticks


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def leaf_samples(rec: np.ndarray, mhz: float):
    """Features and measured join time (microseconds, count + write pass) of
    the active leaves of one tick's timing log (rows of 8 floats)."""
    cnt, nsq = rec[:, 0], rec[:, 1]
    a = (cnt > 0) & (nsq > 0)
    X = np.stack([np.log2(np.float32(1) + cnt[a]), np.log2(np.float32(1) + nsq[a]),
                  rec[a, 2] * np.float32(1 / 16), rec[a, 3]], axis=1).astype(np.float32)
    us = (rec[a, 4].astype(np.float64) + rec[a, 5]) / mhz
    return X, us


def sort_passes(n_leaves: int) -> int:
    """Radix passes of the leaf-keyed sort (8-bit digits, keys below n_leaves)."""
    return (int(n_leaves - 1).bit_length() + 7) // 8 if n_leaves > 1 else 0


def collect(name: str, n_ticks: int, cand=CAND, warm: int = 3, torch=None, log=print) -> list:
    """One record per logged tick of every candidate threshold: features and
    measured leaf times from a scene with the timing log, counts and phase
    times (eager, profiled) from a twin scene without it, since logging
    slows the join."""
    wl = workloads.make(name, n_ticks=n_ticks)
    ticks = serving.pack_ticks(wl, torch)
    caps = serving.scene_capacities(wl)
    nq = max(q for _, _, q in ticks)
    rows = []
    kw = {k: caps[k] for k in ("capacity_subqueries", "capacity_covering", "capacity_results",
                               "split_slots")}
    for th in cand:
        logged = Scene(wl.n, nq, th=th, timing_log=True, **kw)
        plain = Scene(wl.n, nq, th=th, profile=True, **kw)
        for i, (buf, m, q) in enumerate(ticks):
            ids, x, y, qid, xa, ya, xb, yb = serving.tick_views(buf, m, q, torch)
            for sc in (logged, plain):
                sc.apply_updates(ids, x, y)
                sc.run_tick(qid, xa, ya, xb, yb)
            s = plain.stats()
            logged.stats()
            if i < warm:
                continue
            rec, mhz = logged.timing_log()
            X, us = leaf_samples(rec.cpu().numpy(), mhz)
            ph = plain.phase_times()
            rows.append(dict(wl=name, th=th, tick=i, X=X, us=us, n_isect=s["n_isect"],
                             n_cov=s["n_cov"], n_leaves=s["n_leaves"], n_present=s["n_present"],
                             rebuilt=s["rebuilt"], phase_ms={k: ph[k] for k in PHASES}))
        log(f"collected {name} th={th}: {len(ticks) - warm} ticks, "
            f"{sum(len(r['us']) for r in rows if r['th'] == th and r['wl'] == name)} leaves")
        logged.close()
        plain.close()
        del logged, plain
    del ticks
    torch.cuda.empty_cache()
    return rows


def init_params(seed: int) -> np.ndarray:
    """He initialisation of the FP32 master parameters (biases zero)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = np.zeros(4545, np.float32)
    p[0:256] = rng.normal(0, math.sqrt(2 / 4), 256)        # W1
    p[320:4416] = rng.normal(0, math.sqrt(2 / 64), 4096)   # W2
    p[4480:4544] = rng.normal(0, math.sqrt(1 / 64), 64)    # w3
    return p


class Trainer:
    """FP32 master parameters, Adam moments and the BF16 copy on the device;
    every step runs the library's gradient and Adam kernels."""

    def __init__(self, torch, seed: int = 0, batch: int = 65536):
        self.torch, self.lib = torch, binding.load()
        self.P = int(self.lib.sj_mlp_param_count())
        dev = "cuda"
        self.master = torch.from_numpy(init_params(seed)).to(dev)
        self.m = torch.zeros(self.P, device=dev)
        self.v = torch.zeros(self.P, device=dev)
        self.w = torch.empty(self.P, dtype=torch.int16, device=dev)
        self.g = torch.empty(self.P + 1, device=dev)
        self.nb = int(self.lib.sj_mlp_scratch_bytes(batch))
        self.scratch = torch.empty(self.nb, dtype=torch.uint8, device=dev)
        self.stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        self.steps = 0
        self._ok(self.lib.sj_mlp_round(_ptr(self.master), _ptr(self.w), self.stream))

    def _ok(self, rc):
        if rc != 0:
            raise RuntimeError(f"MLP call failed ({rc}): {self.lib.sj_last_error(None).decode()}")

    def step(self, X, T, lr: float) -> None:
        n = X.shape[0]
        self.steps += 1
        self._ok(self.lib.sj_mlp_grad(_ptr(self.w), _ptr(X), _ptr(T), n, _ptr(self.g),
                                      _ptr(self.scratch), self.nb, self.stream))
        self._ok(self.lib.sj_mlp_adam(_ptr(self.master), _ptr(self.g), _ptr(self.m), _ptr(self.v),
                                      _ptr(self.w), self.steps, ctypes.c_float(lr), self.stream))

    def loss(self, X, T) -> float:
        """Mean squared error of the current BF16 network on (X, T)."""
        self._ok(self.lib.sj_mlp_grad(_ptr(self.w), _ptr(X), _ptr(T), X.shape[0], _ptr(self.g),
                                      _ptr(self.scratch), self.nb, self.stream))
        return float(self.g[-1].item())

    def predict(self, X):
        y = self.torch.empty(X.shape[0], dtype=self.torch.float32, device="cuda")
        if X.shape[0]:
            self._ok(self.lib.sj_mlp_forward(_ptr(self.w), _ptr(X), X.shape[0], _ptr(y),
                                             self.stream))
        return y

    def bits(self) -> np.ndarray:
        return self.w.cpu().numpy().view(np.uint16).copy()


def train(rows: list, torch, steps: int = 3000, batch: int = 65536, lr: float = 3e-3,
          max_samples: int = 2_000_000, seed: int = 0, log=print) -> tuple:
    """Trains on the rows' leaves (ticks with index % 6 == 5 held out):
    minibatch Adam on ln(microseconds), cosine learning-rate decay."""
    rng = np.random.Generator(np.random.PCG64(seed))
    val = [r for r in rows if r["tick"] % 6 == 5]
    trn = [r for r in rows if r["tick"] % 6 != 5]

    def stack(rs):
        X = np.concatenate([r["X"] for r in rs])
        T = np.log(np.maximum(np.concatenate([r["us"] for r in rs]), 0.02)).astype(np.float32)
        return X, T

    Xt, Tt = stack(trn)
    Xv, Tv = stack(val)
    if len(Tt) > max_samples:
        pick = rng.choice(len(Tt), max_samples, replace=False)
        Xt, Tt = Xt[pick], Tt[pick]
    tr = Trainer(torch, seed=seed, batch=batch)
    dXv, dTv = torch.from_numpy(Xv).cuda(), torch.from_numpy(Tv).cuda()
    n = len(Tt)
    nbatch = max(1, n // batch)
    t0 = time.perf_counter()
    k = 0
    history = []
    while k < steps:
        perm = rng.permutation(n)
        dX = torch.from_numpy(Xt[perm]).cuda()
        dT = torch.from_numpy(Tt[perm]).cuda()
        for b in range(nbatch):
            if k >= steps:
                break
            lo, hi = b * batch, min(n, (b + 1) * batch)
            cur = lr * (0.02 + 0.98 * 0.5 * (1 + math.cos(math.pi * k / steps)))
            tr.step(dX[lo:hi], dT[lo:hi], cur)
            k += 1
            if k % 500 == 0 or k == steps:
                history.append((k, tr.loss(dXv, dTv)))
                log(f"step {k}: validation MSE {history[-1][1]:.4f}")
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    yv = tr.predict(dXv).cpu().numpy().astype(np.float64)
    res = yv - Tv
    stats = dict(train_samples=int(n), val_samples=int(len(Tv)), steps=steps, batch=batch,
                 seconds=round(secs, 2), val_mse=float(np.mean(res ** 2)),
                 val_r2=float(1 - np.mean(res ** 2) / np.var(Tv)),
                 val_median_abs_ln_error=float(np.median(np.abs(res))), history=history)
    return tr, stats


def fit_terms(rows: list, tr: Trainer, torch) -> tuple:
    """Non-negative least squares of the threshold-dependent phase time of a
    tick (microseconds) on [sum exp(prediction), |Q_I|, |Q_C|, leaves,
    max exp(prediction for one task), sort passes x objects] plus one
    intercept per workload (constants do not move the argmin).  The sum is
    the join's work, the maximum its critical path (one wave per task, at
    most 64 subqueries); a linear fit of both stands for the makespan."""
    from scipy.optimize import nnls
    names = sorted({r["wl"] for r in rows})
    A, b = [], []
    for r in rows:
        X = r["X"]
        y = tr.predict(torch.from_numpy(X).cuda()).cpu().numpy().astype(np.float64)
        Xc = X.copy()
        Xc[:, 1] = np.minimum(Xc[:, 1], np.float32(np.log2(65.0)))
        yc = tr.predict(torch.from_numpy(Xc).cuda()).cpu().numpy().astype(np.float64)
        r["msum"] = float(np.exp(y).sum()) if len(y) else 0.0
        r["mmax"] = float(np.exp(yc).max()) if len(yc) else 0.0
        A.append([r["msum"], r["n_isect"], r["n_cov"], r["n_leaves"], r["mmax"],
                  sort_passes(r["n_leaves"]) * r["n_present"]] +
                 [1.0 if r["wl"] == nm else 0.0 for nm in names])
        b.append(1e3 * sum(r["phase_ms"][k] for k in COST_PHASES))
    A, b = np.array(A), np.array(b)
    scale = np.maximum(np.abs(A).max(axis=0), 1e-30)
    x, _ = nnls(A / scale, b)
    x = x / scale
    pred = A @ x
    r2 = float(1 - np.sum((b - pred) ** 2) / np.sum((b - b.mean()) ** 2))
    # per workload: measured mean time per threshold and the threshold the
    # fitted cost picks on average
    per = {}
    for nm in names:
        meas, cost = {}, {}
        for th in sorted({r["th"] for r in rows}):
            sel = [i for i, r in enumerate(rows) if r["wl"] == nm and r["th"] == th]
            meas[th] = float(b[sel].mean())
            cost[th] = float((A[sel, :6] @ x[:6]).mean())
        per[nm] = dict(measured_us=meas, predicted_us=cost,
                       best_measured=min(meas, key=meas.get), best_predicted=min(cost, key=cost.get))
    return [float(v) for v in x[:6]], dict(r2=r2, intercepts=dict(zip(names, map(float, x[6:]))),
                                           per_workload=per)


def save(path: Path, bits: np.ndarray, coef, cand, info: dict) -> None:
    path.parent.mkdir(parents=True, exist_ok=True)
    doc = dict(format=1, params_bf16=[int(v) for v in bits], coef=list(coef), cand=list(cand),
               features="log2(1+objects), log2(1+intersecting subqueries), level/16, "
                        "mean overlap fraction of the subqueries with the leaf",
               target="ln microseconds of the leaf's join (count + write pass, one wave)",
               cost="coef0*sum exp(mlp) + coef1*|Q_I| + coef2*|Q_C| + coef3*leaves "
                    "+ coef4*max exp(mlp of one task) + coef5*sort passes*objects "
                    "(microseconds of the threshold-dependent tick phases)",
               training=info)
    path.write_text(json.dumps(doc, indent=1) + "\n")


def load(path: Path = MODEL_PATH) -> dict:
    doc = json.loads(Path(path).read_text())
    bits = np.array(doc["params_bf16"], np.uint16)
    if len(bits) != 4545:
        raise ValueError(f"{path}: expected 4545 parameters, found {len(bits)}")
    return dict(bits=bits, coef=[float(v) for v in doc["coef"]],
                cand=[int(v) for v in doc["cand"]], doc=doc)


def install(scene: Scene, model: dict, torch) -> None:
    w = torch.from_numpy(model["bits"].view(np.int16).copy()).cuda()
    scene.set_cost_model(w, model["coef"], model["cand"])


def run_ticks(scene: Scene, ticks: list, torch, warm: int, hashes: bool = True) -> dict:
    """Graph-launched ticks; per-tick latency (launch to results on the host)
    of the ticks after warm, and each tick's (count, hash) per query.  The
    first tick (the build, its tuning and the graph capture) is reported
    apart."""
    prep = [scene.prepare_tick(*serving.tick_views(buf, m, q, torch)) for buf, m, q in ticks]
    lat, pairs, digests, ths = [], 0, [], []
    torch.cuda.synchronize()
    first = None
    for i, (buf, m, q) in enumerate(ticks):
        h0 = time.perf_counter()
        scene.tick_graph(prep[i])
        r = scene.fetch()
        h1 = time.perf_counter()
        if i == 0:
            first = (h1 - h0) * 1e3
        if i >= warm:
            lat.append((h1 - h0) * 1e3)
            pairs += r.total_pairs
        s = scene.stats()
        ths.append(s["th"])
        if hashes:
            c, h = scene.hashes()
            digests.append((c.cpu().numpy().tobytes(), h.cpu().numpy().tobytes()))
    wall = 1e-3 * sum(lat)  # ticks run back to back; checks between them are not counted
    k = len(ticks) - warm
    return dict(ticks_per_s=k / wall, ms_per_tick=1e3 * wall / k, first_tick_ms=first,
                p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                pairs_per_s=pairs / wall, th=ths, digests=digests)


def compare(name: str, n_ticks: int, warm: int, torch, model: dict, th_fixed: int = 64,
            tune_every: int = 0, schedule: bool = False, log=print, **overrides) -> dict:
    """The same ticks with the fixed threshold and with the learned one (and,
    with schedule, the learned threshold plus the learned task order)."""
    wl = workloads.make(name, n_ticks=n_ticks, **overrides)
    ticks = serving.pack_ticks(wl, torch)
    caps = serving.scene_capacities(wl)
    nq = max(q for _, _, q in ticks)
    kw = dict(capacity_subqueries=caps["capacity_subqueries"],
              capacity_covering=caps["capacity_covering"],
              capacity_results=caps["capacity_results"], split_slots=caps["split_slots"])
    out = dict(workload=name, objects=wl.n, queries_per_tick=nq, ticks=n_ticks - warm)
    fixed = Scene(wl.n, nq, th=th_fixed, **kw)
    out["fixed"] = run_ticks(fixed, ticks, torch, warm)
    fixed.close()
    del fixed
    torch.cuda.empty_cache()
    log(f"{name}: fixed th={th_fixed} {out['fixed']['ms_per_tick']:.3f} ms/tick")
    learned = Scene(wl.n, nq, th=th_fixed, th_min=min(model["cand"]), thresh_mlp=True,
                    tune_every=tune_every, **kw)
    install(learned, model, torch)
    out["learned"] = run_ticks(learned, ticks, torch, warm)
    info = learned.tune_info()
    learned.close()
    del learned
    log(f"{name}: learned {out['learned']['ms_per_tick']:.3f} ms/tick, th {sorted(set(out['learned']['th']))}")
    if schedule:
        sch = Scene(wl.n, nq, th=th_fixed, th_min=min(model["cand"]), thresh_mlp=True,
                    schedule_mlp=True, tune_every=tune_every, **kw)
        install(sch, model, torch)
        out["learned_schedule"] = run_ticks(sch, ticks, torch, warm)
        sch.close()
        del sch
        d = out["learned_schedule"].pop("digests")
        out["learned_schedule"]["th"] = sorted(set(out["learned_schedule"]["th"]))
        out["learned_schedule"]["identical_results"] = d == out["fixed"]["digests"]
        out["learned_schedule"]["speedup_ticks_per_s"] = (
            out["learned_schedule"]["ticks_per_s"] / out["fixed"]["ticks_per_s"])
        log(f"{name}: learned threshold + schedule "
            f"{out['learned_schedule']['ms_per_tick']:.3f} ms/tick")
    out["identical_results"] = out["fixed"].pop("digests") == out["learned"].pop("digests")
    out["fixed"]["th"] = sorted(set(out["fixed"]["th"]))
    out["learned"]["th"] = sorted(set(out["learned"]["th"]))
    out["learned"]["tunings"] = info["n_tunes"]
    out["learned"]["last_costs"] = dict(zip(info["cand"], info["cost"]))
    out["speedup_ticks_per_s"] = out["learned"]["ticks_per_s"] / out["fixed"]["ticks_per_s"]
    out["p99_ratio"] = out["learned"]["p99_ms"] / out["fixed"]["p99_ms"]
    del ticks
    torch.cuda.empty_cache()
    return out


def mix(torch, model: dict, fixed=(64, 128, 256, 384), n_ticks: int = 6, warm: int = 2,
        n_scenes: int = 16, log=print) -> dict:
    """The serving mix's scenes (16 scenes of 1e5-8e6 objects, hotspot and
    segment workloads) each run alone on the same ticks with every fixed
    threshold and with the learned one: the total time of all scenes' ticks
    per configuration, identical per-query results required.  One fixed
    threshold has to serve every scene; the learned one is chosen per scene."""
    specs = serving.make_specs(n_scenes)
    tot = {f"fixed {t}": 0.0 for t in fixed}
    tot["learned"] = 0.0
    per_scene, same = [], True
    for sp in specs:
        sp.wl.n_ticks = n_ticks
        ticks = serving.pack_ticks(sp.wl, torch)
        caps = serving.scene_capacities(sp.wl)
        nq = max(q for _, _, q in ticks)
        kw = dict(capacity_subqueries=caps["capacity_subqueries"],
                  capacity_covering=caps["capacity_covering"],
                  capacity_results=caps["capacity_results"], split_slots=caps["split_slots"])
        row, ref = {"objects": sp.wl.n, "kind": sp.wl.params.get("kind")}, None
        for label, th in [(f"fixed {t}", t) for t in fixed] + [("learned", None)]:
            if th is None:
                sc = Scene(sp.wl.n, nq, th=64, th_min=min(model["cand"]), thresh_mlp=True, **kw)
                install(sc, model, torch)
            else:
                sc = Scene(sp.wl.n, nq, th=th, th_min=min(th, 64), **kw)
            r = run_ticks(sc, ticks, torch, warm)
            if th is None:
                row["learned_th"] = sorted(set(r["th"]))
            sc.close()
            d = r.pop("digests")
            same = same and (ref is None or d == ref)
            ref = d if ref is None else ref
            row[label] = r["ms_per_tick"]
            tot[label] += r["ms_per_tick"]
        per_scene.append(row)
        log(json.dumps(row))
        del ticks
        torch.cuda.empty_cache()
    best_fixed = min((v, k) for k, v in tot.items() if k != "learned")
    return dict(total_ms_per_round=tot, best_fixed=best_fixed[1],
                learned_vs_best_fixed=best_fixed[0] / tot["learned"], identical_results=same,
                scenes=per_scene)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--out", default=str(MODEL_PATH))
    t.add_argument("--steps", type=int, default=3000)
    t.add_argument("--seed", type=int, default=0)
    c = sub.add_parser("compare")
    c.add_argument("--workload", default="hotspot", choices=sorted(workloads.WORKLOADS))
    c.add_argument("--ticks", type=int, default=60)
    c.add_argument("--warmup", type=int, default=8)
    c.add_argument("--model", default=str(MODEL_PATH))
    c.add_argument("--schedule", action="store_true",
                   help="also run the learned threshold with the learned task order")
    m = sub.add_parser("mix", help="the serving mix's scenes alone: learned vs fixed thresholds")
    m.add_argument("--fixed", default="64,128,256,384")
    m.add_argument("--ticks", type=int, default=6)
    m.add_argument("--scenes", type=int, default=16)
    m.add_argument("--model", default=str(MODEL_PATH))
    args = ap.parse_args(argv)
    import torch
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    if args.cmd == "train":
        rows = []
        for name, n in TRAIN_SETS:
            rows += collect(name, n, torch=torch, log=log)
        tr, stats = train(rows, torch, steps=args.steps, seed=args.seed, log=log)
        coef, fit = fit_terms(rows, tr, torch)
        info = dict(logged_ticks=len(rows), sets=[f"{n}:{k}" for n, k in TRAIN_SETS],
                    network=stats, terms=fit)
        save(Path(args.out), tr.bits(), coef, CAND, info)
        print(json.dumps(dict(coef=coef, logged_ticks=len(rows), val_r2=stats["val_r2"],
                              terms_r2=fit["r2"], per_workload={
                                  k: (v["best_measured"], v["best_predicted"])
                                  for k, v in fit["per_workload"].items()})))
        return 0
    model = load(Path(args.model))
    if args.cmd == "mix":
        out = mix(torch, model, tuple(int(v) for v in args.fixed.split(",")), args.ticks,
                  n_scenes=args.scenes, log=log)
        print(json.dumps(out))
        return 0 if out["identical_results"] else 1
    out = compare(args.workload, args.ticks + args.warmup, args.warmup, torch, model,
                  schedule=args.schedule, log=log)
    print(json.dumps(out))
    return 0 if out["identical_results"] else 1


if __name__ == "__main__":
    sys.exit(main())
