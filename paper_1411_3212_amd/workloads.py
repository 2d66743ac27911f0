"""Seeded synthetic moving-object workloads.

This module only draws inputs: object positions per tick and the range
queries issued during the tick.  It holds none of the join's arithmetic and is
shared by the HIP path's tests/benchmark and by the CPU oracle's tests, so that
both sides consume bit-identical inputs.

All draws use ``numpy.random.Generator(PCG64(seed))`` in float64 and are
rounded to binary32 (round-to-nearest-even) when emitted.  A query is a
rectangle centred on its issuer: with ``h = f32(side) / 2`` (an exact halving)
the corners are ``fl32(x - h)`` and ``fl32(x + h)``, so the issuer always lies
inside its own query (the paper's result set of a query includes the object
that issued it).

Workloads (the paper's experiments use uniform, Gaussian-hotspot and road
network data; the road network is replaced by random line segments):

* ``uniform_1tick``   4,096 objects uniform in [0,1)^2, 1,024 square queries
  of side 0.01 centred on distinct objects, 1 tick.
* ``hotspot``         1M objects: 20 Gaussian hotspots (sigma 0.01) holding 90%
  of the objects, 10% uniform; random walk with step r ~ U[0, 5e-4] in a
  uniformly random direction, reflected at 0 and 1; each tick 10% of the
  objects issue a square query of side 0.002; 100 ticks.
* ``segments``        4M objects on 1,000 random segments (jitter sigma 2e-4),
  moving along their segment at U[1e-4, 1e-3] per tick and bouncing at the
  ends; 50% issue rectangles with sides U[5e-4, 4e-3]; 50 ticks.
* ``hotspot_20m``     as ``hotspot`` with 20M objects.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Iterator

import numpy as np


@dataclass
class Tick:
    """One tick's batch: position updates (id, x, y) and range queries
    (qid = issuing object, lower-left and upper-right corners)."""

    ids: np.ndarray
    x: np.ndarray
    y: np.ndarray
    qid: np.ndarray
    xa: np.ndarray
    ya: np.ndarray
    xb: np.ndarray
    yb: np.ndarray

    @property
    def nq(self) -> int:
        return int(len(self.qid))

    @property
    def rects(self):
        return (self.xa, self.ya, self.xb, self.yb)


def centred_rects(x32: np.ndarray, y32: np.ndarray, w, h):
    """Corners of rectangles of width w and height h (float64, scalars or
    arrays) centred on binary32 points, computed in binary32."""
    hx = (np.asarray(w, dtype=np.float64).astype(np.float32) / np.float32(2)).astype(np.float32)
    hy = (np.asarray(h, dtype=np.float64).astype(np.float32) / np.float32(2)).astype(np.float32)
    xa = (x32 - hx).astype(np.float32)
    xb = (x32 + hx).astype(np.float32)
    ya = (y32 - hy).astype(np.float32)
    yb = (y32 + hy).astype(np.float32)
    return xa, ya, xb, yb


@dataclass
class Workload:
    name: str
    n: int
    n_ticks: int
    seed: int
    params: dict = field(default_factory=dict)

    def ticks(self) -> Iterator[Tick]:
        gen = _GENERATORS[self.params.get("kind", self.name)]
        return gen(self)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _uniform_1tick(w: Workload) -> Iterator[Tick]:
    rng = _rng(w.seed)
    n = w.n
    x = rng.random(n).astype(np.float32)
    y = rng.random(n).astype(np.float32)
    nq = int(w.params.get("nq", 1024))
    side = float(w.params.get("side", 0.01))
    for _ in range(w.n_ticks):
        qid = rng.choice(n, size=nq, replace=False).astype(np.uint32)
        xa, ya, xb, yb = centred_rects(x[qid], y[qid], side, side)
        yield Tick(np.arange(n, dtype=np.uint32), x.copy(), y.copy(), qid, xa, ya, xb, yb)


def _hotspot_positions(rng: np.random.Generator, n: int, n_hot: int, sigma: float,
                       frac_uniform: float):
    centres = rng.random((n_hot, 2))
    uni = rng.random(n) < frac_uniform
    pos = rng.random((n, 2))
    hot = np.nonzero(~uni)[0]
    which = rng.integers(0, n_hot, size=len(hot))
    p = centres[which] + rng.normal(0.0, sigma, size=(len(hot), 2))
    bad = np.nonzero(((p < 0.0) | (p > 1.0)).any(axis=1))[0]
    while len(bad):  # resample points that fall outside the unit square
        p[bad] = centres[which[bad]] + rng.normal(0.0, sigma, size=(len(bad), 2))
        bad = bad[((p[bad] < 0.0) | (p[bad] > 1.0)).any(axis=1)]
    pos[hot] = p
    return pos


def _reflect01(v: np.ndarray) -> None:
    np.abs(v, out=v)
    over = v > 1.0
    v[over] = 2.0 - v[over]


def _hotspot(w: Workload) -> Iterator[Tick]:
    rng = _rng(w.seed)
    n = w.n
    P = w.params
    pos = _hotspot_positions(rng, n, int(P.get("hotspots", 20)), float(P.get("sigma", 0.01)),
                             float(P.get("uniform", 0.10)))
    step = float(P.get("step", 5e-4))
    rate = float(P.get("query_rate", 0.10))
    side = float(P.get("side", 0.002))
    ids = np.arange(n, dtype=np.uint32)
    nq = int(round(rate * n))
    for k in range(w.n_ticks):
        if k > 0:
            r = rng.random(n) * step
            th = rng.random(n) * (2.0 * np.pi)
            pos[:, 0] += r * np.cos(th)
            pos[:, 1] += r * np.sin(th)
            _reflect01(pos[:, 0])
            _reflect01(pos[:, 1])
        x = pos[:, 0].astype(np.float32)
        y = pos[:, 1].astype(np.float32)
        qid = rng.choice(n, size=nq, replace=False).astype(np.uint32)
        xa, ya, xb, yb = centred_rects(x[qid], y[qid], side, side)
        yield Tick(ids, x, y, qid, xa, ya, xb, yb)


def _segments(w: Workload) -> Iterator[Tick]:
    rng = _rng(w.seed)
    n = w.n
    P = w.params
    nseg = int(P.get("segments", 1000))
    a = rng.random((nseg, 2))
    b = rng.random((nseg, 2))
    length = np.sqrt(((b - a) ** 2).sum(axis=1))
    length = np.maximum(length, 1e-9)
    seg = rng.choice(nseg, size=n, p=length / length.sum())
    t = rng.random(n)
    jit = rng.normal(0.0, float(P.get("jitter", 2e-4)), size=(n, 2))
    speed = rng.uniform(float(P.get("vmin", 1e-4)), float(P.get("vmax", 1e-3)), size=n)
    sign = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    dt = speed / length[seg]
    rate = float(P.get("query_rate", 0.5))
    smin, smax = float(P.get("qmin", 5e-4)), float(P.get("qmax", 4e-3))
    ids = np.arange(n, dtype=np.uint32)
    nq = int(round(rate * n))
    A = a[seg]
    D = b[seg] - a[seg]
    for k in range(w.n_ticks):
        if k > 0:
            t += sign * dt
            hi = t > 1.0
            t[hi] = 2.0 - t[hi]
            sign[hi] = -sign[hi]
            lo = t < 0.0
            t[lo] = -t[lo]
            sign[lo] = -sign[lo]
            np.clip(t, 0.0, 1.0, out=t)
        pos = A + t[:, None] * D + jit
        np.clip(pos, 0.0, 1.0, out=pos)
        x = pos[:, 0].astype(np.float32)
        y = pos[:, 1].astype(np.float32)
        qid = rng.choice(n, size=nq, replace=False).astype(np.uint32)
        wq = rng.uniform(smin, smax, size=nq)
        hq = rng.uniform(smin, smax, size=nq)
        xa, ya, xb, yb = centred_rects(x[qid], y[qid], wq, hq)
        yield Tick(ids, x, y, qid, xa, ya, xb, yb)


_GENERATORS = {
    "uniform_1tick": _uniform_1tick,
    "hotspot": _hotspot,
    "segments": _segments,
}

WORKLOADS = {
    "uniform_1tick": dict(n=4096, n_ticks=1, seed=1, params=dict(kind="uniform_1tick", nq=1024,
                                                                 side=0.01)),
    "hotspot": dict(n=1_000_000, n_ticks=100, seed=2, params=dict(kind="hotspot")),
    "segments": dict(n=4_000_000, n_ticks=50, seed=3, params=dict(kind="segments")),
    "hotspot_20m": dict(n=20_000_000, n_ticks=50, seed=4, params=dict(kind="hotspot")),
}


def make(name: str, **overrides) -> Workload:
    """A named workload; ``n``, ``n_ticks``, ``seed`` and any generator
    parameter can be overridden (e.g. a smaller ``hotspot`` for tests)."""
    spec = dict(WORKLOADS[name])
    params = dict(spec.pop("params"))
    for key in ("n", "n_ticks", "seed"):
        if key in overrides:
            spec[key] = overrides.pop(key)
    params.update(overrides)
    return Workload(name=name, params=params, **spec)


def issuer_points(t: Tick):
    """Points of k-nearest-neighbour queries: each issuer's position in the
    tick's updates (every generator here updates every object on every tick,
    in id order)."""
    if len(t.ids) == 0 or int(t.ids[-1]) != len(t.ids) - 1:
        raise ValueError("issuer_points needs a tick that updates objects 0..n-1 in order")
    return t.x[t.qid], t.y[t.qid]
