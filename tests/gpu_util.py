"""Helpers of the GPU tests: move workload ticks to the device, run them
through the library, and compute the oracle's answer on the same inputs."""
import sys

import numpy as np

import oracle
from paper_1411_3212_amd.binding import Scene


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev_u32(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).cuda()


def dev_f32(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def gpu_tick(scene: Scene, t, updates=True):
    if updates and len(t.ids):
        scene.apply_updates(dev_u32(t.ids), dev_f32(t.x), dev_f32(t.y))
    scene.run_tick(dev_u32(t.qid), *(dev_f32(r) for r in t.rects))


def oracle_apply(st: oracle.State, t):
    if len(t.ids):
        oracle.apply_updates(st, t.ids, t.x, t.y)


def oracle_lists(st: oracle.State, t):
    live = oracle.live_queries(st.N, t.qid)
    off, ids = oracle.brute_lists(st, live, t.rects)
    return [ids[off[k]:off[k + 1]].tolist() for k in range(len(t.qid))]


def oracle_count_hash(st: oracle.State, t, grid=True):
    live = oracle.live_queries(st.N, t.qid)
    f = oracle.grid_hash if grid else oracle.brute_hash
    return f(st, t.qid, live, t.rects)


def gpu_count_hash(scene: Scene):
    cnt, h = scene.hashes()
    return cnt.cpu().numpy().view(np.uint64), h.cpu().numpy().view(np.uint64)


class T:
    """A tick assembled by hand (same fields as workloads.Tick)."""

    def __init__(self, ids=(), x=(), y=(), qid=(), rects=((), (), (), ())):
        self.ids = np.asarray(ids, np.uint32)
        self.x = np.asarray(x, np.float32)
        self.y = np.asarray(y, np.float32)
        self.qid = np.asarray(qid, np.uint32)
        self.xa, self.ya, self.xb, self.yb = (np.asarray(r, np.float32) for r in rects)

    @property
    def rects(self):
        return (self.xa, self.ya, self.xb, self.yb)

    @property
    def nq(self):
        return len(self.qid)
