"""The cost-based rebuild policy (rent or buy on the device clock): results
are identical to the oracle and to the periodic policy on every tick, and a
tree made stale by a sudden shift of the objects is rebuilt within a few
ticks (quadtree reuse, Section "Index creation (QUAD)": the partitioning is
kept while the distribution does not change significantly)."""
import numpy as np
import pytest

import oracle
from gpu_util import T, gpu_count_hash, gpu_tick, oracle_apply, oracle_count_hash, say
from paper_1411_3212_amd import workloads
from paper_1411_3212_amd.binding import Scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.synchronize()


def test_cost_policy_results_and_rebuild_after_a_shift():
    wl = workloads.make("hotspot", n=200_000, n_ticks=24)
    st = oracle.State(wl.n)
    kw = dict(capacity_subqueries=64 * 20_000, capacity_covering=64 * 20_000,
              capacity_results=1024 * 20_000)
    cost = Scene(wl.n, 20_000, th=64, rebuild="cost", **kw)
    auto = Scene(wl.n, 20_000, th=64, rebuild="auto", **kw)
    rebuilt = []
    for k, t in enumerate(wl.ticks()):
        if k >= 8:  # every object jumps: the frame and the leaves of the kept tree are stale
            x = (t.x * np.float32(0.5) + np.float32(0.25)).astype(np.float32)
            y = (t.y * np.float32(0.5)).astype(np.float32)
            xa, ya, xb, yb = workloads.centred_rects(x[t.qid], y[t.qid], 0.002, 0.002)
            t = T(ids=t.ids, x=x, y=y, qid=t.qid, rects=(xa, ya, xb, yb))
        oracle_apply(st, t)
        gpu_tick(cost, t)
        gpu_tick(auto, t)
        c1, h1 = gpu_count_hash(cost)
        c2, h2 = gpu_count_hash(auto)
        assert np.array_equal(c1, c2) and np.array_equal(h1, h2), f"tick {k}"
        if k % 6 == 0 or k in (8, 9):
            oc, oh = oracle_count_hash(st, t, grid=True)
            assert np.array_equal(c1, oc) and np.array_equal(h1, oh), f"tick {k}"
        rebuilt.append(cost.stats()["rebuilt"])
        say(f"tick {k}: cost policy rebuilt {rebuilt[-1]}")
    assert rebuilt[0] == 1
    assert any(rebuilt[9:16]), "the stale tree was not rebuilt within 7 ticks of the shift"
