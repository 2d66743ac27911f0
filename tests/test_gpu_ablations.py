"""The ablation paths against the oracle: the paper's baseline filter
(UG_Baseline, Algorithm SQB: results appended through atomics) gives the
same result sets as the lock-free join and the brute force, on the
quadtree and on the uniform grid; the per-CU test counters add up to the
filtering work and name every compute unit."""
import numpy as np
import pytest

import oracle
from gpu_util import gpu_count_hash, gpu_tick, oracle_apply, oracle_count_hash, oracle_lists, \
    say
from paper_1411_3212_amd import workloads
from paper_1411_3212_amd.binding import SJ_EOVERFLOW, Scene, SjError

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.synchronize()


def c1():
    wl = workloads.make("uniform_1tick")
    t = next(wl.ticks())
    st = oracle.State(wl.n)
    oracle_apply(st, t)
    return wl, t, st


@pytest.mark.parametrize("grid", [0, 40])
@pytest.mark.parametrize("th", [4, 64])
def test_baseline_filter_lists_equal_brute_force(grid, th):
    wl, t, st = c1()
    say(f"baseline filter c1 grid={grid} th={th}")
    sc = Scene(wl.n, t.nq, th=th, grid_split=grid, atomic_results=True,
               capacity_subqueries=64 * t.nq)
    gpu_tick(sc, t)
    r = sc.fetch()
    assert r.n_runs == 0 and r.n_pairs == r.n_isect_ids
    assert r.to_lists() == oracle_lists(st, t)
    ref = Scene(wl.n, t.nq, th=th, grid_split=grid, capacity_subqueries=64 * t.nq)
    gpu_tick(ref, t)
    assert ref.fetch().n_isect_ids == r.n_pairs
    pairs = r.pairs.cpu().numpy().view(np.uint32).reshape(-1, 2)
    assert (pairs[:, 0] < t.nq).all()
    with pytest.raises(SjError):
        sc.expand(sel=[0, 1])  # a selection needs the runs


def test_baseline_filter_hotspot_1m_hashes_equal_oracle():
    from bench import scene_config
    wl = workloads.make("hotspot", n_ticks=2)
    st = oracle.State(wl.n)
    sc = Scene(wl.n, int(0.1 * wl.n), atomic_results=True, **scene_config(wl))
    for k, t in enumerate(wl.ticks()):
        say(f"baseline filter hotspot 1M tick {k}")
        oracle_apply(st, t)
        gpu_tick(sc, t)
        cnt, h = gpu_count_hash(sc)
        oc, oh = oracle_count_hash(st, t, grid=True)
        assert np.array_equal(cnt, oc) and np.array_equal(h, oh)


def test_baseline_filter_overflow_is_reported():
    wl, t, st = c1()
    sc = Scene(wl.n, t.nq, th=64, atomic_results=True, capacity_results=16)
    gpu_tick(sc, t)
    with pytest.raises(SjError) as ei:
        sc.fetch()
    assert ei.value.code == SJ_EOVERFLOW


def test_cu_counters_add_up_to_the_filtering_work_on_every_cu():
    import torch
    from bench import scene_config
    wl = workloads.make("hotspot", n_ticks=1)
    t = next(wl.ticks())
    for atomic in (False, True):
        sc = Scene(wl.n, t.nq, cu_counters=True, atomic_results=atomic, **scene_config(wl))
        gpu_tick(sc, t)
        c = sc.cu_counters()
        s = sc.stats()
        assert int(c.sum()) == s["tests"]
        n_cu = torch.cuda.get_device_properties(0).multi_processor_count
        used = int((c > 0).sum())
        say(f"atomic={atomic}: tests {s['tests']} on {used} CU slots of {n_cu} CUs, "
            f"max {int(c.max())} min {int(c[c > 0].min())}")
        assert used == n_cu  # one slot per compute unit, every one busy
