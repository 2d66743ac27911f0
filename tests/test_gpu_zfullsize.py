"""Parity at the full sizes of the workloads the benchmark and the serving
runtime use (Definition 1: result sets are integer data and must be
identical to the oracle's on the same binary32 inputs).

* every query of a tick: result size and order-independent pair-set hash
  against the oracle's uniform grid;
* 300 sampled queries: literal lists, expanded and sorted on the device
  (sj_expand_results with SJ_SORTED), against the oracle's brute force;
* the segment workload (4M objects, 2M rectangles per tick), the 20M-object
  hotspot workload at the fixed threshold 64 and with the learned
  threshold, and the 16-scene serving mix at its specified sizes;
* query splitting with lists shorter than the subqueries of a query (the
  count and write passes walk such queries twice).

Each test runs a few ticks so that the oracle's CPU time stays bounded.
"""
import numpy as np
import pytest

import oracle
from gpu_util import T, gpu_count_hash, gpu_tick, oracle_apply, oracle_count_hash, \
    oracle_lists, say
from paper_1411_3212_amd import costmodel, serving, workloads
from paper_1411_3212_amd.binding import Scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.synchronize()


def check_tick(sc: Scene, st: oracle.State, t, rng, n_lists: int = 300, label: str = ""):
    """Every query by count + hash against the grid oracle, n_lists sampled
    queries by device-expanded sorted lists against the brute force."""
    cnt, h = gpu_count_hash(sc)
    oc, oh = oracle_count_hash(st, t, grid=True)
    assert np.array_equal(cnt, oc), f"{label}: counts differ at {np.nonzero(cnt != oc)[0][:5]}"
    assert np.array_equal(h, oh), f"{label}: hashes differ at {np.nonzero(h != oh)[0][:5]}"
    s = sc.stats()
    assert s["n_isect_ids"] + s["cov_pairs"] == int(oc.sum())
    if n_lists:
        sample = np.sort(rng.choice(t.nq, min(n_lists, t.nq), replace=False)).astype(np.uint32)
        got = sc.fetch().to_lists(sel=sample)
        sub = T(qid=t.qid[sample], rects=tuple(r[sample] for r in t.rects))
        want = oracle_lists(st, sub)
        assert got == want, f"{label}: sampled lists differ"
    return int(oc.sum())


def scene_for(wl, th=64, **kw):
    """A scene with the benchmark's capacities for the workload."""
    from bench import scene_config
    cfg = scene_config(wl, th)
    cfg.update(kw)
    return Scene(wl.n, serving.scene_capacities(wl, th)["nq"], **cfg)


def test_segments_4m_full_size():
    """4M objects on 1,000 segments, 2M rectangles per tick: a tick that
    builds the quadtree and two that keep it."""
    wl = workloads.make("segments", n_ticks=3)
    st = oracle.State(wl.n)
    sc = scene_for(wl)
    rng = np.random.default_rng(3)
    for k, t in enumerate(wl.ticks()):
        say(f"segments 4M tick {k}: {t.nq} queries")
        oracle_apply(st, t)
        gpu_tick(sc, t)
        pairs = check_tick(sc, st, t, rng, label=f"segments tick {k}")
        s = sc.stats()
        assert s["rebuilt"] == (1 if k == 0 else 0)
        say(f"  {pairs} pairs identical, {s['n_leaves']} leaves")


def test_hotspot_20m_fixed_threshold_full_size():
    """20M objects, 2M queries per tick, fixed threshold 64 (dense cores:
    queries overlap far more leaves than the split's list slots, so both
    split passes take the long-query path there)."""
    wl = workloads.make("hotspot_20m", n_ticks=3)
    st = oracle.State(wl.n)
    sc = scene_for(wl, 64)
    rng = np.random.default_rng(4)
    for k, t in enumerate(wl.ticks()):
        say(f"hotspot 20M th 64 tick {k}")
        oracle_apply(st, t)
        if k == 2:  # the graph launch of the benchmark
            from gpu_util import dev_f32, dev_u32
            sc.tick_graph(dev_u32(t.ids), dev_f32(t.x), dev_f32(t.y), dev_u32(t.qid),
                          *(dev_f32(r) for r in t.rects))
        else:
            gpu_tick(sc, t)
        pairs = check_tick(sc, st, t, rng, label=f"hotspot 20M tick {k}")
        s = sc.stats()
        assert s["rebuilt"] == (1 if k == 0 else 0)
        say(f"  {pairs} pairs identical, {s['n_leaves']} leaves, l_deep {s['l_deep']}")


def test_hotspot_20m_learned_threshold_full_size():
    """The same workload with the threshold chosen by the cost model: the
    tuned build and a tick that keeps its quadtree."""
    import torch
    wl = workloads.make("hotspot_20m", n_ticks=2)
    model = costmodel.load()
    st = oracle.State(wl.n)
    sc = scene_for(wl, 64, th_min=min(model["cand"]), thresh_mlp=True)
    costmodel.install(sc, model, torch)
    rng = np.random.default_rng(5)
    for k, t in enumerate(wl.ticks()):
        say(f"hotspot 20M learned tick {k}")
        oracle_apply(st, t)
        gpu_tick(sc, t)
        check_tick(sc, st, t, rng, label=f"hotspot 20M learned tick {k}")
        info = sc.tune_info()
        assert info["n_tunes"] == 1 and sc.stats()["th"] == info["chosen"]
        say(f"  threshold {info['chosen']}")


def test_serving_mix_16_scenes_full_size():
    """The serving mix at its specified sizes (16 scenes of 1e5-8e6 objects,
    even scenes hotspot, odd scenes segments): every served tick's per-query
    counts and hashes equal those of the scene run alone, and one tick of
    every scene equals the oracle's grid."""
    import torch
    specs = serving.make_specs()
    say("serving mix: " + " ".join(str(sp.wl.n) for sp in specs))
    serving.upload(specs, 2, torch)
    reqs = serving.poisson_requests(len(specs), 48, rate_per_scene=50.0, n_ticks=2, seed=9)
    r = serving.serve(specs, reqs, 96 << 30, max_running=4, torch=torch, keep_arrays=True)
    by_scene = {}
    for tag, (_, s, k) in enumerate(reqs):
        by_scene.setdefault(s, []).append((tag, k))
    for s, lst in sorted(by_scene.items()):
        alone = serving.serve_alone(specs[s], [k for _, k in lst], torch, keep_arrays=True)
        for (tag, k), (dig, arr) in zip(lst, alone):
            assert r["digest"][tag] == dig, (s, tag)
            assert np.array_equal(r["arrays"][tag][0], arr[0]), (s, tag)
            assert np.array_equal(r["arrays"][tag][1], arr[1]), (s, tag)
    say("served ticks equal the scenes run alone")
    for s, sp in enumerate(specs):
        if s not in by_scene:
            continue
        sp.wl.n_ticks = 2
        ticks = list(sp.wl.ticks())
        st = oracle.State(sp.wl.n)
        tag, k = by_scene[s][0]
        # the scene's requests replay ticks in request order: positions are
        # those of the ticks served so far
        oracle_apply(st, ticks[k])
        t = ticks[k]
        oc, oh = oracle_count_hash(st, t, grid=True)
        assert np.array_equal(r["arrays"][tag][0], oc), (s, tag)
        assert np.array_equal(r["arrays"][tag][1], oh), (s, tag)
        say(f"scene {s} ({sp.wl.n} objects) tick {k}: {int(oc.sum())} pairs identical to the grid")


@pytest.mark.parametrize("slots", [1, 2])
@pytest.mark.parametrize("th", [1, 64])
@pytest.mark.parametrize("covering", [True, False])
def test_split_with_short_query_lists(slots, th, covering):
    """Queries with more subqueries than split_slots are enumerated again by
    the write pass and placed after the listed ones: c1 (4,096 objects) and a
    hotspot scene (200K objects, dense cores) against the oracle."""
    c1 = workloads.make("uniform_1tick")
    t1 = next(c1.ticks())
    st1 = oracle.State(c1.n)
    oracle_apply(st1, t1)
    sc = Scene(c1.n, t1.nq, th=th, split_slots=slots, covering=covering,
               capacity_subqueries=512 * t1.nq, capacity_covering=512 * t1.nq)
    gpu_tick(sc, t1)
    assert sc.fetch().to_lists() == oracle_lists(st1, t1)
    cnt, h = gpu_count_hash(sc)
    oc, oh = oracle_count_hash(st1, t1, grid=False)
    assert np.array_equal(cnt, oc) and np.array_equal(h, oh)
    wl = workloads.make("hotspot", n=200_000, n_ticks=2)
    st = oracle.State(wl.n)
    per = 4096 if th == 1 else 256
    sc = Scene(wl.n, int(0.1 * wl.n), th=th, split_slots=slots, covering=covering,
               capacity_subqueries=per * int(0.1 * wl.n), capacity_covering=per * int(0.1 * wl.n),
               capacity_results=2048 * int(0.1 * wl.n))
    rng = np.random.default_rng(slots * 10 + th)
    for k, t in enumerate(wl.ticks()):
        say(f"split slots={slots} th={th} covering={covering} hotspot 200K tick {k}")
        oracle_apply(st, t)
        gpu_tick(sc, t)
        s = sc.stats()
        assert s["n_isect"] + s["n_cov"] > slots * t.nq  # the long path is taken
        check_tick(sc, st, t, rng, n_lists=200, label=f"slots {slots} th {th} tick {k}")
