"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Result sets are integer data: they must be identical (bit-exact ids) to the
brute-force evaluation of Definition 1 on the same binary32 inputs.  The
index (sorted codes, leaf table) and the subquery split are compared with the
oracle's Algorithm 1 and query splitting.  At full size every query is
checked by count + pair-set hash against the oracle's grid, and a sample of
queries by literal lists against the brute force.
"""
import numpy as np
import pytest

import oracle
from gpu_util import T, dev_f32, dev_u32, gpu_count_hash, gpu_tick, oracle_apply, \
    oracle_count_hash, oracle_lists, say
from paper_1411_3212_amd import workloads
from paper_1411_3212_amd.binding import SJ_EDATA, SJ_EINVAL, SJ_EOVERFLOW, Scene, SjError

pytestmark = pytest.mark.gpu
F32 = np.float32


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


def run_scene(n, t, **kw):
    sc = Scene(n, max(t.nq, 1), **kw)
    gpu_tick(sc, t)
    return sc


# ----------------------------------------------------------- small, exact

def test_uniform_1tick_lists_equal_brute_force():
    wl, t, st = c1()
    say("uniform_1tick n=4096 nq=1024 th=64")
    want = oracle_lists(st, t)
    sc = run_scene(wl.n, t, th=64)
    r = sc.fetch()
    assert r.to_lists() == want
    s = sc.stats()
    assert s["n_present"] == wl.n and s["rebuilt"] == 1
    assert r.total_pairs == sum(len(w) for w in want)
    assert all(int(q) in w for q, w in zip(t.qid, want))


@pytest.mark.parametrize("th", [1, 16, 64, 384, 1_000_000])
@pytest.mark.parametrize("covering,reorder", [(True, True), (False, True), (True, False)])
def test_results_do_not_depend_on_threshold_or_switches(th, covering, reorder):
    wl, t, st = c1()
    say(f"switches th={th} covering={covering} reorder={reorder}")
    want = oracle_lists(st, t)
    sc = run_scene(wl.n, t, th=th, covering=covering, reorder=reorder)
    assert sc.fetch().to_lists() == want
    s = sc.stats()
    if not covering:
        assert s["n_cov"] == 0 and s["cov_pairs"] == 0


@pytest.mark.parametrize("th", [1, 4, 64, 384])
def test_index_equals_oracle_algorithm_1(th):
    wl, t, st = c1()
    say(f"index parity th={th}")
    sc = run_scene(wl.n, t, th=th)
    v = sc.index_view()
    fr = oracle.frame(st)
    assert (F32(v["x0"]), F32(v["y0"]), v["e"]) == (F32(fr[0]), F32(fr[1]), fr[2])
    codes, ids = oracle.sorted_codes(st, fr)
    assert np.array_equal(v["codes"].cpu().numpy().view(np.uint32), codes)
    assert np.array_equal(v["ids"].cpu().numpy().view(np.uint32), ids)
    lv = oracle.quadtree(codes, th, 16)
    assert v["n_leaves"] == len(lv) and v["l_deep"] == lv.l_deep
    assert np.array_equal(v["leaf_start"].cpu().numpy().view(np.uint32).astype(np.uint64), lv.start)
    assert np.array_equal(v["leaf_level"].cpu().numpy(), lv.lvl.astype(np.int32))
    beg = v["leaf_beg"].cpu().numpy().view(np.uint32)
    assert np.array_equal(beg[:-1], lv.beg) and beg[-1] == wl.n


@pytest.mark.parametrize("th", [4, 64])
def test_split_and_work_counters_equal_oracle(th):
    wl, t, st = c1()
    say(f"split parity th={th}")
    sc = run_scene(wl.n, t, th=th)
    s = sc.stats()
    r = sc.fetch()
    fr = oracle.frame(st)
    codes, ids = oracle.sorted_codes(st, fr)
    lv = oracle.quadtree(codes, th, 16)
    live = oracle.live_queries(wl.n, t.qid)
    oi, li, oc, lc = oracle.split(live, t.rects, fr, lv)
    cnt = lv.count
    li_act, lc_act = li[cnt[li] > 0], lc[cnt[lc] > 0]
    assert s["n_isect"] == len(li_act) and s["n_cov"] == len(lc_act)
    per_leaf = np.bincount(li_act, minlength=len(lv))
    # filtering work = sum over active leaves of |intersecting subqueries| x |objects|
    assert s["tests"] == int((per_leaf * cnt).sum())
    assert s["n_tasks"] == int((per_leaf > 0).sum())
    assert s["cov_pairs"] == int(cnt[lc_act].sum())
    co = r.cov_off.cpu().numpy().view(np.uint32)
    cl = r.cov_leaf.cpu().numpy().view(np.uint32)
    qp = r.query_pos.cpu().numpy().view(np.uint32)
    for k in range(t.nq):
        want = [x for x in lc[oc[k]:oc[k + 1]] if cnt[x] > 0]
        p = qp[k]
        assert sorted(cl[co[p]:co[p + 1]].tolist()) == want


def test_edges_corners_signed_zero_and_degenerate_queries():
    xa, ya, xb, yb = F32(0.25), F32(0.25), F32(0.75), F32(0.5)
    nx = np.nextafter
    pts = [(xa, ya), (xb, yb), (xa, yb), (xb, ya), (xa, F32(0.3)), (xb, F32(0.3)),
           (F32(0.5), ya), (F32(0.5), yb), (nx(xa, F32(-1)), F32(0.3)), (nx(xb, F32(2)), F32(0.3)),
           (F32(0.5), nx(ya, F32(-1))), (F32(0.5), nx(yb, F32(2))), (F32(-0.0), F32(0.0)),
           (F32(0.0), F32(-0.0)), (F32(1.0), F32(1.0))]
    n = len(pts)
    rects = [(xa, ya, xb, yb), (-0.0, -0.0, 0.0, 0.0), (0.5, 0.25, 0.5, 0.25), (-5, -5, 5, 5),
             (2, 2, 3, 3), (1.0, 1.0, 1.0, 1.0), (-1, 0.3, 0.25, 0.3)]
    t = T(ids=range(n), x=[p[0] for p in pts], y=[p[1] for p in pts], qid=range(len(rects)),
          rects=tuple(np.array(rects, np.float64)[:, c].astype(F32) for c in range(4)))
    st = oracle.State(n)
    oracle_apply(st, t)
    want = oracle_lists(st, t)
    assert want[0] == list(range(8))
    for th in (1, 2, 64):
        sc = run_scene(n, t, th=th)
        assert sc.fetch().to_lists() == want


@pytest.mark.parametrize("n", [32, 33, 64, 65, 511, 512, 513, 767, 768, 769, 1536, 1537, 2000])
def test_leaf_sizes_around_the_register_blocks(n):
    """A leaf of n objects (a cluster in the lower-left level-1 quadrant, one
    more object in the opposite corner, the threshold above n) queried by
    150 random rectangles, so that a task holds 64 subqueries and the leaf
    several tasks: the half-wave rounds (at most 32 objects), every chunk
    count of a one-block task (up to 12 chunks, 768 objects) and the
    multi-block tasks beyond, each with a full and a partial last chunk."""
    rng = np.random.default_rng(n)
    x = np.append(rng.uniform(0.1, 0.3, n), 0.9).astype(F32)
    y = np.append(rng.uniform(0.1, 0.3, n), 0.9).astype(F32)
    nq = 150
    c = rng.uniform(0.1, 0.3, (nq, 2))
    h = rng.uniform(0.005, 0.12, (nq, 2))
    rects = tuple(a.astype(F32) for a in (c[:, 0] - h[:, 0], c[:, 1] - h[:, 1],
                                           c[:, 0] + h[:, 0], c[:, 1] + h[:, 1]))
    t = T(ids=range(n + 1), x=x, y=y, qid=rng.integers(0, n, nq), rects=rects)
    st = oracle.State(n + 1)
    oracle_apply(st, t)
    codes, _ = oracle.sorted_codes(st, oracle.frame(st))
    assert int(oracle.quadtree(codes, 1_000_000, 16).count.max()) == n  # the construction
    want = oracle_lists(st, t)
    say(f"leaf sizes n={n}")
    sc = run_scene(n + 1, t, th=1_000_000, capacity_subqueries=4 * nq,
                   capacity_results=(n + 1) * nq)
    assert sc.fetch().to_lists() == want


def test_absent_objects_superseded_queries_and_empty_scenes():
    # objects 0..9, only the even ones have a position; queries by object 3
    # twice (only the last is answered) and by absent object 5
    n = 10
    t = T(ids=[0, 2, 4, 6, 8], x=[0.1, 0.2, 0.3, 0.4, 0.5], y=[0.1, 0.2, 0.3, 0.4, 0.5],
          qid=[3, 5, 3], rects=([0.0, 0.0, 0.15], [0.0, 0.0, 0.15], [1.0, 1.0, 0.35],
                                [1.0, 1.0, 0.35]))
    st = oracle.State(n)
    oracle_apply(st, t)
    want = oracle_lists(st, t)
    assert want == [[], [0, 2, 4, 6, 8], [2, 4]]
    sc = run_scene(n, t, th=1)
    assert sc.fetch().to_lists() == want
    # a scene where nobody has a position yet, then no queries at all
    e = T(qid=[1, 2], rects=([0.0, -1.0], [0.0, -1.0], [1.0, 1.0], [1.0, 1.0]))
    sc = run_scene(n, e, th=1)
    assert sc.fetch().to_lists() == [[], []]
    sc.run_tick(*(dev_u32([]),), *(dev_f32([]) for _ in range(4)))
    assert sc.fetch().to_lists() == []


def test_single_object_and_duplicates_beyond_threshold():
    n = 200
    x = np.full(n, 0.3, F32)
    y = np.full(n, 0.6, F32)
    x[150:] = np.linspace(0, 1, 50, dtype=F32)
    q = [(0.3, 0.6, 0.3, 0.6), (0.0, 0.0, 1.0, 1.0), (0.29, 0.59, 0.31, 0.61)]
    t = T(ids=range(n), x=x, y=y, qid=[0, 1, 2],
          rects=tuple(np.array(q)[:, c].astype(F32) for c in range(4)))
    st = oracle.State(n)
    oracle_apply(st, t)
    want = oracle_lists(st, t)
    sc = run_scene(n, t, th=8)
    assert sc.fetch().to_lists() == want
    s = sc.stats()
    assert s["l_deep"] == 16  # 150 coincident points cannot be split below th
    one = T(ids=[7], x=[0.5], y=[0.5], qid=[7], rects=([0.5], [0.5], [0.5], [0.5]))
    sc = run_scene(n, one, th=8)
    assert sc.fetch().to_lists() == [[7]]


def test_invalid_inputs_are_reported_and_ignored():
    n = 16
    t = T(ids=range(n), x=np.linspace(0, 1, n), y=np.linspace(0, 1, n), qid=[0, 1],
          rects=([0.6, 0.0], [0.0, 0.0], [0.4, 1.0], [1.0, 1.0]))  # query 0 inverted
    sc = run_scene(n, t, th=2)
    with pytest.raises(SjError) as ei:
        sc.fetch()
    assert ei.value.code == SJ_EDATA
    bad = T(ids=[3, 99], x=[0.1, 0.2], y=[0.1, 0.2], qid=[3], rects=([0.0], [0.0], [1.0], [1.0]))
    sc = run_scene(n, bad, th=2)
    with pytest.raises(SjError) as ei:
        sc.fetch()
    assert ei.value.code == SJ_EINVAL
    nan = T(ids=[3], x=[np.nan], y=[0.2], qid=[3], rects=([0.0], [0.0], [1.0], [1.0]))
    sc = run_scene(n, nan, th=2)
    with pytest.raises(SjError) as ei:
        sc.fetch()
    assert ei.value.code == SJ_EDATA


def test_overflow_is_detected_and_tick_can_be_rerun():
    wl, t, st = c1()
    want = oracle_lists(st, t)
    sc = Scene(wl.n, t.nq, th=64, capacity_results=16)
    gpu_tick(sc, t)
    with pytest.raises(SjError) as ei:
        sc.fetch()
    assert ei.value.code == SJ_EOVERFLOW
    sc = Scene(wl.n, t.nq, th=64, capacity_subqueries=8)
    gpu_tick(sc, t)
    with pytest.raises(SjError) as ei:
        sc.fetch()
    assert ei.value.code == SJ_EOVERFLOW
    # run_tick leaves positions unchanged: the same tick again after growing
    big = Scene(wl.n, t.nq, th=64)
    gpu_tick(big, t)
    assert big.fetch().to_lists() == want


def test_outputs_are_deterministic_and_expand_matches():
    wl, t, st = c1()
    want = oracle_lists(st, t)
    outs = []
    for _ in range(2):
        sc = run_scene(wl.n, t, th=16)
        r = sc.fetch()
        outs.append([x.cpu().numpy().tobytes() for x in
                     (r.query_pos, r.isect_slot_off, r.slot_run, r.run_off, r.isect_id, r.cov_off,
                      r.cov_leaf,
                      r.leaf_beg, r.sorted_id)])
        off, ids = sc.expand()
        off, ids = off.cpu().numpy(), ids.cpu().numpy()
        assert [sorted(ids[off[k]:off[k + 1]].tolist()) for k in range(t.nq)] == want
        cnt, h = gpu_count_hash(sc)
        oc, oh = oracle_count_hash(st, t, grid=False)
        assert np.array_equal(cnt, oc) and np.array_equal(h, oh)
    assert outs[0] == outs[1]


# ----------------------------------------------------------- multi-tick

@pytest.mark.parametrize("name,rebuild,th", [("hotspot", "auto", 64), ("hotspot", "always", 16),
                                             ("hotspot", "never", 384),
                                             ("segments", "auto", 64)])
def test_ticks_with_index_reuse_match_oracle(name, rebuild, th):
    wl = workloads.make(name, n=30_011, n_ticks=4)
    say(f"{name} n={wl.n} rebuild={rebuild} th={th}")
    st = oracle.State(wl.n)
    sc = Scene(wl.n, wl.n, th=th, rebuild=rebuild, rebuild_period=3)
    for k, t in enumerate(wl.ticks()):
        oracle_apply(st, t)
        gpu_tick(sc, t)
        cnt, h = gpu_count_hash(sc)
        oc, oh = oracle_count_hash(st, t, grid=False)
        assert np.array_equal(cnt, oc) and np.array_equal(h, oh), f"tick {k}"
        s = sc.stats()
        if rebuild == "always" or k == 0:
            assert s["rebuilt"] == 1
        if rebuild == "never" and k > 0:
            assert s["rebuilt"] == 0


def test_objects_leaving_the_frame_of_a_reused_index():
    n = 5000
    rng = np.random.default_rng(4)
    x0 = (rng.random(n) * 0.5).astype(F32)
    y0 = (rng.random(n) * 0.5).astype(F32)
    q = rng.random((300, 2)) * 1.6 - 0.3
    rect = lambda: tuple(a.astype(F32) for a in (q[:, 0], q[:, 1], q[:, 0] + 0.1, q[:, 1] + 0.1))
    qid = rng.choice(n, 300, replace=False)
    sc = Scene(n, 300, th=16, rebuild="never")
    st = oracle.State(n)
    for k in range(3):
        x = x0 + F32(0.4 * k)
        y = y0 - F32(0.3 * k)
        t = T(ids=range(n), x=x, y=y, qid=qid, rects=rect())
        oracle_apply(st, t)
        gpu_tick(sc, t)
        assert sc.fetch().to_lists() == oracle_lists(st, t), f"tick {k}"
        assert sc.stats()["rebuilt"] == (1 if k == 0 else 0)


def test_kept_quadtree_of_one_level():
    # at most th objects: the four level-1 quadrants are the leaves (the
    # root is always split) and the start table has four cells; ticks that
    # keep the quadtree map objects to those leaves
    n = 40
    rng = np.random.default_rng(7)
    sc = Scene(n, n, th=64, rebuild="never")
    st = oracle.State(n)
    for k in range(3):
        x = rng.uniform(0.2, 0.6, n).astype(F32)
        y = rng.uniform(0.2, 0.6, n).astype(F32)
        h = F32(0.05)
        rects = (x - h, y - h, x + h, y + h)
        t = T(ids=range(n), x=x, y=y, qid=range(n), rects=rects)
        oracle_apply(st, t)
        gpu_tick(sc, t)
        assert sc.fetch().to_lists() == oracle_lists(st, t), f"tick {k}"
        s = sc.stats()
        assert s["n_leaves"] == 4 and s["rebuilt"] == (1 if k == 0 else 0)


def test_partial_updates_keep_last_known_positions():
    n = 3000
    wl = workloads.make("hotspot", n=n, n_ticks=3)
    st = oracle.State(n)
    sc = Scene(n, n, th=32)
    rng = np.random.default_rng(1)
    for k, t in enumerate(wl.ticks()):
        sel = np.sort(rng.choice(n, n // 3, replace=False)) if k else np.arange(n)
        # duplicates within the batch: the later entry must win
        dup = sel[:50]
        part = T(ids=np.r_[sel, dup], x=np.r_[t.x[sel], t.x[dup] + F32(0.01)],
                 y=np.r_[t.y[sel], t.y[dup]], qid=t.qid, rects=t.rects)
        oracle_apply(st, part)
        gpu_tick(sc, part)
        assert sc.fetch().to_lists() == oracle_lists(st, part), f"tick {k}"


def test_several_update_calls_in_one_tick():
    # three calls before one tick: the latest update of an object wins across
    # calls; objects not updated keep their position from earlier ticks
    n = 2000
    rng = np.random.default_rng(7)
    st = oracle.State(n)
    sc = Scene(n, n, th=16)
    for k in range(3):
        calls = []
        for c in range(3):
            ids = rng.choice(n, n // 2, replace=True).astype(np.uint32)
            if k == 0 and c == 0:
                ids = np.arange(n, dtype=np.uint32)
            calls.append(T(ids=ids, x=rng.random(len(ids)), y=rng.random(len(ids))))
        qid = rng.choice(n, 200, replace=True).astype(np.uint32)  # repeated issuers
        c = rng.random((200, 2))
        q = T(qid=qid, rects=tuple(a.astype(F32) for a in (c[:, 0], c[:, 1], c[:, 0] + 0.05,
                                                           c[:, 1] + 0.05)))
        for u in calls:
            oracle_apply(st, u)
            sc.apply_updates(dev_u32(u.ids), dev_f32(u.x), dev_f32(u.y))
        sc.run_tick(dev_u32(q.qid), *(dev_f32(r) for r in q.rects))
        assert sc.fetch().to_lists() == oracle_lists(st, q), f"tick {k}"


# ------------------------------------------------------------- full size

def test_hotspot_full_size_ticks():
    """The benchmark's workload (1M objects, 100K queries per tick) in the
    benchmark's configuration: every query by count + hash against the CPU
    grid, 500 sampled queries by literal lists against the brute force."""
    from bench import scene_config
    wl = workloads.make("hotspot", n_ticks=3)
    st = oracle.State(wl.n)
    sc = Scene(wl.n, int(0.1 * wl.n), **scene_config(wl))
    rng = np.random.default_rng(0)
    for k, t in enumerate(wl.ticks()):
        say(f"hotspot 1M tick {k}")
        oracle_apply(st, t)
        gpu_tick(sc, t)
        cnt, h = gpu_count_hash(sc)
        oc, oh = oracle_count_hash(st, t, grid=True)
        assert np.array_equal(cnt, oc) and np.array_equal(h, oh)
        lists = sc.fetch().to_lists() if k == 0 else None
        if lists is not None:
            sample = rng.choice(t.nq, 500, replace=False)
            sub = T(qid=t.qid[sample], rects=tuple(r[sample] for r in t.rects))
            want = oracle_lists(st, sub)
            assert [lists[i] for i in sample] == want


def test_million_query_batches_in_spatial_order():
    """Batches of at least 2^20 queries are split in the spatial order of
    their corners: every query by count + hash against the CPU grid, over a
    tick that builds the quadtree and one that reuses it, and 300 sampled
    queries by literal lists against the brute force."""
    from bench import scene_config
    wl = workloads.make("hotspot", n=1_200_000, n_ticks=2, query_rate=0.9)
    st = oracle.State(wl.n)
    cfg = scene_config(wl)
    sc = Scene(wl.n, int(0.9 * wl.n), **cfg)
    rng = np.random.default_rng(1)
    for k, t in enumerate(wl.ticks()):
        say(f"hotspot 1.2M objects, {t.nq} queries, tick {k}")
        assert t.nq >= 1 << 20
        oracle_apply(st, t)
        gpu_tick(sc, t)
        cnt, h = gpu_count_hash(sc)
        oc, oh = oracle_count_hash(st, t, grid=True)
        assert np.array_equal(cnt, oc) and np.array_equal(h, oh)
        if k == 1:
            lists = sc.fetch().to_lists()
            sample = rng.choice(t.nq, 300, replace=False)
            sub = T(qid=t.qid[sample], rects=tuple(r[sample] for r in t.rects))
            want = oracle_lists(st, sub)
            assert [lists[i] for i in sample] == want


def test_graph_ticks_equal_eager_ticks():
    """Updates + tick replayed as a captured graph give the same bytes as the
    eager calls, through quadtree builds, reuse, and buffer changes (fixed
    buffers on ticks 0-3, fresh ones on every later tick)."""
    import torch
    wl = workloads.make("hotspot", n=40_000, n_ticks=8)
    eager = Scene(wl.n, wl.n, th=32, rebuild_period=3)
    graph = Scene(wl.n, wl.n, th=32, rebuild_period=3)
    slots = None
    st = oracle.State(wl.n)
    for k, t in enumerate(wl.ticks()):
        say(f"graph tick {k}")
        oracle_apply(st, t)
        gpu_tick(eager, t)
        d = [dev_u32(t.ids), dev_f32(t.x), dev_f32(t.y), dev_u32(t.qid)] + \
            [dev_f32(r) for r in t.rects]
        if k < 4:
            if slots is None:
                slots = [torch.empty_like(a) for a in d]
            for a, b in zip(slots, d):
                a.copy_(b)
            graph.tick_graph(*slots)
        else:
            graph.tick_graph(*d)
        if k % 2 == 1:  # ticks the host has not fetched: device decides
            continue
        re, rg = eager.fetch(), graph.fetch()
        for a, b in zip((re.query_pos, re.isect_slot_off, re.slot_run, re.run_off, re.isect_id,
                         re.cov_off,
                         re.cov_leaf, re.leaf_beg),
                        (rg.query_pos, rg.isect_slot_off, rg.slot_run, rg.run_off, rg.isect_id,
                         rg.cov_off,
                         rg.cov_leaf, rg.leaf_beg)):
            assert torch.equal(a, b)
        cnt, h = gpu_count_hash(graph)
        oc, oh = oracle_count_hash(st, t, grid=False)
        assert np.array_equal(cnt, oc) and np.array_equal(h, oh), f"tick {k}"
        assert eager.stats()["rebuilt"] == graph.stats()["rebuilt"]
