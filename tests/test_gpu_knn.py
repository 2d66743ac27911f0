"""k-nearest-neighbour queries on the range-query pipeline (the paper's
future work, Section "Conclusions") against the oracle's brute force: ids
and binary32 squared distances of every slot must be identical (the
selection key is compare-only once d2 is computed, and both sides compute
d2 with the same three rounded operations)."""
import numpy as np
import pytest

import oracle
from gpu_util import T, dev_f32, dev_u32, oracle_apply, say
from paper_1411_3212_amd import workloads
from paper_1411_3212_amd.binding import SJ_EDATA, SJ_EINVAL, Scene, SjError

pytestmark = pytest.mark.gpu
NONE = 0xFFFFFFFF


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.synchronize()


def gpu_knn(sc, t, qx, qy, k, updates=True):
    if updates and len(t.ids):
        sc.apply_updates(dev_u32(t.ids), dev_f32(t.x), dev_f32(t.y))
    ids, d2 = sc.run_knn(dev_u32(t.qid), dev_f32(qx), dev_f32(qy), k)
    return ids.cpu().numpy().view(np.uint32), d2.cpu().numpy()


def check(st, t, qx, qy, k, ids, d2, sel=None, label=""):
    live = oracle.live_queries(st.N, t.qid)
    if sel is not None:
        live, qx, qy, ids, d2 = live[sel], qx[sel], qy[sel], ids[sel], d2[sel]
    wi, wd = oracle.knn(st, live, qx, qy, k)
    bad = np.nonzero((wi != ids).any(axis=1) | (wd.view(np.uint32) != d2.view(np.uint32))
                     .any(axis=1))[0]
    assert len(bad) == 0, f"{label}: {len(bad)} queries differ, first {bad[:5]}: " \
                          f"gpu {ids[bad[0]][:8]} oracle {wi[bad[0]][:8]}"


@pytest.mark.parametrize("k", [1, 5, 16, 64])
@pytest.mark.parametrize("th", [4, 64, 1_000_000])
def test_uniform_1tick_every_query(k, th):
    wl = workloads.make("uniform_1tick")
    t = next(wl.ticks())
    st = oracle.State(wl.n)
    oracle_apply(st, t)
    qx, qy = workloads.issuer_points(t)
    say(f"knn uniform_1tick k={k} th={th}")
    sc = Scene(wl.n, t.nq, th=th, capacity_subqueries=256 * t.nq, capacity_covering=256 * t.nq)
    ids, d2 = gpu_knn(sc, t, qx, qy, k)
    check(st, t, qx, qy, k, ids, d2, label=f"k={k} th={th}")
    assert (ids[:, 0] == t.qid).all()  # the issuer is its own nearest (distance 0, unique points)
    assert sc.stats()["knn_fallback"] == 0


def test_edge_cases():
    """Fewer present objects than k, absent objects, superseded queries,
    duplicate positions beyond the threshold (leaves at l_max), query points
    outside the objects' frame, an empty tick."""
    rng = np.random.default_rng(7)
    n = 600
    x = rng.random(n).astype(np.float32) * 0.5
    y = rng.random(n).astype(np.float32) * 0.5
    x[100:300] = np.float32(0.25)  # 200 objects on one point
    y[100:300] = np.float32(0.125)
    present = np.sort(rng.choice(n, 500, replace=False)).astype(np.uint32)
    t = T(ids=present, x=x[present], y=y[present],
          qid=[5, 7, 5, 150, 9, 11, 13, 400],
          rects=([0.1, 0.2, 0.3, 0.25, -3.0, 0.5, 7.0, 0.25], [0.1, 0.2, 0.3, 0.125, -3.0, 0.5,
                                                                -2.0, 0.125], [0] * 8, [0] * 8))
    qx, qy = t.xa.copy(), t.ya.copy()
    st = oracle.State(n)
    oracle_apply(st, t)
    for k in (1, 16, 64):
        say(f"knn edge cases k={k}")
        sc = Scene(n, 16, th=8)
        ids, d2 = gpu_knn(sc, t, qx, qy, k)
        check(st, t, qx, qy, k, ids, d2, label=f"edge k={k}")
        assert (ids[0] == NONE).all()  # query 0 is superseded by query 2 (same issuer)
    # fewer objects than k: every present object, then empty slots
    few = T(ids=[3, 1, 2], x=[0.5, 0.25, 0.75], y=[0.5, 0.5, 0.5], qid=[1], rects=([0.3], [0.5],
                                                                                [0], [0]))
    st2 = oracle.State(8)
    oracle_apply(st2, few)
    sc = Scene(8, 4)
    ids, d2 = gpu_knn(sc, few, few.xa, few.ya, 5)
    assert ids[0].tolist() == [1, 3, 2, NONE, NONE] and np.isinf(d2[0, 3:]).all()
    check(st2, few, few.xa, few.ya, 5, ids, d2, label="few")
    # a tick with no queries, then a query at a non-finite point
    ids, d2 = gpu_knn(sc, T(), np.zeros(0, np.float32), np.zeros(0, np.float32), 3)
    assert ids.shape == (0, 3)
    bad = T(qid=[1], rects=([np.nan], [0.5], [0], [0]))
    with pytest.raises(SjError) as e:
        gpu_knn(sc, bad, bad.xa, bad.ya, 3, updates=False)
    assert e.value.code == SJ_EDATA
    with pytest.raises(SjError) as e:
        gpu_knn(sc, few, few.xa, few.ya, 65)
    assert e.value.code == SJ_EINVAL


def test_objects_outside_the_kept_frame_take_the_fallback():
    """The quadtree of tick 0 (four leaves of 5,000 objects: threshold above
    n) is kept (rebuild never).  On tick 1 all objects but five jump far
    east of its frame, where the cell mapping clamps them into the eastern
    leaves.  A query at one of the five: its leaf counts thousands of
    objects, so its square comes from the leaf's farthest corner, and holds
    only the five: fewer than k, so it cannot be proved complete and the
    fallback scan answers it.  Queries at the far objects get squares
    spanning everything.  Every answer equals the brute force."""
    rng = np.random.default_rng(8)
    n = 20000
    x = rng.random(n).astype(np.float32)
    y = rng.random(n).astype(np.float32)
    q = np.arange(0, n, 100, dtype=np.uint32)
    t0 = T(ids=np.arange(n), x=x, y=y, qid=q, rects=(x[q], y[q], x[q], y[q]))
    x1, y1 = x.copy(), y.copy()
    x1[:5] = np.float32(0.9) + np.arange(5, dtype=np.float32) * np.float32(0.01)
    y1[:5] = np.float32(0.9)
    x1[5:] = (np.float32(50.0) + x[5:]).astype(np.float32)
    q1 = np.concatenate([np.arange(5), np.arange(100, n, 500)]).astype(np.uint32)
    t1 = T(ids=np.arange(n), x=x1, y=y1, qid=q1, rects=(x1[q1], y1[q1], x1[q1], y1[q1]))
    st = oracle.State(n)
    sc = Scene(n, len(q), th=1_000_000, rebuild="never", capacity_results=n * len(q))
    fb = []
    for k, t in enumerate((t0, t1)):
        say(f"knn kept frame tick {k}")
        oracle_apply(st, t)
        ids, d2 = gpu_knn(sc, t, t.xa, t.ya, 8)
        check(st, t, t.xa, t.ya, 8, ids, d2, label=f"kept frame tick {k}")
        s = sc.stats()
        fb.append(s["knn_fallback"])
        assert s["rebuilt"] == (1 if k == 0 else 0)
    assert fb[0] == 0 and fb[1] >= 5, fb


@pytest.mark.parametrize("name,n,k", [("hotspot", 200_000, 16), ("segments", 200_000, 8)])
def test_moving_workload_every_query(name, n, k):
    """Two ticks (one that builds the quadtree, one that keeps it) of a
    hotspot and a segment workload: every query against the brute force."""
    wl = workloads.make(name, n=n, n_ticks=2)
    st = oracle.State(wl.n)
    from bench import scene_config
    cfg = scene_config(wl, 64)
    cfg.pop("th", None)
    nq = max(int(0.5 * n), 1)
    sc = Scene(wl.n, nq, th=64, **cfg)
    for i, t in enumerate(wl.ticks()):
        say(f"knn {name} {n} tick {i} k={k} nq={t.nq}")
        oracle_apply(st, t)
        qx, qy = workloads.issuer_points(t)
        ids, d2 = gpu_knn(sc, t, qx, qy, k)
        check(st, t, qx, qy, k, ids, d2, label=f"{name} tick {i}")
        s = sc.stats()
        assert s["rebuilt"] == (1 if i == 0 else 0)
        say(f"  fallback {s['knn_fallback']}")


@pytest.mark.parametrize("name,k", [("hotspot", 16), ("hotspot_20m", 16)])
def test_full_size_sampled(name, k):
    """The full hotspot workloads (1M and 20M objects, 10% of them issuing a
    kNN query per tick): 400 sampled queries of a building tick and of a
    keeping tick against the brute force."""
    wl = workloads.make(name, n_ticks=2)
    st = oracle.State(wl.n)
    from bench import scene_config
    cfg = scene_config(wl, 256)
    cfg.pop("th", None)
    sc = Scene(wl.n, int(0.1 * wl.n), th=256, **cfg)
    rng = np.random.default_rng(11)
    for i, t in enumerate(wl.ticks()):
        say(f"knn {name} tick {i} k={k} nq={t.nq}")
        oracle_apply(st, t)
        qx, qy = workloads.issuer_points(t)
        ids, d2 = gpu_knn(sc, t, qx, qy, k)
        sel = np.sort(rng.choice(t.nq, 400, replace=False))
        check(st, t, qx, qy, k, ids, d2, sel=sel, label=f"{name} tick {i}")
        say(f"  fallback {sc.stats()['knn_fallback']}")
