"""The uniform-grid index (the paper's UG method) on the GPU against the
oracle: the grid cells of the objects, the query split over the grid
(intersecting and covering cells, filtering work), and result sets
identical to the brute force and to the quadtree's (Definition 1)."""
import numpy as np
import pytest

import oracle
from gpu_util import T, gpu_count_hash, gpu_tick, oracle_apply, oracle_count_hash, \
    oracle_lists, say
from paper_1411_3212_amd import workloads
from paper_1411_3212_amd.binding import Scene

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


@pytest.mark.parametrize("s", [1, 7, 64, 110, 1000])
def test_grid_index_split_and_results_equal_oracle(s):
    wl, t, st = c1()
    say(f"uniform grid s={s} c1")
    sc = Scene(wl.n, t.nq, grid_split=s, capacity_subqueries=64 * t.nq,
               capacity_covering=4096 * t.nq)
    gpu_tick(sc, t)
    assert sc.fetch().to_lists() == oracle_lists(st, t)
    # index: objects sorted (stably, by id) by their grid cell
    fr = oracle.frame(st)
    cell = oracle.ug_cells(st, fr, s)
    present = np.nonzero(st.has)[0]
    order = present[np.argsort(cell[present], kind="stable")]
    v = sc.index_view()
    assert (np.float32(v["x0"]), np.float32(v["y0"]), v["e"]) == \
        (np.float32(fr[0]), np.float32(fr[1]), fr[2])
    assert np.array_equal(v["ids"].cpu().numpy().view(np.uint32), order)
    assert np.array_equal(v["codes"].cpu().numpy().view(np.uint32), cell[order])
    b = oracle.ug_bits(s)
    count = np.bincount(cell[present], minlength=1 << (2 * b))
    beg = v["leaf_beg"].cpu().numpy().view(np.uint32)
    assert v["n_leaves"] == 1 << (2 * b)
    assert np.array_equal(np.diff(beg.astype(np.int64)), count)
    # split over the grid and the filtering work
    live = oracle.live_queries(wl.n, t.qid)
    oi, li, oc, lc = oracle.ug_split(live, t.rects, fr, s, count.astype(np.uint32))
    stt = sc.stats()
    assert stt["n_isect"] == len(li) and stt["n_cov"] == len(lc)
    per_cell = np.bincount(li, minlength=len(count))
    assert stt["tests"] == int((per_cell * count).sum())
    assert stt["cov_pairs"] == int(count[lc].sum())
    r = sc.fetch()
    co = r.cov_off.cpu().numpy().view(np.uint32)
    cl = r.cov_leaf.cpu().numpy().view(np.uint32)
    qp = r.query_pos.cpu().numpy().view(np.uint32)
    for k in range(t.nq):
        p = qp[k]
        assert sorted(cl[co[p]:co[p + 1]].tolist()) == sorted(lc[oc[k]:oc[k + 1]].tolist())


@pytest.mark.parametrize("covering,reorder", [(False, True), (True, False)])
def test_grid_results_do_not_depend_on_switches(covering, reorder):
    wl, t, st = c1()
    sc = Scene(wl.n, t.nq, grid_split=37, covering=covering, reorder=reorder,
               capacity_subqueries=64 * t.nq)
    gpu_tick(sc, t)
    assert sc.fetch().to_lists() == oracle_lists(st, t)


def test_grid_edges_and_degenerate_queries():
    # points on the frame's far edges land in the last column / row; zero-area
    # and whole-space queries
    xs = np.array([0.0, 1.0, 1.0, 0.0, 0.5, 0.25, 0.75, 0.999999], np.float32)
    ys = np.array([0.0, 1.0, 0.0, 1.0, 0.5, 0.75, 0.25, 0.999999], np.float32)
    n = len(xs)
    q = [(0.0, 0.0, 0.0, 0.0), (-1, -1, 2, 2), (0.5, 0.5, 0.5, 0.5), (0.2, 0.2, 0.8, 0.8),
         (0.9, 0.9, 1.0, 1.0)]
    t = T(ids=range(n), x=xs, y=ys, qid=range(len(q)),
          rects=tuple(np.array(q)[:, c].astype(np.float32) for c in range(4)))
    st = oracle.State(n)
    oracle_apply(st, t)
    want = oracle_lists(st, t)
    for s in (1, 3, 110, 4096):
        sc = Scene(n, len(q), grid_split=s, capacity_covering=1 << 26)
        gpu_tick(sc, t)
        assert sc.fetch().to_lists() == want, s


@pytest.mark.parametrize("s", [95, 110])
def test_grid_hotspot_1m_equals_oracle_and_quadtree(s):
    """1M hotspot objects, 100K queries per tick, two ticks: every query by
    count + hash against the CPU grid and against the quadtree's results,
    300 sampled queries by lists against the brute force."""
    from bench import scene_config
    wl = workloads.make("hotspot", n_ticks=2)
    st = oracle.State(wl.n)
    cfg = scene_config(wl)
    ug = Scene(wl.n, int(0.1 * wl.n), grid_split=s,
               **{k: v for k, v in cfg.items() if k not in ("th", "split_slots")})
    quad = Scene(wl.n, int(0.1 * wl.n), **cfg)
    rng = np.random.default_rng(s)
    for k, t in enumerate(wl.ticks()):
        say(f"grid s={s} hotspot 1M tick {k}")
        oracle_apply(st, t)
        gpu_tick(ug, t)
        gpu_tick(quad, t)
        cnt, h = gpu_count_hash(ug)
        oc, oh = oracle_count_hash(st, t, grid=True)
        assert np.array_equal(cnt, oc) and np.array_equal(h, oh)
        qc, qh = gpu_count_hash(quad)
        assert np.array_equal(cnt, qc) and np.array_equal(h, qh)
        sample = np.sort(rng.choice(t.nq, 300, replace=False)).astype(np.uint32)
        sub = T(qid=t.qid[sample], rects=tuple(r[sample] for r in t.rects))
        assert ug.fetch().to_lists(sel=sample) == oracle_lists(st, sub)
        say(f"  {ug.stats()['n_isect']} intersecting, {ug.stats()['n_cov']} covering subqueries")
