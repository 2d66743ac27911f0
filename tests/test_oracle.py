"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each check is chosen so that a plausible mistake in the oracle (a dropped
term, a wrong comparison or index, a transposed operand) fails one of them:
published hash values, the paper's worked examples (counts reproduced on
constructed layouts), closed forms, brute force in plain Python on tiny
inputs, a textbook recursive quadtree, the paper's own lookup-table query
enumeration, and invariants (union over leaves = brute force, disjointness,
covering soundness).
"""
import numpy as np
import pytest

import oracle
from conftest import read_golden
from paper_1411_3212_amd import workloads

F32 = np.float32


# ----------------------------------------------------------------- helpers

def state_from(xs, ys, present=None):
    st = oracle.State(len(xs))
    ids = np.arange(len(xs), dtype=np.uint32)
    if present is not None:
        ids = ids[np.asarray(present, bool)]
    oracle.apply_updates(st, ids, np.asarray(xs, F32)[ids], np.asarray(ys, F32)[ids])
    return st


def py_brute(px, py, has, rects, live):
    """Definition 1 in plain Python: closed rectangle, present objects only."""
    xa, ya, xb, yb = rects
    out = []
    for k in range(len(xa)):
        res = []
        if live[k]:
            for j in range(len(px)):
                if has[j] and xa[k] <= px[j] <= xb[k] and ya[k] <= py[j] <= yb[k]:
                    res.append(j)
        out.append(res)
    return out


def as_lists(off, ids):
    return [list(map(int, ids[off[k]:off[k + 1]])) for k in range(len(off) - 1)]


def rects_of(qs):
    qs = np.asarray(qs, np.float64).reshape(-1, 4)
    return tuple(qs[:, c].astype(F32) for c in range(4))


def demorton_py(z, nbits):
    i = j = 0
    for b in range(nbits):
        i |= ((z >> (2 * b)) & 1) << b
        j |= ((z >> (2 * b + 1)) & 1) << b
    return i, j


# ------------------------------------------------------------------- hash

def test_mix64_matches_published_splitmix64_outputs():
    with open(__import__("conftest").GOLDEN + "/splitmix64_seed0.txt") as f:
        pairs = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    gamma = 0x9E3779B97F4A7C15
    for k, (state, out) in enumerate(pairs):
        assert int(state, 16) == ((k + 1) * gamma) % 2**64
        assert oracle.mix64(int(state, 16)) == int(out, 16)


def test_pair_set_hash_is_sum_of_mix64_over_pairs():
    rng = np.random.default_rng(11)
    xs, ys = rng.random(300), rng.random(300)
    st = state_from(xs, ys)
    qid = np.array([5, 17, 250], np.uint32)
    rects = rects_of([[0.1, 0.1, 0.5, 0.5], [0, 0, 1, 1], [0.7, 0.2, 0.75, 0.9]])
    live = np.ones(3, np.uint8)
    cnt, h = oracle.brute_hash(st, qid, live, rects)
    ref = py_brute(st.px, st.py, st.has, rects, live)
    for k in range(3):
        assert cnt[k] == len(ref[k])
        want = sum(oracle.mix64((int(qid[k]) << 32) | j) for j in ref[k]) % 2**64
        assert int(h[k]) == want
    assert cnt[1] == 300  # the unit square holds every object


# ------------------------------------------------------ updates and queries

def test_latest_update_wins_and_invalid_updates_are_skipped():
    st = oracle.State(4)
    bad = oracle.apply_updates(st, [1, 2, 1, 7, 3], [0.1, 0.2, 0.3, 0.4, np.nan],
                               [0.5, 0.6, 0.7, 0.8, 0.9])
    assert bad == 2  # id 7 >= N, NaN coordinate
    assert st.has.tolist() == [0, 1, 1, 0]
    assert st.px[1] == F32(0.3) and st.py[1] == F32(0.7)
    # a later batch overwrites, an object without update keeps its position
    oracle.apply_updates(st, [2], [0.25], [0.65])
    assert st.px[2] == F32(0.25) and st.px[1] == F32(0.3)


def test_latest_query_of_an_object_is_the_live_one():
    live = oracle.live_queries(10, [3, 4, 3, 9, 4, 3])
    assert live.tolist() == [0, 0, 0, 1, 1, 1]


# ------------------------------------------------------------ Definition 1

def test_result_set_example_includes_the_issuer(golden):
    keys, rows = golden("result_set_example.txt")
    st = oracle.State(4)
    rows = np.array(rows)
    oracle.apply_updates(st, rows[:, 0].astype(np.uint32), rows[:, 1], rows[:, 2])
    q = keys["query"]
    rects = rects_of([[float(v) for v in q[1:]]])
    off, ids = oracle.brute_lists(st, np.ones(1, np.uint8), rects)
    assert ids.tolist() == [int(v) for v in keys["result"]]
    assert int(q[0]) in ids.tolist()


def test_closed_rectangle_edges_corners_and_just_outside():
    xa, ya, xb, yb = F32(0.25), F32(0.25), F32(0.75), F32(0.5)
    nxt = np.nextafter
    pts = [
        (xa, ya), (xb, yb), (xa, yb), (xb, ya),            # corners: in
        (xa, F32(0.3)), (xb, F32(0.3)), (F32(0.5), ya), (F32(0.5), yb),  # edges: in
        (nxt(xa, F32(-1)), F32(0.3)), (nxt(xb, F32(2)), F32(0.3)),       # just outside
        (F32(0.5), nxt(ya, F32(-1))), (F32(0.5), nxt(yb, F32(2))),
    ]
    st = state_from([p[0] for p in pts], [p[1] for p in pts])
    off, ids = oracle.brute_lists(st, np.ones(1, np.uint8), rects_of([[xa, ya, xb, yb]]))
    assert ids.tolist() == list(range(8))


def test_signed_zero_zero_area_whole_and_disjoint_queries():
    st = state_from([0.0, -0.0, 0.5, 1.0], [0.0, 0.0, 0.5, 1.0])
    rects = rects_of([
        [-0.0, -0.0, 0.0, 0.0],      # +0 and -0 compare equal: both zeros in
        [0.5, 0.5, 0.5, 0.5],        # zero-area query: exactly that point
        [-1, -1, 2, 2],              # covers everything
        [2, 2, 3, 3],                # disjoint from every object
        [0.6, 0.0, 0.4, 1.0],        # inverted: empty
    ])
    off, ids = oracle.brute_lists(st, np.ones(5, np.uint8), rects)
    assert as_lists(off, ids) == [[0, 1], [2], [0, 1, 2, 3], [], []]


def test_empty_inputs_and_absent_objects():
    st = oracle.State(5)
    off, ids = oracle.brute_lists(st, np.ones(1, np.uint8), rects_of([[-1, -1, 2, 2]]))
    assert as_lists(off, ids) == [[]]
    st = state_from([0.1, 0.2, 0.3], [0.1, 0.2, 0.3], present=[1, 0, 1])
    off, ids = oracle.brute_lists(st, np.ones(1, np.uint8), rects_of([[0, 0, 1, 1]]))
    assert as_lists(off, ids) == [[0, 2]]
    off, ids = oracle.brute_lists(st, np.zeros(0, np.uint8), rects_of(np.zeros((0, 4))))
    assert len(off) == 1 and len(ids) == 0


def test_superseded_query_has_empty_result():
    st = state_from([0.5], [0.5])
    qid = [0, 0]
    live = oracle.live_queries(1, qid)
    off, ids = oracle.brute_lists(st, live, rects_of([[0, 0, 1, 1], [0, 0, 1, 1]]))
    assert as_lists(off, ids) == [[], [0]]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_brute_force_equals_plain_python_loop(seed):
    rng = np.random.default_rng(seed)
    n, nq = 200, 40
    xs = rng.random(n).astype(F32)
    ys = rng.random(n).astype(F32)
    xs[:10] = F32(0.5)  # ties on query edges
    present = rng.random(n) < 0.9
    st = state_from(xs, ys, present)
    c = rng.random((nq, 2))
    s = rng.random((nq, 2)) * 0.3
    rects = rects_of(np.c_[c - s, c + s])
    rects[0][:5] = F32(0.5)
    qid = rng.integers(0, n, nq).astype(np.uint32)
    live = oracle.live_queries(n, qid)
    off, ids = oracle.brute_lists(st, live, rects)
    assert as_lists(off, ids) == py_brute(st.px, st.py, st.has, rects, live)


def test_grid_oracle_equals_brute_force_on_workloads():
    wl = workloads.make("uniform_1tick")
    t = next(wl.ticks())
    st = oracle.State(wl.n)
    oracle.apply_updates(st, t.ids, t.x, t.y)
    live = oracle.live_queries(wl.n, t.qid)
    cb, hb = oracle.brute_hash(st, t.qid, live, t.rects)
    cg, hg = oracle.grid_hash(st, t.qid, live, t.rects)
    assert np.array_equal(cb, cg) and np.array_equal(hb, hg)
    assert cb.min() >= 1  # issuer always in its own result
    for name in ("hotspot", "segments"):
        wl = workloads.make(name, n=60_000, n_ticks=2)
        st = oracle.State(wl.n)
        for t in wl.ticks():
            oracle.apply_updates(st, t.ids, t.x, t.y)
            live = oracle.live_queries(wl.n, t.qid)
            cb, hb = oracle.brute_hash(st, t.qid, live, t.rects)
            cg, hg = oracle.grid_hash(st, t.qid, live, t.rects)
            assert np.array_equal(cb, cg) and np.array_equal(hb, hg)
            assert cb.min() >= 1


# ------------------------------------------------- frame and cell mapping

@pytest.mark.parametrize("ext,e", [(0.75, 0), (1.0, 0), (1.5, 1), (0.5, -1), (0.3, -1),
                                   (3.0, 2), (2.0 ** -20, -20)])
def test_frame_side_is_smallest_power_of_two_covering_the_extent(ext, e):
    st = state_from([0.25, 0.25 + ext], [0.5, 0.5 + ext / 2])
    x0, y0, ee, n = oracle.frame(st)
    assert (x0, y0, ee, n) == (F32(0.25), F32(0.5), e, 2)


def test_frame_of_a_single_point_and_of_nothing():
    assert oracle.frame(state_from([0.3], [0.7]))[2] == -100
    assert oracle.frame(oracle.State(3)) == (0.0, 0.0, 0, 0)


def test_cell_mapping_closed_forms():
    # on the unit frame, k / 2^16 lies exactly at the start of cell k
    for k in [0, 1, 2, 12345, 32768, 65534, 65535]:
        assert oracle.cell(k / 65536.0, 0.0, 0) == k
        if k:
            assert oracle.cell(float(np.nextafter(F32(k / 65536.0), F32(0))), 0.0, 0) == k - 1
    assert oracle.cell(1.0, 0.0, 0) == 65535       # clamped to the last cell
    assert oracle.cell(-0.5, 0.0, 0) == 0          # clamped to the first cell
    assert oracle.cell(1e30, 0.0, 0) == 65535
    assert oracle.cell(0.75, 0.5, -1) == 32768     # frame [0.5, 1): (0.25) * 2^17
    assert oracle.cell(3.0, 2.0, 1) == 32768       # frame [2, 4)


def test_cell_mapping_is_monotone():
    rng = np.random.default_rng(5)
    v = np.sort(np.concatenate([rng.random(2000) * 1.4 - 0.2,
                                np.linspace(0.3, 0.3000001, 50)]).astype(F32))
    c = [oracle.cell(float(a), 0.1, 0) for a in v]
    assert all(a <= b for a, b in zip(c, c[1:]))


def test_morton_closed_forms():
    assert oracle.morton(1, 0) == 1 and oracle.morton(0, 1) == 2
    assert oracle.morton(3, 3) == 15
    assert oracle.morton(0xFFFF, 0) == 0x55555555
    assert oracle.morton(0, 0xFFFF) == 0xAAAAAAAA
    rng = np.random.default_rng(3)
    for i, j in rng.integers(0, 65536, (50, 2)):
        bi, bj = format(int(i), "016b"), format(int(j), "016b")
        want = int("".join(b + a for a, b in zip(bi, bj)), 2)
        assert oracle.morton(int(i), int(j)) == want


# ------------------------------------------------------------ Algorithm 1

def textbook_quadtree(ci, cj, th, l_max):
    """Recursive PR-quadtree: a quadrant with more than th objects below
    level l_max is split into four; every other quadrant is a leaf."""
    leaves = []

    def rec(l, zi, zj, objs):
        s = 16 - (l + 1)
        for dj in (0, 1):
            for di in (0, 1):
                ti, tj = 2 * zi + di, 2 * zj + dj
                sub = [o for o in objs if (ci[o] >> s) == ti and (cj[o] >> s) == tj]
                if len(sub) > th and l + 1 < l_max:
                    rec(l + 1, ti, tj, sub)
                else:
                    leaves.append((l + 1, ti, tj, len(sub)))

    rec(0, 0, 0, list(range(len(ci))))
    return sorted(leaves)


def oracle_tree(st, th, l_max):
    fr = oracle.frame(st)
    codes, ids = oracle.sorted_codes(st, fr)
    return fr, codes, ids, oracle.quadtree(codes, th, l_max)


def leaf_tuples(lv):
    out = []
    for l, z, c in zip(lv.lvl, lv.z, lv.count):
        i, j = demorton_py(int(z), int(l))
        out.append((int(l), i, j, int(c)))
    return sorted(out)


def test_quadtree_construction_example(golden):
    keys, rows = golden("quadtree_construction_example.txt")
    rows = np.array(rows)
    st = state_from(rows[:, 0], rows[:, 1])
    fr, codes, ids, lv = oracle_tree(st, int(keys["th"][0]), int(keys["l_max"][0]))
    assert fr[:3] == (0.0, 0.0, 0)
    assert len(lv) == int(keys["leaves"][0])
    assert int((lv.lvl == 2).sum()) == int(keys["leaves_level2"][0])
    assert sorted(lv.z[lv.lvl == 1].tolist()) == [int(v) for v in keys["level1_leaf_codes"]]
    assert lv.l_deep == int(keys["l_deep"][0])
    # each level-1 leaf spans 4 cells of the level-l_deep grid
    for z in lv.z[lv.lvl == 1]:
        i, j = demorton_py(int(z), 1)
        cells = [(a, b) for a in range(4) for b in range(4) if (a >> 1, b >> 1) == (i, j)]
        assert len(cells) == 4


@pytest.mark.parametrize("seed,th,l_max", [(0, 1, 16), (1, 3, 16), (2, 8, 5), (3, 1, 3),
                                           (4, 20, 16), (5, 2, 16)])
def test_quadtree_equals_textbook_recursion(seed, th, l_max):
    rng = np.random.default_rng(seed)
    n = 300
    pts = np.concatenate([rng.random((n // 2, 2)),
                          0.3 + 0.01 * rng.standard_normal((n - n // 2, 2))])
    pts[:12] = (0.3, 0.3)  # duplicates: more than th at the finest level
    st = state_from(pts[:, 0], pts[:, 1])
    fr, codes, ids, lv = oracle_tree(st, th, l_max)
    ci = [oracle.cell(float(x), fr[0], fr[2]) for x in st.px]
    cj = [oracle.cell(float(y), fr[1], fr[2]) for y in st.py]
    assert leaf_tuples(lv) == textbook_quadtree(ci, cj, th, l_max)


def test_quadtree_invariants_on_workload():
    wl = workloads.make("hotspot", n=50_000, n_ticks=1)
    t = next(wl.ticks())
    st = oracle.State(wl.n)
    oracle.apply_updates(st, t.ids, t.x, t.y)
    for th in (16, 64, 384):
        fr, codes, ids, lv = oracle_tree(st, th, 16)
        start = lv.start
        size = np.uint64(1) << (np.uint64(2) * (np.uint64(16) - lv.lvl.astype(np.uint64)))
        assert start[0] == 0 and int(start[-1] + size[-1]) == 2**32   # partition of Z-space
        assert np.array_equal(start[1:], start[:-1] + size[:-1])
        assert np.array_equal(lv.beg[1:], lv.end[:-1]) and lv.end[-1] == wl.n
        assert (lv.count[lv.lvl < 16] <= th).all()
        # objects of a leaf are exactly the sorted codes inside its Z-interval
        assert np.array_equal(lv.beg, np.searchsorted(codes, start, side="left"))
        assert np.array_equal(np.sort(ids), np.arange(wl.n))


def test_quadtree_duplicates_stop_at_l_max():
    st = state_from([0.2] * 10 + [0.9], [0.2] * 10 + [0.9])
    fr, codes, ids, lv = oracle_tree(st, 4, 16)
    assert lv.count.max() == 10 and lv.lvl[np.argmax(lv.count)] == 16
    assert lv.l_deep == 16


def test_quadtree_of_no_objects_is_the_four_root_quadrants():
    lv = oracle.quadtree(np.zeros(0, np.uint32), 4, 16)
    assert len(lv) == 4 and (lv.count == 0).all() and lv.l_deep == 1


# ---------------------------------------------------------- query splitting

def test_query_split_example(golden):
    keys, rows = golden("query_split_example.txt")
    rows = np.array(rows)
    st = state_from(rows[:, 0], rows[:, 1])
    fr, codes, ids, lv = oracle_tree(st, int(keys["th"][0]), int(keys["l_max"][0]))
    rects = rects_of([[float(v) for v in keys["query"]]])
    oi, li, oc, lc = oracle.split(np.ones(1, np.uint8), rects, fr, lv)
    assert len(li) + len(lc) == int(keys["subqueries"][0])
    assert len(li) == int(keys["intersecting"][0]) and len(lc) == int(keys["covering"][0])
    issuer = int(keys["issuer"][0])
    pos = int(np.nonzero(ids == issuer)[0][0])
    assert lv.beg[lc[0]] <= pos < lv.end[lc[0]]   # the issuer's own leaf is covered


def zmap_split(lv, fr, rect):
    """The paper's query indexing: enumerate the level-l_deep cells under the
    (clipped) query, map each through the Morton-ordered lookup table z_map
    to its leaf, and keep one subquery per leaf (the cell with minimal grid
    coordinates)."""
    ld = lv.l_deep
    zmap = {}
    for t, (l, z) in enumerate(zip(lv.lvl, lv.z)):
        i, j = demorton_py(int(z), int(l))
        s = ld - int(l)
        for di in range(1 << s):
            for dj in range(1 << s):
                zmap[((i << s) + di, (j << s) + dj)] = t
    sh = 16 - ld
    i0, i1 = oracle.cell(rect[0], fr[0], fr[2]) >> sh, oracle.cell(rect[2], fr[0], fr[2]) >> sh
    j0, j1 = oracle.cell(rect[1], fr[1], fr[2]) >> sh, oracle.cell(rect[3], fr[1], fr[2]) >> sh
    seen = {}
    for j in range(j0, j1 + 1):
        for i in range(i0, i1 + 1):
            t = zmap[(i, j)]
            if t not in seen:
                seen[t] = (i, j)
    return sorted(seen)


def test_split_matches_lookup_table_enumeration_without_duplicates():
    rng = np.random.default_rng(8)
    pts = np.concatenate([rng.random((150, 2)), 0.6 + 0.02 * rng.standard_normal((150, 2))])
    st = state_from(np.clip(pts[:, 0], 0, 1), np.clip(pts[:, 1], 0, 1))
    fr, codes, ids, lv = oracle_tree(st, 4, 7)
    c = rng.random((60, 2))
    s = rng.random((60, 2)) * 0.25
    q = np.c_[c - s, c + s]
    rects = rects_of(q)
    oi, li, oc, lc = oracle.split(np.ones(60, np.uint8), rects, fr, lv)
    for k in range(60):
        mine = sorted(li[oi[k]:oi[k + 1]].tolist() + lc[oc[k]:oc[k + 1]].tolist())
        assert len(set(mine)) == len(mine)
        rk = [float(rects[c_][k]) for c_ in range(4)]
        assert mine == zmap_split(lv, fr, rk)


@pytest.mark.parametrize("name,th", [("uniform_1tick", 64), ("hotspot", 16), ("hotspot", 384),
                                     ("segments", 64)])
def test_union_over_leaves_equals_brute_force(name, th):
    wl = workloads.make(name) if name == "uniform_1tick" else workloads.make(name, n=40_000,
                                                                            n_ticks=1)
    t = next(wl.ticks())
    st = oracle.State(wl.n)
    oracle.apply_updates(st, t.ids, t.x, t.y)
    live = oracle.live_queries(wl.n, t.qid)
    fr, codes, ids, lv = oracle_tree(st, th, 16)
    oi, li, oc, lc = oracle.split(live, t.rects, fr, lv)
    sx, sy = st.px[ids], st.py[ids]
    off, bids = oracle.brute_lists(st, live, t.rects)
    tests = 0
    for k in range(t.nq):
        xa, ya, xb, yb = (r[k] for r in t.rects)
        got = []
        for leaf in li[oi[k]:oi[k + 1]]:
            b, e = lv.beg[leaf], lv.end[leaf]
            tests += e - b
            m = (xa <= sx[b:e]) & (sx[b:e] <= xb) & (ya <= sy[b:e]) & (sy[b:e] <= yb)
            got.extend(ids[b:e][m].tolist())
        for leaf in lc[oc[k]:oc[k + 1]]:
            b, e = lv.beg[leaf], lv.end[leaf]
            inside = (xa <= sx[b:e]) & (sx[b:e] <= xb) & (ya <= sy[b:e]) & (sy[b:e] <= yb)
            assert inside.all()  # covering soundness
            got.extend(ids[b:e].tolist())
        assert len(got) == len(set(got))  # per-leaf lists are disjoint
        assert sorted(got) == bids[off[k]:off[k + 1]].tolist()
    # the filtering work is sum over leaves of |intersecting subqueries| x |objects|
    per_leaf = np.bincount(li, minlength=len(lv))
    assert tests == int((per_leaf * lv.count).sum())


def test_intersecting_subquery_count_follows_perimeter_over_cell_side():
    # a 128 x 128 lattice with th = 1 makes the quadtree a uniform grid of
    # side 1/128; squares of side s then give about 4 s / side intersecting
    # subqueries each (cost model for uniform distributions).
    g = (np.arange(128) + 0.5) / 128
    X, Y = np.meshgrid(g, g)
    xs = np.r_[0.0, X.ravel(), 1.0 - 2**-20]
    ys = np.r_[0.0, Y.ravel(), 1.0 - 2**-20]
    st = state_from(xs, ys)
    fr, codes, ids, lv = oracle_tree(st, 1, 7)
    rng = np.random.default_rng(2)
    c = 0.2 + 0.6 * rng.random((200, 2))
    side = 12.3 / 128
    rects = rects_of(np.c_[c - side / 2, c + side / 2])
    oi, li, oc, lc = oracle.split(np.ones(200, np.uint8), rects, fr, lv)
    predicted = 200 * 4 * side / (1 / 128)
    assert abs(len(li) - predicted) / predicted < 0.10


def test_split_with_query_corners_on_leaf_edge_cells():
    # corners placed in the first and the last finest-level cell of leaves:
    # the leaf owning that cell must be split off exactly once
    rng = np.random.default_rng(9)
    pts = np.concatenate([rng.random((200, 2)), 0.4 + 0.03 * rng.standard_normal((200, 2))])
    pts = np.clip(pts, 0.0, 1.0)
    pts[0] = (0.0, 0.0)
    pts[1] = (0.999, 0.999)
    st = state_from(pts[:, 0], pts[:, 1])
    fr, codes, ids, lv = oracle_tree(st, 3, 8)
    assert fr[:3] == (0.0, 0.0, 0)
    qs = []
    for t in rng.integers(0, len(lv), 80):
        i, j = demorton_py(int(lv.z[t]), int(lv.lvl[t]))
        s = 16 - int(lv.lvl[t])
        ilo, ihi = i << s, ((i + 1) << s) - 1
        jlo, jhi = j << s, ((j + 1) << s) - 1
        w = rng.integers(0, 3000, 2) / 65536
        # lower-left corner in the leaf's last cell / upper-right in its first
        qs.append([(ihi + 0.5) / 65536, (jhi + 0.5) / 65536,
                   (ihi + 0.5) / 65536 + w[0], (jhi + 0.5) / 65536 + w[1]])
        qs.append([(ilo + 0.5) / 65536 - w[0], (jlo + 0.5) / 65536 - w[1],
                   (ilo + 0.5) / 65536, (jlo + 0.5) / 65536])
    rects = rects_of(qs)
    oi, li, oc, lc = oracle.split(np.ones(len(qs), np.uint8), rects, fr, lv)
    for k in range(len(qs)):
        mine = sorted(li[oi[k]:oi[k + 1]].tolist() + lc[oc[k]:oc[k + 1]].tolist())
        rk = [float(rects[c_][k]) for c_ in range(4)]
        assert mine == zmap_split(lv, fr, rk)
