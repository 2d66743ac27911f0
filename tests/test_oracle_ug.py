"""Pins of the oracle's uniform grid (the UG method: Definition "MBR
partitioning into a uniform grid", UG index creation and query indexing,
equation nr_isect) against closed forms, the quadtree split of a complete
tree, and brute force."""
import numpy as np
import pytest

import oracle
from test_oracle import rects_of, state_from

F32 = np.float32


@pytest.mark.parametrize("b", [1, 3, 7, 10, 16])
def test_power_of_two_split_factor_is_the_complete_quadtree_level(b):
    # with s = 2^b columns the grid is the quadtree's level b: the column of
    # a finest cell is its top b bits
    f = np.arange(0, 65536, 7, dtype=np.int64)
    got = [oracle.ug_col(int(v), 1 << b) for v in f]
    assert got == (f >> (16 - b)).tolist()
    assert oracle.ug_bits(1 << b) == b


@pytest.mark.parametrize("s", [1, 3, 95, 110, 1000, 40000, 65535, 65536])
def test_columns_partition_the_frame_into_nearly_equal_widths(s):
    cols = np.array([oracle.ug_col(v, s) for v in range(65536)])
    assert cols[0] == 0 and cols[-1] == s - 1
    assert (np.diff(cols) >= 0).all() and (np.diff(cols) <= 1).all()  # monotone, no gaps
    width = np.bincount(cols, minlength=s)
    assert set(width.tolist()) <= {65536 // s, -(-65536 // s)}  # floor or ceil of 2^16 / s
    assert width.sum() == 65536
    assert (1 << oracle.ug_bits(s)) >= s > (1 << oracle.ug_bits(s)) >> 1 or s == 1


def test_cells_are_columns_and_rows_interleaved():
    rng = np.random.default_rng(3)
    xs, ys = rng.random(500), rng.random(500)
    xs[:4] = [0.0, 1.0, 0.5, 0.25]
    ys[:4] = [0.0, 1.0, 0.25, 0.5]
    st = state_from(xs, ys, present=np.arange(500) % 7 != 3)
    fr = oracle.frame(st)
    s = 110
    cell = oracle.ug_cells(st, fr, s)
    b = oracle.ug_bits(s)
    for j in range(500):
        if not st.has[j]:
            assert cell[j] == 0xffffffff
            continue
        ci = oracle.ug_col(oracle.cell(float(st.px[j]), fr[0], fr[2]), s)
        cj = oracle.ug_col(oracle.cell(float(st.py[j]), fr[1], fr[2]), s)
        assert cell[j] == oracle.morton(ci, cj, b)
        assert ci < s and cj < s


def test_split_counts_are_the_cell_range_when_every_cell_is_occupied():
    s = 37
    b = oracle.ug_bits(s)
    count = np.ones(1 << (2 * b), np.uint32)
    rng = np.random.default_rng(5)
    c = rng.random((300, 2))
    w = rng.random((300, 2)) * 0.3
    rects = rects_of(np.c_[c - w / 2, c + w / 2])
    fr = (0.0, 0.0, 0)
    oi, li, oc, lc = oracle.ug_split(np.ones(300, np.uint8), rects, fr, s, count)
    for k in range(300):
        i0, i1 = (oracle.ug_col(oracle.cell(float(rects[0][k]), 0.0, 0), s),
                  oracle.ug_col(oracle.cell(float(rects[2][k]), 0.0, 0), s))
        j0, j1 = (oracle.ug_col(oracle.cell(float(rects[1][k]), 0.0, 0), s),
                  oracle.ug_col(oracle.cell(float(rects[3][k]), 0.0, 0), s))
        n_all = (i1 - i0 + 1) * (j1 - j0 + 1)
        n_cov = max(0, i1 - i0 - 1) * max(0, j1 - j0 - 1)
        assert oc[k + 1] - oc[k] == n_cov
        assert (oi[k + 1] - oi[k]) + (oc[k + 1] - oc[k]) == n_all
        cells = li[oi[k]:oi[k + 1]].tolist() + lc[oc[k]:oc[k + 1]].tolist()
        assert len(set(cells)) == len(cells)


@pytest.mark.parametrize("b", [2, 5])
def test_power_of_two_grid_split_equals_the_quadtree_split_of_the_complete_tree(b):
    # leaves = every level-b cell in Morton order: the quadtree split (pinned
    # by the paper's mapping example) must name the same cells
    n = 1 << (2 * b)
    lv = oracle.Leaves(np.full(n, b, np.uint32), np.arange(n, dtype=np.uint32),
                       np.zeros(n, np.uint32), np.zeros(n, np.uint32), b)
    rng = np.random.default_rng(b)
    c = rng.random((200, 2)) * 1.2 - 0.1
    w = rng.random((200, 2)) * 0.4
    rects = rects_of(np.c_[c - w / 2, c + w / 2])
    fr = (0.0, 0.0, 0)
    live = np.ones(200, np.uint8)
    qi, qli, qc, qlc = oracle.split(live, rects, fr, lv)
    ui, uli, uc, ulc = oracle.ug_split(live, rects, fr, 1 << b, np.ones(n, np.uint32))
    for k in range(200):
        assert sorted(uli[ui[k]:ui[k + 1]].tolist()) == sorted(qli[qi[k]:qi[k + 1]].tolist())
        assert sorted(ulc[uc[k]:uc[k + 1]].tolist()) == sorted(qlc[qc[k]:qc[k + 1]].tolist())


@pytest.mark.parametrize("s", [1, 10, 95, 300])
def test_union_over_grid_cells_is_the_brute_force_result(s):
    wl = __import__("paper_1411_3212_amd").workloads.make("hotspot", n=20_000, n_ticks=1)
    t = next(wl.ticks())
    st = oracle.State(wl.n)
    oracle.apply_updates(st, t.ids, t.x, t.y)
    live = oracle.live_queries(wl.n, t.qid)
    fr = oracle.frame(st)
    cell = oracle.ug_cells(st, fr, s)
    b = oracle.ug_bits(s)
    count = np.bincount(cell[st.has == 1], minlength=1 << (2 * b)).astype(np.uint32)
    oi, li, oc, lc = oracle.ug_split(live, t.rects, fr, s, count)
    boff, bids = oracle.brute_lists(st, live, t.rects)
    order = np.argsort(cell, kind="stable")
    beg = np.searchsorted(cell[order], np.arange((1 << (2 * b)) + 1))
    xa, ya, xb, yb = t.rects
    for k in range(0, t.nq, 7):
        got = []
        for z in li[oi[k]:oi[k + 1]]:
            ids = order[beg[z]:beg[z + 1]]
            inside = (xa[k] <= st.px[ids]) & (st.px[ids] <= xb[k]) & \
                     (ya[k] <= st.py[ids]) & (st.py[ids] <= yb[k])
            got.extend(ids[inside].tolist())
        for z in lc[oc[k]:oc[k + 1]]:
            ids = order[beg[z]:beg[z + 1]]
            # covering soundness: every object of a covering cell is inside
            assert ((xa[k] <= st.px[ids]) & (st.px[ids] <= xb[k]) &
                    (ya[k] <= st.py[ids]) & (st.py[ids] <= yb[k])).all()
            got.extend(ids.tolist())
        assert len(got) == len(set(got))
        assert sorted(got) == bids[boff[k]:boff[k + 1]].tolist()


@pytest.mark.parametrize("cells", [10.3, 40.3])
def test_subquery_counts_follow_equation_nr_isect_on_uniform_data(cells):
    # uniform objects, squares of side `cells` grid cells: intersecting
    # subqueries about perimeter / cell side; covering ones about area /
    # cell side^2 minus the intersecting ones, which holds once the query
    # spans many cells (it leaves out the one extra row and column a square
    # touches: 25% low at 10 cells, 5% at 40)
    rng = np.random.default_rng(4)
    fr = (0.0, 0.0, 0)
    s = 100 if cells < 20 else 400
    count = np.ones(1 << (2 * oracle.ug_bits(s)), np.uint32)  # dense data: every cell occupied
    side = cells / s
    c = (0.5 * side + 0.01) + (1 - side - 0.02) * rng.random((400, 2))
    rects = rects_of(np.c_[c - side / 2, c + side / 2])
    oi, li, oc, lc = oracle.ug_split(np.ones(400, np.uint8), rects, fr, s, count)
    cs = 1.0 / s
    pi = 400 * 4 * side / cs
    pc = 400 * side * side / cs**2 - pi
    assert abs(len(li) - pi) / pi < 0.10
    if cells > 20:
        assert abs(len(lc) - pc) / pc < 0.10
