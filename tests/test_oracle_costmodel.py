"""Pins of the oracle of the learned threshold choice: the overlap feature
and the leaf geometry in closed form, the features of a hand-built scene,
and the cost of a network whose output is constant."""
import numpy as np
import pytest

import oracle
from oracle import costmodel, mlp


def test_overlap_fraction_closed_forms():
    lx, ly, s = np.array([0.0]), np.array([0.0]), np.array([2.0])
    f = lambda *r: float(costmodel.overlap_fraction(r, lx, ly, s)[0])
    assert f(-1, -1, 1, 3) == 0.5          # left half
    assert f(-1, -1, 3, 3) == 1.0          # contains the leaf
    assert f(0.5, 0.5, 1.5, 1.5) == 0.25   # centred square of half the side
    assert f(2.0, 0.0, 3.0, 1.0) == 0.0    # touches the right edge only
    assert f(0.0, 0.0, 0.0, 2.0) == 0.0    # degenerate (zero width)
    assert f(1.0, 1.0, 5.0, 1.5) == 0.125  # half of the width x a quarter of the height


def test_leaf_geometry_closed_form():
    st = oracle.State(3)
    oracle.apply_updates(st, np.arange(3, dtype=np.uint32), np.array([0.0, 0.9, 0.3], np.float32),
                         np.array([0.0, 0.9, 0.6], np.float32))
    fr = oracle.frame(st)
    assert (float(fr[0]), float(fr[1]), int(fr[2])) == (0.0, 0.0, 0)
    # level 1 leaves in Morton order: (0,0) (1,0) (0,1) (1,1); level 2 code 5 =
    # x 0b11, y 0b00
    lv = oracle.Leaves(np.array([1, 1, 1, 1, 2], np.uint32), np.array([0, 1, 2, 3, 5], np.uint32),
                       np.zeros(5, np.uint32), np.zeros(5, np.uint32), 2)
    x, y, s = costmodel.leaf_geometry(fr, lv)
    assert list(x) == [0.0, 0.5, 0.0, 0.5, 0.75] and list(y) == [0.0, 0.0, 0.5, 0.5, 0.0]
    assert list(s) == [0.5, 0.5, 0.5, 0.5, 0.25]


def hand_scene():
    """Five objects in a unit frame, threshold 2: four level-1 leaves (BL 2
    objects, BR 1, TL 0, TR 2); one query [0.25, 0.75] x [0, 0.5]."""
    x = np.array([0.0, 0.1, 0.7, 0.9, 0.6], np.float32)
    y = np.array([0.0, 0.1, 0.2, 0.9, 0.6], np.float32)
    st = oracle.State(5)
    oracle.apply_updates(st, np.arange(5, dtype=np.uint32), x, y)
    rects = tuple(np.array([v], np.float32) for v in (0.25, 0.0, 0.75, 0.5))
    live = oracle.live_queries(5, np.array([0], np.uint32))
    return st, live, rects


def test_features_of_a_hand_built_scene():
    st, live, rects = hand_scene()
    fr = oracle.frame(st)
    codes, _ = oracle.sorted_codes(st, fr)
    lv = oracle.quadtree(codes, 2, 16)
    assert list(lv.lvl) == [1, 1, 1, 1] and list(lv.count) == [2, 1, 0, 2]
    feats, n_isect, n_cov, L, n_obj = costmodel.candidate_terms(live, rects, fr, lv)
    # the query's y range ends on the first cell row of the top leaves: it
    # intersects TL (empty, inactive) and TR with zero area
    assert (n_isect, n_cov, L, n_obj) == (3, 0, 4, 5)
    want = np.array([[np.log2(3), 1.0, 1 / 16, 0.5],    # BL: half its width, full height
                     [1.0, 1.0, 1 / 16, 0.5],           # BR
                     [np.log2(3), 1.0, 1 / 16, 0.0]])   # TR: touches along an edge
    assert np.allclose(feats, want, rtol=0, atol=1e-15)


@pytest.mark.parametrize("k", [1.0, 7.5])
def test_cost_of_a_constant_network(k):
    """All weights zero and b3 = ln k: every active leaf predicts k."""
    st, live, rects = hand_scene()
    p = np.zeros(mlp.P)
    p[-1] = np.log(k)
    coef = (2.0, 3.0, 5.0, 7.0, 11.0, 13.0)
    costs, sums, chosen = costmodel.choose(st, live, rects, p, coef, [8, 2])
    # th 2: the hand scene; th 8: the same tree, since the root is always split
    assert np.allclose(sums, 3 * k)
    # 4 leaves: keys below 4 take one radix pass over the 5 objects
    assert np.allclose(costs, 2 * 3 * k + 3 * 3 + 5 * 0 + 7 * 4 + 11 * k + 13 * 1 * 5)
    assert chosen == 8  # the first of equal costs


def test_critical_path_term_caps_the_subqueries_of_a_task():
    """A network predicting 0.01 (1 + objects)(1 + subqueries): the sum term
    takes a leaf's own subquery count, the maximum term at most 64 (one join
    task)."""
    p = np.zeros(mlp.P)
    p[0:2] = np.log(2.0)   # W1 row 0 on log2(1 + objects), log2(1 + subqueries)
    p[320] = 1.0           # W2[0][0]
    p[4480] = 1.0          # w3[0]
    p[4544] = np.log(0.01)
    feats = np.array([[np.log2(11.0), np.log2(101.0), 0.5, 0.3],    # 10 objects, 100 subqueries
                      [np.log2(3.0), np.log2(5.0), 0.25, 1.0]])     # 2 objects, 4 subqueries
    c, s = costmodel.cost(p, (1.0, 0.0, 0.0, 0.0, 0.0, 0.0), feats, 0, 0, 0)
    assert np.isclose(s, 0.01 * (11 * 101 + 3 * 5)) and np.isclose(c, s)
    c, _ = costmodel.cost(p, (0.0, 0.0, 0.0, 0.0, 1.0, 0.0), feats, 0, 0, 0)
    assert np.isclose(c, 0.01 * 11 * 65)


@pytest.mark.parametrize("leaves,passes", [(0, 0), (1, 0), (2, 1), (256, 1), (257, 2),
                                           (65536, 2), (65537, 3), (1 << 24, 3), ((1 << 24) + 1, 4)])
def test_sort_passes(leaves, passes):
    assert costmodel.sort_passes(leaves) == passes
