"""Pins of the oracle's k-nearest-neighbour queries (the paper's future work,
Section "Conclusions"; the definition is the reading both sides implement:
the k present objects of smallest (binary32 squared distance, id)).

* a lattice whose squared distances are exact small rationals: the result
  is the set of lattice offsets a^2 + b^2 <= R^2, a closed form;
* ties ordered by id, absent objects, superseded queries, k above the
  number of objects, k = 0;
* exact rational arithmetic (fractions) on random inputs, wherever the gap
  between the k-th and the next distance is far above binary32 rounding;
* against Definition 1's brute force: every object strictly inside the
  square inscribed in the k-th distance circle is a neighbour, every
  neighbour lies in the circumscribed square.
"""
from fractions import Fraction

import numpy as np

import oracle

NONE = 0xFFFFFFFF


def state(x, y, present=None):
    n = len(x)
    st = oracle.State(n)
    ids = np.arange(n, dtype=np.uint32) if present is None else np.asarray(present, np.uint32)
    oracle.apply_updates(st, ids, np.asarray(x, np.float32)[ids], np.asarray(y, np.float32)[ids])
    return st


def test_lattice_closed_form():
    """16 x 16 objects on the lattice (i/64, j/64), ids shuffled; a query at
    lattice point (8/64, 8/64).  Offsets (a, b) have squared distance
    (a^2 + b^2)/4096 exactly, so the 13 nearest are the offsets with
    a^2 + b^2 <= 4, and the 21 nearest add the eight with a^2 + b^2 = 5."""
    rng = np.random.default_rng(1)
    perm = rng.permutation(256)
    x = np.zeros(256, np.float32)
    y = np.zeros(256, np.float32)
    lattice = {}
    for i in range(16):
        for j in range(16):
            o = int(perm[i * 16 + j])
            x[o], y[o] = i / 64, j / 64
            lattice[o] = (i, j)
    st = state(x, y)
    for k, r2 in ((1, 0), (5, 1), (9, 2), (13, 4), (21, 5)):
        ids, d2 = oracle.knn(st, np.ones(1, np.uint8), [8 / 64], [8 / 64], k)
        want = sorted(((a - 8) ** 2 + (b - 8) ** 2, o) for o, (a, b) in lattice.items()
                      if (a - 8) ** 2 + (b - 8) ** 2 <= r2)
        assert len(want) == k
        assert ids[0].tolist() == [o for _, o in want]
        assert d2[0].tolist() == [s / 4096 for s, _ in want]


def test_ties_by_id_absent_superseded_and_short():
    # four objects at the same distance from (0.5, 0.5), one absent
    x = [0.75, 0.5, 0.25, 0.5, 0.5]
    y = [0.5, 0.75, 0.5, 0.25, 0.5]
    st = state(x, y, present=[0, 1, 2, 3])  # object 4 (at the query point) has no position
    ids, d2 = oracle.knn(st, np.ones(1, np.uint8), [0.5], [0.5], 3)
    assert ids[0].tolist() == [0, 1, 2] and d2[0].tolist() == [0.0625] * 3
    ids, d2 = oracle.knn(st, np.ones(1, np.uint8), [0.5], [0.5], 6)
    assert ids[0].tolist() == [0, 1, 2, 3, NONE, NONE]
    assert np.isinf(d2[0, 4:]).all()
    # a superseded query: every slot empty
    ids, d2 = oracle.knn(st, np.array([0, 1], np.uint8), [0.5, 0.5], [0.5, 0.5], 2)
    assert ids[0].tolist() == [NONE, NONE] and ids[1].tolist() == [0, 1]
    ids, d2 = oracle.knn(st, np.ones(3, np.uint8), [0.1, 0.2, 0.3], [0.1, 0.2, 0.3], 0)
    assert ids.shape == (3, 0)


def test_exact_rational_order():
    """Exact squared distances (fractions of the binary32 inputs) order the
    objects as the oracle does wherever consecutive exact distances around
    the k-th differ by far more than binary32 rounding."""
    rng = np.random.default_rng(2)
    n, k = 300, 7
    x = rng.random(n).astype(np.float32)
    y = rng.random(n).astype(np.float32)
    st = state(x, y)
    qx = rng.random(40).astype(np.float32)
    qy = rng.random(40).astype(np.float32)
    ids, _ = oracle.knn(st, np.ones(40, np.uint8), qx, qy, k)
    checked = 0
    for q in range(40):
        fx, fy = Fraction(float(qx[q])), Fraction(float(qy[q]))
        ex = sorted(((Fraction(float(x[o])) - fx) ** 2 + (Fraction(float(y[o])) - fy) ** 2, o)
                    for o in range(n))
        dist = [d for d, _ in ex[:k + 1]]
        if any(b - a <= a * Fraction(1, 1 << 18) for a, b in zip(dist, dist[1:])):
            continue  # a near-tie that rounding may order either way
        assert ids[q].tolist() == [o for _, o in ex[:k]]
        checked += 1
    assert checked >= 30


def test_against_range_brute_force():
    """Objects strictly inside the square inscribed in the circle of the
    k-th distance are all neighbours; every neighbour lies inside the
    circumscribed square (Definition 1 brute force on both squares)."""
    rng = np.random.default_rng(3)
    n, k, nq = 2000, 16, 64
    x = rng.random(n).astype(np.float32)
    y = rng.random(n).astype(np.float32)
    st = state(x, y)
    qx = rng.random(nq).astype(np.float32)
    qy = rng.random(nq).astype(np.float32)
    live = np.ones(nq, np.uint8)
    ids, d2 = oracle.knn(st, live, qx, qy, k)
    r = np.sqrt(d2[:, -1].astype(np.float64))
    inner = r / np.sqrt(2.0) * (1 - 1e-5)
    outer = r * (1 + 1e-5)
    sq = lambda h: (qx - h, qy - h, qx + h, qy + h)
    off_i, in_ids = oracle.brute_lists(st, live, tuple(v.astype(np.float32) for v in sq(inner)))
    off_o, out_ids = oracle.brute_lists(st, live, tuple(v.astype(np.float32) for v in sq(outer)))
    for q in range(nq):
        nb = set(ids[q].tolist())
        assert set(in_ids[off_i[q]:off_i[q + 1]].tolist()) <= nb
        assert nb <= set(out_ids[off_o[q]:off_o[q + 1]].tolist())


def test_selection_invariants():
    """Ascending keys; no unselected present object has a smaller key."""
    rng = np.random.default_rng(4)
    n, k = 500, 10
    x = (rng.random(n) * 0.01).astype(np.float32)  # dense: many close distances
    y = (rng.random(n) * 0.01).astype(np.float32)
    x[::7] = x[3]  # duplicate positions: ties broken by id
    y[::7] = y[3]
    st = state(x, y)
    ids, d2 = oracle.knn(st, np.ones(5, np.uint8), x[[3, 10, 20, 30, 40]], y[[3, 10, 20, 30, 40]], k)
    for q, o in enumerate([3, 10, 20, 30, 40]):
        keys = [(float(d2[q, i]), int(ids[q, i])) for i in range(k)]
        assert keys == sorted(keys)
        kth = keys[-1]
        for j in set(range(n)) - set(ids[q].tolist()):
            assert (oracle.knn_d2(float(x[j]), float(y[j]), float(x[o]), float(y[o])), j) > kth
