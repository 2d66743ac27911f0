"""CPU oracle of the learned threshold choice (test infrastructure only).

For a candidate threshold the quadtree is built by Algorithm 1 and the
queries are split against it (the oracle's own ``quadtree`` and ``split``);
the cost of the tick's filtering and decoding is predicted from the terms of
their complexity (Computational Complexity section, filtering and decoding
equations): over the active leaves c (objects and intersecting subqueries),
exp(MLP(f_c)) with

    f_c = (log2(1 + |P^c|), log2(1 + |Q_I^c|), level / 16,
           mean over the intersecting subqueries of c of the fraction of the
           area of c that their rectangle covers),

plus terms linear in |Q_I|, |Q_C|, the number of leaves, and the largest
prediction for one join task (the join's critical path: one wave joins at
most 64 intersecting subqueries of a leaf; f'_c is f_c with |Q_I^c| capped
at 64):

    cost = coef[0] sum_c exp(MLP(f_c)) + coef[1] |Q_I| + coef[2] |Q_C|
           + coef[3] leaves + coef[4] max_c exp(MLP(f'_c))
           + coef[5] P(leaves) objects,

P(L) = ceil(bit length of (L - 1) / 8): the radix passes of the sort by leaf
index on the ticks that keep the quadtree.

Leaves without objects are inactive and hold no subqueries.  Float64
throughout; shares no code with the HIP kernels.
"""
from __future__ import annotations

import numpy as np

import oracle
from oracle import mlp

TASK_SUB = 64  # intersecting subqueries of a leaf joined by one task


def leaf_geometry(fr, leaves: oracle.Leaves):
    """(x, y, side) of every leaf square in coordinates (float64)."""
    x0, y0, e = float(fr[0]), float(fr[1]), int(fr[2])
    scale = 2.0 ** (16 - e)
    st = leaves.start.astype(np.uint64)
    cx, cy = np.zeros(len(st)), np.zeros(len(st))
    for b in range(16):  # x in the even bits, y in the odd bits
        cx += ((st >> np.uint64(2 * b)) & np.uint64(1)).astype(np.float64) * 2.0 ** b
        cy += ((st >> np.uint64(2 * b + 1)) & np.uint64(1)).astype(np.float64) * 2.0 ** b
    side = 2.0 ** (16 - leaves.lvl.astype(np.float64)) / scale
    return x0 + cx / scale, y0 + cy / scale, side


def overlap_fraction(rect, lx, ly, side):
    """Fraction of the leaf square [lx, lx+side] x [ly, ly+side] covered by
    rect = (xa, ya, xb, yb), in [0, 1] (0 when they do not overlap with
    positive area)."""
    xa, ya, xb, yb = (np.asarray(r, np.float64) for r in rect)
    w = np.minimum(xb, lx + side) - np.maximum(xa, lx)
    h = np.minimum(yb, ly + side) - np.maximum(ya, ly)
    f = (np.maximum(w, 0.0) / side) * (np.maximum(h, 0.0) / side)
    return np.where((w > 0) & (h > 0), np.minimum(f, 1.0), 0.0)


def sort_passes(n_leaves: int) -> int:
    """8-bit radix passes that sort keys below n_leaves."""
    return (int(n_leaves - 1).bit_length() + 7) // 8 if n_leaves > 1 else 0


def candidate_terms(live, rects, fr, leaves: oracle.Leaves):
    """Features of the active leaves and the counts of the linear terms for
    one quadtree: (features [n_active, 4], n_isect, n_cov, n_leaves,
    objects)."""
    oi, li, oc, lc = oracle.split(live, rects, fr, leaves)
    cnt = leaves.count
    q_of = np.repeat(np.arange(len(oi) - 1), np.diff(oi).astype(np.int64))
    act = cnt[li] > 0
    q_of, lj = q_of[act], li[act].astype(np.int64)
    n_cov = int((cnt[lc] > 0).sum())
    L = len(leaves)
    nsq = np.bincount(lj, minlength=L)
    lx, ly, side = leaf_geometry(fr, leaves)
    xa, ya, xb, yb = (np.asarray(r, np.float64)[q_of] for r in rects)
    frac = overlap_fraction((xa, ya, xb, yb), lx[lj], ly[lj], side[lj])
    osum = np.bincount(lj, weights=frac, minlength=L)
    a = (cnt > 0) & (nsq > 0)
    feats = np.stack([np.log2(1.0 + cnt[a]), np.log2(1.0 + nsq[a]),
                      leaves.lvl[a].astype(np.float64) / 16.0, osum[a] / nsq[a]], axis=1)
    return feats, int(len(lj)), n_cov, L, int(cnt.sum())


def cost(params, coef, feats, n_isect, n_cov, n_leaves, n_objects=0):
    """Predicted cost and the sum of the predictions from the features and
    counts (params: the BF16-rounded MLP parameters as values)."""
    if len(feats):
        e = np.exp(mlp.forward(params, feats))
        capped = feats.copy()
        capped[:, 1] = np.minimum(capped[:, 1], np.log2(1.0 + TASK_SUB))
        s, m = float(e.sum()), float(np.exp(mlp.forward(params, capped)).max())
    else:
        s, m = 0.0, 0.0
    return (coef[0] * s + coef[1] * n_isect + coef[2] * n_cov + coef[3] * n_leaves +
            coef[4] * m + coef[5] * sort_passes(n_leaves) * n_objects), s


def choose(st: oracle.State, live, rects, params, coef, cand, l_max: int = 16,
           cap_isect=None, cap_cov=None):
    """Costs of every candidate threshold on the current positions and the
    chosen one (the first of the cheapest).  A candidate whose split needs
    more intersecting or covering subqueries than the capacities is
    infeasible (infinite cost)."""
    fr = oracle.frame(st)
    codes, _ = oracle.sorted_codes(st, fr)
    costs, sums = [], []
    for th in cand:
        lv = oracle.quadtree(codes, th, l_max)
        feats, n_isect, n_cov, L, n_obj = candidate_terms(live, rects, fr, lv)
        c, s = cost(params, coef, feats, n_isect, n_cov, L, n_obj)
        if (cap_isect is not None and n_isect > cap_isect) or \
                (cap_cov is not None and n_cov > cap_cov):
            c = np.inf
        costs.append(c)
        sums.append(s)
    best = int(np.argmin(costs))
    return np.array(costs), np.array(sums), int(cand[best])
