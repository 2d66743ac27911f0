"""Per-leaf timing log of the join: its feature columns equal the oracle's
leaf table, split and overlap on the same inputs, its clocks are sane, and
logging does not change the results."""
import numpy as np
import pytest

import oracle
from paper_1411_3212_amd import workloads
from paper_1411_3212_amd.binding import Scene

from gpu_util import gpu_tick, oracle_apply, oracle_lists, say

pytestmark = pytest.mark.gpu


def leaf_overlap(t, live, fr, lv, oi, li):
    """Mean over each leaf's intersecting subqueries of the fraction of the
    leaf's area that the query rectangle covers (float64)."""
    x0, y0, e = float(fr[0]), float(fr[1]), int(fr[2])
    scale = 2.0 ** (16 - e)
    st = lv.start.astype(np.uint64)
    cx, cy = np.zeros(len(st)), np.zeros(len(st))
    for b in range(16):  # x in the even bits, y in the odd bits
        cx += ((st >> np.uint64(2 * b)) & np.uint64(1)).astype(np.float64) * 2.0 ** b
        cy += ((st >> np.uint64(2 * b + 1)) & np.uint64(1)).astype(np.float64) * 2.0 ** b
    size = 2.0 ** (16 - lv.lvl.astype(np.float64)) / scale
    lx, ly = x0 + cx / scale, y0 + cy / scale
    tot = np.zeros(len(lv))
    num = np.zeros(len(lv))
    xa, ya, xb, yb = (np.asarray(r, np.float64) for r in t.rects)
    cnt = lv.count
    for k in range(len(t.qid)):
        for j in li[oi[k]:oi[k + 1]]:
            if cnt[j] == 0:
                continue
            w = min(xb[k], lx[j] + size[j]) - max(xa[k], lx[j])
            h = min(yb[k], ly[j] + size[j]) - max(ya[k], ly[j])
            tot[j] += min(1.0, max(w, 0) / size[j] * max(h, 0) / size[j])
            num[j] += 1
    return np.where(num > 0, tot / np.maximum(num, 1), 0.0), num


@pytest.mark.parametrize("th", [8, 64])
def test_timing_log_features_match_oracle(th):
    wl = workloads.make("uniform_1tick")
    t = next(wl.ticks())
    st = oracle.State(wl.n)
    oracle_apply(st, t)
    say(f"timing log th={th}")
    sc = Scene(wl.n, t.nq, th=th, timing_log=True)
    gpu_tick(sc, t)
    rec, mhz = sc.timing_log()
    rec = rec.cpu().numpy().astype(np.float64)
    assert mhz > 0
    fr = oracle.frame(st)
    codes, _ = oracle.sorted_codes(st, fr)
    lv = oracle.quadtree(codes, th, 16)
    live = oracle.live_queries(wl.n, t.qid)
    oi, li, _, _ = oracle.split(live, t.rects, fr, lv)
    assert rec.shape == (len(lv), 8)
    assert np.array_equal(rec[:, 0], lv.count)
    assert np.array_equal(rec[:, 2], lv.lvl)
    ovl, nsq = leaf_overlap(t, live, fr, lv, oi, li)
    assert np.array_equal(rec[:, 1], nsq)
    assert np.allclose(rec[:, 3], ovl, atol=1e-4)
    work = rec[:, 0] * rec[:, 1] > 0
    assert np.all(rec[~work, 4:6] == 0)
    assert np.all(rec[work, 4:6] >= 0) and np.all(np.isfinite(rec[:, 4:6]))
    assert (rec[work, 4] > 0).mean() > 0.5 and (rec[work, 5] > 0).mean() > 0.5
    assert np.all(rec[:, 6:] == 0)
    assert sc.fetch().to_lists() == oracle_lists(st, t)
