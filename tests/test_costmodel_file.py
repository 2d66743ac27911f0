"""The committed cost model: parameters, cost terms and candidates are
well formed, and the training driver's host-side helpers behave."""
import numpy as np

from paper_1411_3212_amd import costmodel


def test_committed_model_is_well_formed():
    m = costmodel.load()
    bits = m["bits"]
    assert bits.dtype == np.uint16 and len(bits) == 4545
    vals = (bits.astype(np.uint32) << 16).view(np.float32)
    assert np.isfinite(vals).all() and np.abs(vals).max() < 1e3
    assert len(m["coef"]) == 6 and all(c >= 0 for c in m["coef"]) and any(m["coef"])
    assert 1 <= len(m["cand"]) <= 8 and all(c >= 1 for c in m["cand"])
    assert m["cand"] == sorted(m["cand"])
    tr = m["doc"]["training"]
    assert tr["logged_ticks"] >= 200


def test_leaf_samples_selects_active_leaves():
    rec = np.array([[3, 2, 4, 0.5, 100, 300, 0, 0],    # active
                    [0, 2, 5, 0.0, 0, 0, 0, 0],        # no objects
                    [7, 0, 6, 0.0, 0, 0, 0, 0],        # no subqueries
                    [1, 1, 16, 1.0, 50, 50, 0, 0]], np.float32)
    X, us = costmodel.leaf_samples(rec, 100.0)
    assert X.shape == (2, 4)
    assert np.allclose(X[0], [2.0, np.log2(3), 0.25, 0.5])
    assert np.allclose(X[1], [1.0, 1.0, 1.0, 1.0])
    assert np.allclose(us, [4.0, 1.0])
