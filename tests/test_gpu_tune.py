"""Learned threshold choice on the GPU: the predicted cost of every
candidate equals the oracle's (same quadtrees, splits, features and BF16
network), the cheapest is built, infeasible candidates are skipped, and the
results stay those of the oracle and of a fixed-threshold scene."""
import numpy as np
import pytest

import oracle
from oracle import costmodel, mlp
from paper_1411_3212_amd import workloads
from paper_1411_3212_amd.binding import Scene

from gpu_util import (gpu_count_hash, gpu_tick, oracle_apply, oracle_count_hash, oracle_lists,
                      say)

pytestmark = pytest.mark.gpu

CAND = [4, 8, 16, 32, 64, 128, 256]
COEF = (1.0, 0.02, 0.01, 0.05, 3.0, 1e-4)


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.synchronize()


def model(seed):
    """A random network (small weights): BF16 bits for the device, their
    values for the oracle."""
    bits = mlp.bf16_bits(0.5 * mlp.init_params(seed))
    return bits, mlp.bf16_value(bits).astype(np.float64)


def work_model():
    """A network whose prediction is 0.01 (1 + objects)(1 + subqueries) (up
    to BF16 rounding): cheap leaves favour small thresholds, the linear
    terms large ones, so the cheapest candidate lies inside the range."""
    m = np.zeros(mlp.P, np.float32)
    m[0:2] = np.log(2.0)   # W1 row 0 on log2(1 + objects), log2(1 + subqueries)
    m[320] = 1.0           # W2[0][0]
    m[4480] = 1.0          # w3[0]
    m[4544] = np.log(0.01)
    bits = mlp.bf16_bits(m)
    return bits, mlp.bf16_value(bits).astype(np.float64)


def install(sc, bits, coef=COEF, cand=CAND):
    import torch
    w = torch.from_numpy(bits.view(np.int16).copy()).cuda()
    sc.set_cost_model(w, coef, cand)


def check_choice(info, costs, chosen):
    assert info["n_tunes"] >= 1 and info["cand"] == list(CAND)
    got = np.array(info["cost"], np.float64)
    fin = np.isfinite(costs)
    assert np.array_equal(np.isfinite(got), fin)
    assert np.allclose(got[fin], costs[fin], rtol=1e-3)
    srt = np.sort(costs[fin])
    if len(srt) < 2 or srt[1] > srt[0] * (1 + 1e-3):  # a clear winner
        assert info["chosen"] == chosen
    else:
        assert costs[CAND.index(info["chosen"])] <= srt[0] * (1 + 1e-3)


@pytest.mark.parametrize("name,seed", [("uniform_1tick", 1), ("uniform_1tick", None),
                                       ("hotspot", 2), ("hotspot", None)])
def test_predicted_costs_and_choice_match_oracle(name, seed):
    over = dict(n=60_000, n_ticks=1) if name == "hotspot" else {}
    wl = workloads.make(name, **over)
    t = next(wl.ticks())
    st = oracle.State(wl.n)
    oracle_apply(st, t)
    say(f"tune parity {name} n={wl.n} nq={t.nq} model={seed}")
    bits, params = model(seed) if seed is not None else work_model()
    live = oracle.live_queries(wl.n, t.qid)
    cap = 64 * t.nq
    costs, _, chosen = costmodel.choose(st, live, t.rects, params, COEF, CAND, cap_isect=cap,
                                        cap_cov=cap)
    sc = Scene(wl.n, t.nq, th=64, th_min=4, thresh_mlp=True, capacity_subqueries=cap,
               capacity_covering=cap)
    install(sc, bits)
    gpu_tick(sc, t)
    info = sc.tune_info()
    check_choice(info, costs, chosen)
    s = sc.stats()
    assert s["th"] == info["chosen"]
    # the tick's index is Algorithm 1 at the chosen threshold
    v = sc.index_view()
    fr = oracle.frame(st)
    codes, _ = oracle.sorted_codes(st, fr)
    lv = oracle.quadtree(codes, info["chosen"], 16)
    assert v["n_leaves"] == len(lv)
    assert np.array_equal(v["leaf_level"].cpu().numpy(), lv.lvl.astype(np.int32))
    if name == "uniform_1tick":
        assert sc.fetch().to_lists() == oracle_lists(st, t)
    else:
        cnt, h = gpu_count_hash(sc)
        ocnt, oh = oracle_count_hash(st, t)
        assert np.array_equal(cnt, ocnt) and np.array_equal(h, oh)


def test_candidates_that_overflow_are_infeasible():
    wl = workloads.make("uniform_1tick")
    t = next(wl.ticks())
    st = oracle.State(wl.n)
    oracle_apply(st, t)
    bits, params = model(3)
    live = oracle.live_queries(wl.n, t.qid)
    fr = oracle.frame(st)
    codes, _ = oracle.sorted_codes(st, fr)
    n_isect = [costmodel.candidate_terms(live, t.rects, fr, oracle.quadtree(codes, th, 16))[1]
               for th in CAND]
    cap = (n_isect[1] + n_isect[2]) // 2  # th 4 and 8 overflow, 16 and above fit
    assert n_isect[1] > cap >= n_isect[2]
    say(f"tune overflow cap={cap} n_isect={n_isect}")
    costs, _, chosen = costmodel.choose(st, live, t.rects, params, COEF, CAND, cap_isect=cap,
                                        cap_cov=32 * t.nq)
    assert np.isinf(costs[:2]).all() and np.isfinite(costs[2:]).all()
    sc = Scene(wl.n, t.nq, th=64, th_min=4, thresh_mlp=True, capacity_subqueries=cap)
    install(sc, bits)
    gpu_tick(sc, t)
    info = sc.tune_info()
    check_choice(info, costs, chosen)
    assert sc.stats()["th"] == info["chosen"]  # no error latched by the trials
    assert sc.fetch().to_lists() == oracle_lists(st, t)


@pytest.mark.parametrize("mode", ["eager", "graph"])
def test_tuned_ticks_equal_fixed_threshold_ticks(mode):
    """Every build tunes (period 4, tune_every 1); each tick's result set
    equals the one of a fixed-threshold scene and, on two ticks, the
    oracle's."""
    import torch
    wl = workloads.make("hotspot", n=60_000, n_ticks=10)
    nq = max(t.nq for t in wl.ticks())
    bits, params = work_model()
    kw = dict(capacity_subqueries=64 * nq, capacity_covering=64 * nq, rebuild="auto",
              rebuild_period=4)
    tuned = Scene(wl.n, nq, th=64, th_min=4, thresh_mlp=True, tune_every=1, **kw)
    install(tuned, bits)
    fixed = Scene(wl.n, nq, th=64, **kw)
    st = oracle.State(wl.n)
    chosen = []
    for i, t in enumerate(wl.ticks()):
        say(f"tuned vs fixed {mode} tick {i}")
        oracle_apply(st, t)
        if mode == "graph":
            d = [torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()
                 for a in (t.ids, t.x, t.y, t.qid, t.xa, t.ya, t.xb, t.yb)]
            tuned.tick_graph(*(a if k in (0, 3) else a.view(torch.float32) for k, a in enumerate(d)))
        else:
            gpu_tick(tuned, t)
        gpu_tick(fixed, t)
        a, b = gpu_count_hash(tuned), gpu_count_hash(fixed)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        s = tuned.stats()
        chosen.append(s["th"])
        if i in (0, 9):
            ocnt, oh = oracle_count_hash(st, t)
            assert np.array_equal(a[0], ocnt) and np.array_equal(a[1], oh)
    info = tuned.tune_info()
    assert info["n_tunes"] >= 3  # ticks 0, 4 and 8 build (and any the policy adds)
    assert all(c in CAND for c in chosen)


@pytest.mark.parametrize("thresh", [False, True])
def test_learned_schedule_gives_the_same_results(thresh):
    """Join tasks ordered by the network's predicted time (with or without
    the learned threshold): every tick's result set equals the one of the
    weight-ordered fixed-threshold scene."""
    wl = workloads.make("hotspot", n=60_000, n_ticks=6)
    nq = max(t.nq for t in wl.ticks())
    bits, _ = work_model()
    kw = dict(capacity_subqueries=64 * nq, capacity_covering=64 * nq, rebuild_period=4)
    learned = Scene(wl.n, nq, th=64, th_min=4, thresh_mlp=thresh, schedule_mlp=True, **kw)
    install(learned, bits)
    fixed = Scene(wl.n, nq, th=64, **kw)
    for i, t in enumerate(wl.ticks()):
        say(f"learned schedule thresh={thresh} tick {i}")
        gpu_tick(learned, t)
        gpu_tick(fixed, t)
        a, b = gpu_count_hash(learned), gpu_count_hash(fixed)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        if not thresh:  # same quadtree: same split of the pairs into tested and covered
            assert learned.stats()["n_isect_ids"] == fixed.stats()["n_isect_ids"]
