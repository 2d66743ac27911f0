"""Tick serving (continuous batching of many scenes on one GPU): each tick's
results are the same alone and in the mix, scenes are admitted by the memory
budget, and served results match the oracle."""
import time

import numpy as np
import pytest

import oracle
from gpu_util import oracle_apply, say
from paper_1411_3212_amd import serving

pytestmark = pytest.mark.gpu


def small_specs():
    return serving.make_specs(n_scenes=6, seed=7, nmin=2e4, nmax=1.5e5)


def test_served_results_equal_alone_and_admission_by_budget():
    import torch
    specs = small_specs()
    serving.upload(specs, 3, torch)
    srv_bytes = [serving.Server(1 << 20).scene_bytes(sp.cfg, sp.max_updates) for sp in specs]
    budget = int(max(srv_bytes) + 0.4 * (sum(srv_bytes) - max(srv_bytes)))
    reqs = serving.poisson_requests(len(specs), 36, rate_per_scene=400.0, n_ticks=3)
    say(f"serving {len(specs)} scenes, budget {budget} of {sum(srv_bytes)} bytes")
    r = serving.serve(specs, reqs, budget, max_running=3, torch=torch, keep_arrays=True,
                      evict=False)
    assert len(r["latency_ms"]) == 36 and (r["latency_ms"] > 0).all()
    # not every scene fits at once: some were admitted only after others retired
    assert max(r["admitted_at"].values()) >= min(r["retired_at"].values())
    by_scene = {}
    for tag, (_, s, k) in enumerate(reqs):
        by_scene.setdefault(s, []).append((tag, k))
    for s, lst in by_scene.items():
        alone = serving.serve_alone(specs[s], [k for _, k in lst], torch, keep_arrays=True)
        for (tag, k), (dig, arr) in zip(lst, alone):
            assert r["digest"][tag] == dig, (s, tag)
            assert np.array_equal(r["arrays"][tag][0], arr[0])
            assert np.array_equal(r["arrays"][tag][1], arr[1])
    # two scenes against the oracle (ticks 0..2 replayed in request order)
    for s in (0, 1):
        sp = specs[s]
        sp.wl.n_ticks = 3
        ticks = list(sp.wl.ticks())
        st = oracle.State(sp.wl.n)
        prev = None
        for tag, k in by_scene[s]:
            t = ticks[k]
            oracle_apply(st, t)
            live = oracle.live_queries(sp.wl.n, t.qid)
            cnt, h = oracle.brute_hash(st, t.qid, live, t.rects)
            assert np.array_equal(r["arrays"][tag][0], cnt), (s, tag)
            assert np.array_equal(r["arrays"][tag][1], h), (s, tag)


def test_evicted_scenes_come_back_with_identical_results():
    """A pool smaller than the scenes: the server evicts idle scenes to host
    memory and admits them again when their requests come up; every served
    tick's per-query counts and hashes equal those of the scene run alone
    without interruption, and two scenes' equal the oracle's."""
    import torch
    specs = small_specs()
    serving.upload(specs, 3, torch)
    srv_bytes = [serving.Server(1 << 20).scene_bytes(sp.cfg, sp.max_updates) for sp in specs]
    budget = int(max(srv_bytes) + 0.4 * (sum(srv_bytes) - max(srv_bytes)))
    reqs = serving.poisson_requests(len(specs), 48, rate_per_scene=300.0, n_ticks=3, seed=21)
    say(f"serving {len(specs)} scenes with eviction, budget {budget} of {sum(srv_bytes)} bytes")
    r = serving.serve(specs, reqs, budget, max_running=3, torch=torch, keep_arrays=True)
    say(f"  {r['admissions']} admissions, {r['evictions']} evictions")
    assert r["evictions"] > 0 and r["admissions"] > len(specs)
    by_scene = {}
    for tag, (_, s, k) in enumerate(reqs):
        by_scene.setdefault(s, []).append((tag, k))
    for s, lst in by_scene.items():
        alone = serving.serve_alone(specs[s], [k for _, k in lst], torch, keep_arrays=True)
        for (tag, k), (dig, arr) in zip(lst, alone):
            assert r["digest"][tag] == dig, (s, tag)
            assert np.array_equal(r["arrays"][tag][0], arr[0]), (s, tag)
            assert np.array_equal(r["arrays"][tag][1], arr[1]), (s, tag)
    for s in (2, 3):
        sp = specs[s]
        sp.wl.n_ticks = 3
        ticks = list(sp.wl.ticks())
        st = oracle.State(sp.wl.n)
        for tag, k in by_scene[s]:
            t = ticks[k]
            oracle_apply(st, t)
            live = oracle.live_queries(sp.wl.n, t.qid)
            cnt, h = oracle.brute_hash(st, t.qid, live, t.rects)
            assert np.array_equal(r["arrays"][tag][0], cnt), (s, tag)
            assert np.array_equal(r["arrays"][tag][1], h), (s, tag)


def test_explicit_eviction_between_ticks():
    """sj_server_evict between two ticks of one scene: its queued request
    brings it back, and both ticks equal the uninterrupted scene's; the
    scene object is unavailable while it is evicted."""
    import torch
    from paper_1411_3212_amd.binding import SjError
    sp = small_specs()[1]
    serving.upload([sp], 2, torch)
    need = serving.Server(1 << 20).scene_bytes(sp.cfg, sp.max_updates)
    srv = serving.Server(need + (1 << 20))
    sid = srv.admit(sp.cfg, sp.max_updates)
    got = []
    for k in range(2):
        buf, m, nq = sp.ticks[k]
        srv.submit(sid, k, *serving.tick_views(buf, m, nq, torch), digest=True)
        done, t_end = [], time.monotonic() + 30.0
        while not done and time.monotonic() < t_end:
            done += srv.poll()
        assert done and done[0][2] == 0
        _, _, _, n, pc, ph, _ = done[0]
        off = srv.pool.data_ptr()
        got.append((srv.pool[pc - off:pc - off + 8 * n].view(torch.int64).cpu().numpy(),
                    srv.pool[ph - off:ph - off + 8 * n].view(torch.int64).cpu().numpy()))
        if k == 0:
            srv.evict(sid)
            info = srv.info()
            assert info["resident"] == 0 and info["pool_used"] == 0 and info["evictions"] == 1
            with pytest.raises(SjError):
                srv.evict(sid)
    assert srv.info()["admissions"] == 2
    alone = serving.serve_alone(sp, [0, 1], torch, keep_arrays=True)
    for (c, h), (_, arr) in zip(got, alone):
        assert np.array_equal(c.view(np.uint64), arr[0]) and np.array_equal(h.view(np.uint64), arr[1])
    srv.retire(sid)
    srv.close()


def test_serving_order_does_not_change_results():
    import torch
    specs = small_specs()[:4]
    serving.upload(specs, 2, torch)
    reqs = serving.poisson_requests(len(specs), 16, rate_per_scene=1000.0, n_ticks=2, seed=1)
    a = serving.serve(specs, reqs, 8 << 30, max_running=4, torch=torch, digest=True)
    b = serving.serve(specs, reqs, 8 << 30, max_running=1, torch=torch, digest=True)
    assert a["digest"] == b["digest"] and a["counters"] == b["counters"]


def test_submit_checks_its_inputs():
    """Requests the server cannot run are refused at submission (nothing is
    queued): misaligned or null inputs, more updates than admitted, unknown
    flags."""
    import torch
    from paper_1411_3212_amd.binding import SjError
    sp = small_specs()[0]
    serving.upload([sp], 1, torch)
    buf, m, nq = sp.ticks[0]
    views = serving.tick_views(buf, m, nq, torch)
    need = serving.Server(1 << 20).scene_bytes(sp.cfg, sp.max_updates)
    srv = serving.Server(need + (1 << 20))
    sid = srv.admit(sp.cfg, sp.max_updates)
    assert sid is not None
    lib, h = srv._lib, srv.handle
    p = [v.data_ptr() for v in views]

    def submit(ptrs, m_, nq_, flags=0):
        return lib.sj_server_submit(h, sid, ptrs[0], ptrs[1], ptrs[2], m_, ptrs[3], ptrs[4],
                                    ptrs[5], ptrs[6], ptrs[7], nq_, 1, None, flags)

    for k in range(8):
        bad = list(p)
        bad[k] += 2
        assert submit(bad, m, nq) != 0, f"misaligned input {k}"
        bad[k] = 0
        assert submit(bad, m, nq) != 0, f"null input {k}"
    assert submit(p, sp.max_updates + 1, nq) != 0
    assert submit(p, m, nq, flags=2) != 0
    assert srv.info()["queued"] == 0
    srv.submit(sid, 7, *views)
    assert srv.info()["queued"] + srv.info()["running"] == 1
    done, t_end = [], time.monotonic() + 30.0
    while not done and time.monotonic() < t_end:
        done += srv.poll()
    assert done and done[0][1] == 7 and done[0][2] == 0
    srv.retire(sid)
    with pytest.raises(SjError):
        srv.submit(sid, 8, *views)
    srv.close()
