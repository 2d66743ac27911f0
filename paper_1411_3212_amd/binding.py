"""ctypes binding of libsj (include/sj.h).  Argument marshalling only: every
step of the join runs in the library's HIP kernels.  PyTorch provides the
device memory (the scene's workspace, result buffers) and the stream.

The library must have been built (``paper_1411_3212_amd/build.py``); loading
fails loudly otherwise -- there is no other implementation behind this API.
"""
from __future__ import annotations

import ctypes
from ctypes import POINTER, Structure, byref, c_char_p, c_float, c_int, c_int32, c_size_t, \
    c_uint32, c_uint64, c_void_p
from pathlib import Path

import numpy as np

LIB_PATH = Path(__file__).resolve().parent / "libsj.so"

SJ_OK, SJ_EINVAL, SJ_ENOSPACE, SJ_EOVERFLOW, SJ_EDATA, SJ_EDEVICE, SJ_ESTATE = 0, -1, -2, -3, -4, -5, -6
SJ_COVERING, SJ_REORDER, SJ_PROFILE, SJ_TIMING_LOG, SJ_THRESH_MLP, SJ_SCHEDULE_MLP = \
    1, 2, 4, 8, 16, 32
SJ_UNIFORM_GRID, SJ_ATOMIC_RESULTS, SJ_CU_COUNTERS = 64, 128, 256
CU_SLOTS = 4096
SJ_SORTED = 1  # sj_expand_results: ascending ids per list
COST_TERMS = 6  # SJ_COST_TERMS
REBUILD = {"auto": 0, "always": 1, "never": 2, "cost": 3}
PHASES = ["updates", "index", "build", "leaves", "split", "schedule", "join_count", "join_scan",
          "join_write"]
_NAMES = {0: "SJ_OK", -1: "SJ_EINVAL", -2: "SJ_ENOSPACE", -3: "SJ_EOVERFLOW", -4: "SJ_EDATA",
          -5: "SJ_EDEVICE", -6: "SJ_ESTATE"}


class SjError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class SjConfig(Structure):
    _fields_ = [("capacity_objects", c_uint32), ("capacity_queries", c_uint32),
                ("capacity_subqueries", c_uint64), ("capacity_covering", c_uint64),
                ("capacity_results", c_uint64), ("th_quad", c_uint32), ("th_min", c_uint32),
                ("l_max", c_uint32), ("flags", c_uint32), ("rebuild_policy", c_uint32),
                ("rebuild_period", c_uint32), ("split_slots", c_uint32), ("tune_every", c_uint32),
                ("grid_split", c_uint32)]


class SjResults(Structure):
    _fields_ = [("nq", c_uint32), ("n_leaves", c_uint32), ("n_isect_ids", c_uint64),
                ("n_cov_entries", c_uint64), ("total_pairs", c_uint64), ("n_runs", c_uint64),
                ("d_query_pos", c_void_p), ("d_isect_slot_off", c_void_p), ("d_slot_run", c_void_p), ("d_run_off", c_void_p),
                ("d_isect_id", c_void_p), ("d_cov_off", c_void_p),
                ("d_cov_leaf", c_void_p), ("d_leaf_beg", c_void_p), ("d_sorted_id", c_void_p),
                ("n_present", c_uint32), ("n_tasks", c_uint32), ("n_subqueries", c_uint64),
                ("cov_pairs", c_uint64), ("tests", c_uint64), ("error_bits", c_uint32),
                ("reserved", c_uint32), ("n_pairs", c_uint64), ("d_pairs", c_void_p)]


class SjTickStats(Structure):
    _fields_ = [("n_present", c_uint32), ("n_leaves", c_uint32), ("n_nodes", c_uint32),
                ("l_deep", c_uint32), ("th", c_uint32), ("rebuilt", c_uint32),
                ("n_tasks", c_uint32), ("max_leaf", c_uint32), ("n_isect", c_uint64),
                ("n_cov", c_uint64), ("n_isect_ids", c_uint64), ("cov_pairs", c_uint64),
                ("tests", c_uint64), ("error_bits", c_uint32), ("tick", c_uint32),
                ("knn_fallback", c_uint32), ("reserved", c_uint32)]


class SjIndexView(Structure):
    _fields_ = [("n_present", c_uint32), ("n_leaves", c_uint32), ("l_deep", c_uint32),
                ("x0", c_float), ("y0", c_float), ("e", c_int32),
                ("d_codes", c_void_p), ("d_ids", c_void_p), ("d_leaf_start", c_void_p),
                ("d_leaf_level", c_void_p), ("d_leaf_beg", c_void_p), ("d_pos", c_void_p)]


class SjTimingView(Structure):
    _fields_ = [("n_leaves", c_uint32), ("clock_mhz", c_float), ("d_records", c_void_p)]


class SjTuneInfo(Structure):
    _fields_ = [("n_cand", c_uint32), ("cand", c_uint32 * 8), ("cost", c_float * 8),
                ("mlp_sum", c_float * 8), ("mlp_max", c_float * 8), ("chosen", c_uint32),
                ("n_tunes", c_uint32),
                ("tuned_tick", c_uint32)]


class SjServed(Structure):
    _fields_ = [("tag", c_uint64), ("scene_id", c_uint32), ("status", c_int32), ("nq", c_uint32),
                ("d_count", c_void_p), ("d_hash", c_void_p), ("d_counters", c_void_p)]


class SjServerStats(Structure):
    _fields_ = [("pool_bytes", c_uint64), ("pool_used", c_uint64), ("scenes", c_uint32),
                ("running", c_uint32), ("queued", c_uint32), ("resident", c_uint32),
                ("admissions", c_uint32), ("evictions", c_uint32)]


EXPORTS = {
    "sj_workspace_bytes": (c_size_t, [POINTER(SjConfig)]),
    "sj_scene_create": (c_int, [POINTER(SjConfig), c_void_p, c_size_t, c_void_p,
                                POINTER(c_void_p)]),
    "sj_scene_destroy": (c_int, [c_void_p]),
    "sj_apply_updates": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_uint32]),
    "sj_build_index": (c_int, [c_void_p, c_uint32]),
    "sj_run_tick": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                            c_uint32]),
    "sj_run_knn": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_uint32, c_uint32, c_void_p,
                           c_void_p]),
    "sj_tick_graph": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_uint32, c_void_p,
                              c_void_p, c_void_p, c_void_p, c_void_p, c_uint32]),
    "sj_fetch_results": (c_int, [c_void_p, POINTER(SjResults)]),
    "sj_expand_results": (c_int, [c_void_p, c_void_p, c_uint32, c_uint32, c_void_p, c_void_p,
                                  c_uint64, POINTER(c_uint64)]),
    "sj_result_hashes": (c_int, [c_void_p, c_void_p, c_void_p]),
    "sj_tick_counters": (c_int, [c_void_p, c_void_p]),
    "sj_stats": (c_int, [c_void_p, POINTER(SjTickStats)]),
    "sj_phase_times": (c_int, [c_void_p, POINTER(c_float), c_int]),
    "sj_index_view_get": (c_int, [c_void_p, POINTER(SjIndexView)]),
    "sj_timing_log": (c_int, [c_void_p, POINTER(SjTimingView)]),
    "sj_set_cost_model": (c_int, [c_void_p, c_void_p, POINTER(c_float), POINTER(c_uint32),
                                  c_uint32]),
    "sj_tune_info_get": (c_int, [c_void_p, POINTER(SjTuneInfo)]),
    "sj_last_error": (c_char_p, [c_void_p]),
    "sj_cu_counters": (c_int, [c_void_p, c_void_p, c_uint32]),
    "sj_server_scene_bytes": (c_size_t, [POINTER(SjConfig), c_uint32]),
    "sj_server_create": (c_int, [c_void_p, c_size_t, c_uint32, POINTER(c_void_p)]),
    "sj_server_destroy": (c_int, [c_void_p]),
    "sj_server_admit": (c_int, [c_void_p, POINTER(SjConfig), c_uint32, POINTER(c_uint32)]),
    "sj_server_retire": (c_int, [c_void_p, c_uint32]),
    "sj_server_submit": (c_int, [c_void_p, c_uint32, c_void_p, c_void_p, c_void_p, c_uint32,
                                 c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_uint32,
                                 c_uint64, c_void_p, c_uint32]),
    "sj_server_poll": (c_int, [c_void_p, POINTER(SjServed), c_uint32, POINTER(c_uint32)]),
    "sj_server_add": (c_int, [c_void_p, POINTER(SjConfig), c_uint32, POINTER(c_uint32)]),
    "sj_server_evict": (c_int, [c_void_p, c_uint32]),
    "sj_server_info": (c_int, [c_void_p, POINTER(SjServerStats)]),
    "sj_server_scene": (c_int, [c_void_p, c_uint32, POINTER(c_void_p)]),
    "sj_server_last_error": (c_char_p, [c_void_p]),
    "sj_mlp_param_count": (c_uint32, []),
    "sj_mlp_round": (c_int, [c_void_p, c_void_p, c_void_p]),
    "sj_mlp_forward": (c_int, [c_void_p, c_void_p, c_uint32, c_void_p, c_void_p]),
    "sj_mlp_scratch_bytes": (c_size_t, [c_uint32]),
    "sj_mlp_grad": (c_int, [c_void_p, c_void_p, c_void_p, c_uint32, c_void_p, c_void_p, c_size_t,
                            c_void_p]),
    "sj_mlp_noalloc_scratch_bytes": (c_size_t, []),
    "sj_mlp_grad_noalloc": (c_int, [c_void_p, c_void_p, c_void_p, c_uint32, c_void_p, c_void_p]),
    "sj_mlp_adam": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_uint32, c_float,
                            c_void_p]),
}

_lib = None


def load():
    """Loads libsj.so and declares its exports; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not LIB_PATH.exists():
        raise ImportError(f"libsj is not built ({LIB_PATH} missing): run "
                          "paper_1411_3212_amd/build.py or __graft_entry__.build()")
    lib = ctypes.CDLL(str(LIB_PATH))
    for name, (res, args) in EXPORTS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _require(cond: bool, msg: str):
    """Argument check that stays on under python -O."""
    if not cond:
        raise ValueError(msg)


def _check(rc: int, handle=None):
    if rc != SJ_OK:
        msg = load().sj_last_error(handle)
        raise SjError(rc, msg.decode() if msg else "")


def make_config(capacity_objects: int, capacity_queries: int, *, th: int = 64, th_min: int = 0,
                l_max: int = 16, covering: bool = True, reorder: bool = True,
                rebuild: str = "auto", rebuild_period: int = 32, capacity_subqueries: int = 0,
                capacity_covering: int = 0, capacity_results: int = 0, split_slots: int = 0,
                profile: bool = False, timing_log: bool = False, thresh_mlp: bool = False,
                schedule_mlp: bool = False, tune_every: int = 0, grid_split: int = 0,
                atomic_results: bool = False, cu_counters: bool = False) -> SjConfig:
    """grid_split > 0 selects the uniform-grid index with that split factor;
    atomic_results the baseline filter (appended pairs); cu_counters the
    per-CU test counters."""
    flags = (SJ_COVERING if covering else 0) | (SJ_REORDER if reorder else 0) | \
            (SJ_PROFILE if profile else 0) | (SJ_TIMING_LOG if timing_log else 0) | \
            (SJ_THRESH_MLP if thresh_mlp else 0) | (SJ_SCHEDULE_MLP if schedule_mlp else 0) | \
            (SJ_UNIFORM_GRID if grid_split else 0) | \
            (SJ_ATOMIC_RESULTS if atomic_results else 0) | (SJ_CU_COUNTERS if cu_counters else 0)
    return SjConfig(capacity_objects, capacity_queries, capacity_subqueries, capacity_covering,
                    capacity_results, th, th_min, l_max, flags, REBUILD[rebuild], rebuild_period,
                    split_slots, tune_every, grid_split)


def _ptr(t):
    return c_void_p(t.data_ptr()) if t is not None else None


class Results:
    """Compressed results of a tick as torch views into the workspace (made
    on first access, so a fetch for the counters builds no tensor)."""

    _VIEWS = {  # attribute: (pointer field, length, dtype name)
        "query_pos": ("d_query_pos", lambda r: r.nq, "int32"),
        "isect_slot_off": ("d_isect_slot_off", lambda r: r.nq + 1, "int32"),
        "slot_run": ("d_slot_run", lambda r: r.n_runs, "int32"),
        "run_off": ("d_run_off", lambda r: r.n_runs + 1, "int64"),
        "isect_id": ("d_isect_id", lambda r: r.n_isect_ids, "int32"),
        "cov_off": ("d_cov_off", lambda r: r.nq + 1, "int32"),
        "cov_leaf": ("d_cov_leaf", lambda r: r.n_cov_entries, "int32"),
        "leaf_beg": ("d_leaf_beg", lambda r: r.n_leaves + 1, "int32"),
        "sorted_id": ("d_sorted_id", lambda r: r.n_present if r.n_leaves else 0, "int32"),
        "pairs": ("d_pairs", lambda r: 2 * r.n_pairs, "int32"),
    }

    def __getattr__(self, name):
        spec = Results._VIEWS.get(name)
        if spec is None:
            raise AttributeError(name)
        import torch
        field, length, dtype = spec
        t = self._scene._view(self._ptrs[field], length(self), getattr(torch, dtype))
        setattr(self, name, t)
        return t

    def __init__(self, scene: "Scene", r: SjResults):
        self._scene = scene
        self._ptrs = {f: getattr(r, f) for f, _, _ in Results._VIEWS.values()}
        self.nq = int(r.nq)
        self.n_leaves = int(r.n_leaves)
        self.n_isect_ids = int(r.n_isect_ids)
        self.n_cov_entries = int(r.n_cov_entries)
        self.n_runs = int(r.n_runs)
        self.n_pairs = int(r.n_pairs)
        self.total_pairs = int(r.total_pairs)
        self.n_present = int(r.n_present)
        self.n_tasks = int(r.n_tasks)
        self.n_subqueries = int(r.n_subqueries)
        self.cov_pairs = int(r.cov_pairs)
        self.tests = int(r.tests)
        self.error_bits = int(r.error_bits)

    def counters(self):
        """The tick's counters in the order of Scene.counters_into."""
        return [self.total_pairs, self.n_isect_ids, self.cov_pairs, self.n_subqueries,
                self.n_cov_entries, self.tests, self.n_tasks, self.error_bits]

    def to_lists(self, sel=None):
        """Per-query result lists in the canonical order (ascending ids),
        expanded and sorted on the device (sj_expand_results with SJ_SORTED);
        sel: optional query indices (all queries of the tick by default)."""
        off, ids = self._scene.expand(sel=sel, sorted=True)
        off = off.cpu().numpy()
        ids = ids.cpu().numpy().view(np.uint32)
        return [ids[off[i]:off[i + 1]].tolist() for i in range(len(off) - 1)]


class TickArgs:
    """Checked input tensors of one tick and their marshalled pointers (the
    tensors are held so that the pointers stay valid)."""
    __slots__ = ("c_args", "tensors")

    def __init__(self, c_args, tensors):
        self.c_args = c_args
        self.tensors = tensors


class Scene:
    """One moving-object set joined against range queries tick after tick.

    Inputs are torch CUDA tensors (uint32/int32 ids, float32 coordinates).
    """

    def __init__(self, capacity_objects: int, capacity_queries: int, *, th: int = 64,
                 th_min: int = 0, l_max: int = 16, covering: bool = True, reorder: bool = True,
                 rebuild: str = "auto", rebuild_period: int = 32, capacity_subqueries: int = 0,
                 capacity_covering: int = 0, capacity_results: int = 0, split_slots: int = 0,
                 profile: bool = False, timing_log: bool = False, thresh_mlp: bool = False,
                 schedule_mlp: bool = False, tune_every: int = 0, grid_split: int = 0,
                 atomic_results: bool = False, cu_counters: bool = False, device=None,
                 stream=None):
        import torch
        self._lib = load()
        self.device = torch.device(device if device is not None else "cuda")
        self.cfg = make_config(capacity_objects, capacity_queries, th=th, th_min=th_min,
                               l_max=l_max, covering=covering, reorder=reorder, rebuild=rebuild,
                               rebuild_period=rebuild_period,
                               capacity_subqueries=capacity_subqueries,
                               capacity_covering=capacity_covering,
                               capacity_results=capacity_results, split_slots=split_slots,
                               profile=profile, timing_log=timing_log, thresh_mlp=thresh_mlp,
                               schedule_mlp=schedule_mlp, tune_every=tune_every,
                               grid_split=grid_split, atomic_results=atomic_results,
                               cu_counters=cu_counters)
        nbytes = int(self._lib.sj_workspace_bytes(byref(self.cfg)))
        if nbytes == 0:
            raise SjError(SJ_EINVAL, "invalid configuration")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = c_void_p()
        rc = self._lib.sj_scene_create(byref(self.cfg), _ptr(self.ws), nbytes,
                                       c_void_p(self.stream.cuda_stream), byref(h))
        _check(rc, None)
        self.handle = h
        self._keep = []
        self._graph_key = None  # inputs of the last tick_graph call, checked and kept
        self._last_tick = None

    @property
    def workspace_bytes(self) -> int:
        return int(self.ws.numel())

    def close(self):
        if getattr(self, "handle", None):
            self._lib.sj_scene_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _view(self, ptr, count, dtype):
        import torch
        item = dtype.itemsize
        if count == 0 or not ptr:
            return torch.empty(0, dtype=dtype, device=self.device)
        off = int(ptr) - self.ws.data_ptr()
        assert 0 <= off and off + count * item <= self.ws.numel(), "view outside the workspace"
        return self.ws[off:off + count * item].view(dtype)

    @staticmethod
    def _dev(t, dtype, n=None):
        _require(t.is_cuda and t.is_contiguous() and t.dtype == dtype,
                 f"expected a contiguous CUDA tensor of {dtype}, got {t.dtype} "
                 f"(cuda={t.is_cuda}, contiguous={t.is_contiguous()})")
        if n is not None:
            _require(t.numel() == n, f"expected {n} elements, got {t.numel()}")
        return t

    def apply_updates(self, ids, x, y):
        import torch
        m = ids.numel()
        ids = self._dev(ids, ids.dtype if ids.dtype in (torch.int32, torch.uint32) else torch.int32)
        self._dev(x, torch.float32, m)
        self._dev(y, torch.float32, m)
        _check(self._lib.sj_apply_updates(self.handle, _ptr(ids), _ptr(x), _ptr(y), m), self.handle)
        self._keep = [ids, x, y]
        self._graph_key = None

    def build_index(self, th: int = 0):
        _check(self._lib.sj_build_index(self.handle, th), self.handle)

    def run_tick(self, qid, xa, ya, xb, yb):
        import torch
        nq = qid.numel()
        qid = self._dev(qid, qid.dtype if qid.dtype in (torch.int32, torch.uint32) else torch.int32)
        for t in (xa, ya, xb, yb):
            self._dev(t, torch.float32, nq)
        _check(self._lib.sj_run_tick(self.handle, _ptr(qid), _ptr(xa), _ptr(ya), _ptr(xb),
                                     _ptr(yb), nq), self.handle)
        self._keep = [qid, xa, ya, xb, yb]
        self._graph_key = None

    def run_knn(self, qid, qx, qy, k: int, out_id=None, out_d2=None):
        """Closes the tick with k-nearest-neighbour queries at points (qx,
        qy); returns (ids int32 [nq, k], d2 float32 [nq, k]), ascending by
        (d2, id), empty slots id -1 (0xffffffff) and d2 inf.  Synchronises."""
        import torch
        nq = qid.numel()
        qid = self._dev(qid, qid.dtype if qid.dtype in (torch.int32, torch.uint32) else torch.int32)
        self._dev(qx, torch.float32, nq)
        self._dev(qy, torch.float32, nq)
        if out_id is None:
            out_id = torch.empty((nq, k), dtype=torch.int32, device=self.device)
        if out_d2 is None:
            out_d2 = torch.empty((nq, k), dtype=torch.float32, device=self.device)
        self._dev(out_id, torch.int32, nq * k)
        self._dev(out_d2, torch.float32, nq * k)
        self._keep = [qid, qx, qy]
        self._graph_key = None
        _check(self._lib.sj_run_knn(self.handle, _ptr(qid), _ptr(qx), _ptr(qy), nq, int(k),
                                    _ptr(out_id), _ptr(out_d2)), self.handle)
        return out_id, out_d2

    def prepare_tick(self, ids, x, y, qid, xa, ya, xb, yb) -> "TickArgs":
        """Checks one tick's input tensors once; tick_graph(prepared) then
        launches without looking at them again."""
        import torch
        args = (ids, x, y, qid, xa, ya, xb, yb)
        m, nq = ids.numel(), qid.numel()
        for t in (ids, qid):
            _require(t.is_cuda and t.is_contiguous() and t.dtype in (torch.int32, torch.uint32),
                     "ids and qid must be contiguous CUDA int32/uint32 tensors")
        for t, n in ((x, m), (y, m), (xa, nq), (ya, nq), (xb, nq), (yb, nq)):
            self._dev(t, torch.float32, n)
        p = [_ptr(t) for t in args]
        return TickArgs((p[0], p[1], p[2], m, p[3], p[4], p[5], p[6], p[7], nq), args)

    def tick_graph(self, *args):
        """Updates + tick as one graph launch (captured once per quadtree
        decision and size, replayed afterwards on any buffers).  Takes the
        eight input tensors, or a TickArgs from prepare_tick."""
        if len(args) == 1 and isinstance(args[0], TickArgs):
            ta = args[0]
        else:
            key = tuple((id(t), t.data_ptr(), t.numel()) for t in args)
            if key != self._graph_key:  # the same tensors as the last call were checked then
                self._graph_args = self.prepare_tick(*args)
                self._graph_key = key
            ta = self._graph_args
        self._last_tick = ta  # its tensors live while the tick may still read them
        _check(self._lib.sj_tick_graph(self.handle, *ta.c_args), self.handle)

    def fetch(self) -> Results:
        r = SjResults()
        _check(self._lib.sj_fetch_results(self.handle, byref(r)), self.handle)
        return Results(self, r)

    def expand(self, sel=None, sorted: bool = False):
        """(off[n+1] int64, ids int32): per-query lists with covering leaves
        expanded, for every query of the tick or the query indices sel (a
        sequence or an int32 tensor); ascending ids per list if sorted."""
        import torch
        flags = SJ_SORTED if sorted else 0
        n = c_uint64()
        if sel is None:
            _check(self._lib.sj_expand_results(self.handle, None, 0, flags, None, None, 0,
                                               byref(n)), self.handle)
            r = SjResults()
            _check(self._lib.sj_fetch_results(self.handle, byref(r)), self.handle)
            nsel, dsel = int(r.nq), None
        else:
            if not isinstance(sel, torch.Tensor):
                sel = torch.from_numpy(np.ascontiguousarray(sel, dtype=np.uint32).view(np.int32))
            dsel = self._dev(sel.to(self.device).contiguous(), torch.int32)
            nsel = int(dsel.numel())
        off = torch.empty(nsel + 1, dtype=torch.int64, device=self.device)
        if dsel is not None:
            _check(self._lib.sj_expand_results(self.handle, _ptr(dsel), nsel, flags, _ptr(off),
                                               None, 0, byref(n)), self.handle)
        ids = torch.empty(max(int(n.value), 1), dtype=torch.int32, device=self.device)
        _check(self._lib.sj_expand_results(self.handle, _ptr(dsel) if dsel is not None else None,
                                           nsel, flags, _ptr(off), _ptr(ids), ids.numel(),
                                           byref(n)), self.handle)
        return off, ids[:int(n.value)]

    def cu_counters(self) -> np.ndarray:
        """Containment tests of the last tick's filtering per CU slot
        (SJ_CU_COUNTERS), uint64[CU_SLOTS]."""
        out = np.zeros(CU_SLOTS, np.uint64)
        _check(self._lib.sj_cu_counters(self.handle, out.ctypes.data_as(c_void_p), CU_SLOTS),
               self.handle)
        return out

    def hashes(self):
        """Per-query (count, pair-set hash) as int64 tensors (hash bits are
        the unsigned 64-bit value)."""
        import torch
        r = SjResults()
        _check(self._lib.sj_fetch_results(self.handle, byref(r)), self.handle)
        cnt = torch.empty(max(int(r.nq), 1), dtype=torch.int64, device=self.device)
        h = torch.empty(max(int(r.nq), 1), dtype=torch.int64, device=self.device)
        _check(self._lib.sj_result_hashes(self.handle, _ptr(cnt), _ptr(h)), self.handle)
        return cnt[:r.nq], h[:r.nq]

    def counters_into(self, out):
        """Enqueues a copy of the last tick's 8 counters into ``out`` (an
        int64 CUDA tensor of 8 elements, or a view of a larger one)."""
        import torch
        _require(out.is_cuda and out.dtype == torch.int64 and out.numel() >= 8,
                 "out must be a CUDA int64 tensor of at least 8 elements")
        _check(self._lib.sj_tick_counters(self.handle, _ptr(out)), self.handle)

    def stats(self, check: bool = True) -> dict:
        s = SjTickStats()
        rc = self._lib.sj_stats(self.handle, byref(s))
        if check:
            _check(rc, self.handle)
        d = {k: int(getattr(s, k)) for k, _ in SjTickStats._fields_}
        d["status"] = rc
        return d

    def phase_times(self) -> dict:
        buf = (c_float * len(PHASES))()
        _check(self._lib.sj_phase_times(self.handle, buf, len(PHASES)), self.handle)
        return {k: float(buf[i]) for i, k in enumerate(PHASES)}

    def set_cost_model(self, w, coef, cand):
        """Installs the cost model: w = BF16 parameters (int16/uint16 device
        tensor of sj_mlp_param_count() values, copied), coef = COST_TERMS floats,
        cand = candidate thresholds (1..8, each >= th_min)."""
        import torch
        _require(w.is_cuda and w.dtype in (torch.int16, torch.uint16) and w.is_contiguous(),
                 "weights must be a contiguous CUDA int16/uint16 tensor of bf16 bits")
        _require(len(coef) == COST_TERMS, f"expected {COST_TERMS} cost coefficients")
        cf = (c_float * COST_TERMS)(*[float(v) for v in coef])
        cd = (c_uint32 * len(cand))(*[int(v) for v in cand])
        _check(self._lib.sj_set_cost_model(self.handle, _ptr(w), cf, cd, len(cand)), self.handle)

    def tune_info(self) -> dict:
        t = SjTuneInfo()
        _check(self._lib.sj_tune_info_get(self.handle, byref(t)), self.handle)
        n = int(t.n_cand)
        return dict(cand=list(t.cand[:n]), cost=list(t.cost[:n]), mlp_sum=list(t.mlp_sum[:n]),
                    mlp_max=list(t.mlp_max[:n]),
                    chosen=int(t.chosen), n_tunes=int(t.n_tunes), tuned_tick=int(t.tuned_tick))

    def timing_log(self):
        """(records [n_leaves, 8] float32 device view, clock MHz) of the
        last tick: objects, intersecting subqueries, level, mean overlap,
        count-pass ticks, write-pass ticks, 0, 0."""
        import torch
        v = SjTimingView()
        _check(self._lib.sj_timing_log(self.handle, byref(v)), self.handle)
        rec = self._view(v.d_records, int(v.n_leaves) * 8, torch.float32)
        return rec.view(int(v.n_leaves), 8), float(v.clock_mhz)

    def index_view(self) -> dict:
        import torch
        v = SjIndexView()
        _check(self._lib.sj_index_view_get(self.handle, byref(v)), self.handle)
        n, L = int(v.n_present), int(v.n_leaves)
        return dict(n_present=n, n_leaves=L, l_deep=int(v.l_deep), x0=float(v.x0),
                    y0=float(v.y0), e=int(v.e),
                    codes=self._view(v.d_codes, n, torch.int32),
                    ids=self._view(v.d_ids, n, torch.int32),
                    leaf_start=self._view(v.d_leaf_start, L, torch.int32),
                    leaf_level=self._view(v.d_leaf_level, L, torch.int32),
                    leaf_beg=self._view(v.d_leaf_beg, L + 1, torch.int32),
                    pos=self._view(v.d_pos, 2 * self.cfg.capacity_objects,
                                   torch.float32).view(-1, 2))


class Server:
    """Tick-serving runtime (sj_server_*): scenes admitted by the memory of
    one device pool, ticks of different scenes overlapping on the device."""

    def __init__(self, pool_bytes: int, max_running: int = 4, device=None):
        import torch
        self._lib = load()
        self.device = torch.device(device if device is not None else "cuda")
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=self.device)
        h = c_void_p()
        rc = self._lib.sj_server_create(_ptr(self.pool), self.pool.numel(), max_running, byref(h))
        if rc != SJ_OK:
            raise SjError(rc, self._lib.sj_server_last_error(None).decode())
        self.handle = h
        self._keep = {}
        self._done = (SjServed * 256)()
        self._inflight = {}

    def _check(self, rc):
        if rc != SJ_OK:
            raise SjError(rc, self._lib.sj_server_last_error(self.handle).decode())

    def scene_bytes(self, cfg: SjConfig, max_updates: int) -> int:
        return int(self._lib.sj_server_scene_bytes(byref(cfg), max_updates))

    def admit(self, cfg: SjConfig, max_updates: int):
        """Scene id, or None if the scene does not fit in the pool now."""
        sid = c_uint32()
        rc = self._lib.sj_server_admit(self.handle, byref(cfg), max_updates, byref(sid))
        if rc == SJ_ENOSPACE:
            return None
        self._check(rc)
        return int(sid.value)

    def add(self, cfg: SjConfig, max_updates: int) -> int:
        """Scene id of a scene admitted on demand and evicted when idle."""
        sid = c_uint32()
        self._check(self._lib.sj_server_add(self.handle, byref(cfg), max_updates, byref(sid)))
        return int(sid.value)

    def evict(self, sid: int):
        """Moves an idle resident scene to host memory (sj_server_evict)."""
        self._check(self._lib.sj_server_evict(self.handle, sid))

    def retire(self, sid: int):
        self._check(self._lib.sj_server_retire(self.handle, sid))
        self._keep.pop(sid, None)

    def submit(self, sid: int, tag: int, ids, x, y, qid, xa, ya, xb, yb, record=None,
               digest: bool = False):
        """record: optional int64 CUDA tensor view of 10 elements receiving
        the tick's counters and (with digest) the result digest."""
        m, nq = ids.numel(), qid.numel()
        self._check(self._lib.sj_server_submit(self.handle, sid, _ptr(ids), _ptr(x), _ptr(y), m,
                                               _ptr(qid), _ptr(xa), _ptr(ya), _ptr(xb),
                                               _ptr(yb), nq, tag, _ptr(record),
                                               1 if digest else 0))
        # the tick reads these until it is retired
        self._inflight[(sid, tag)] = (ids, x, y, qid, xa, ya, xb, yb, record)

    def poll(self):
        """Finished ticks: list of (scene, tag, status, nq, count_ptr,
        hash_ptr, counters_ptr); outputs stay valid until the scene's next
        tick is retired."""
        n = c_uint32()
        self._check(self._lib.sj_server_poll(self.handle, self._done, len(self._done), byref(n)))
        done = self._done[:n.value]
        for d in done:
            self._inflight.pop((d.scene_id, d.tag), None)
        return [(d.scene_id, d.tag, d.status, d.nq, d.d_count, d.d_hash, d.d_counters)
                for d in done]

    def info(self) -> dict:
        st = SjServerStats()
        self._check(self._lib.sj_server_info(self.handle, byref(st)))
        return {k: int(getattr(st, k)) for k, _ in SjServerStats._fields_}

    def close(self):
        if getattr(self, "handle", None):
            self._lib.sj_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
