"""CPU oracle for the per-tick spatial join (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP path in
``paper_1411_3212_amd`` and never imports it.

The arithmetic lives in ``sj_oracle.c`` (plain C, gcc, OpenMP over queries);
this module only compiles it and marshals numpy arrays.  What each function
computes, with the passage of the paper it follows:

* ``apply_updates`` / ``live_queries`` -- tick batching: the most recent
  update / query of an object within a tick is the one that counts
  (Section "Batch processing").
* ``brute_counts`` / ``brute_lists`` / ``brute_hash`` -- Definition 1 (result
  set of a range query), a closed rectangle, written out as a nested loop.
* ``grid_hash`` -- the same definition through an independent uniform grid
  (double-precision cell mapping), a second check at scale.
* ``frame`` / ``cell`` / ``morton`` -- the index frame over the objects' MBR
  and the finest-level cell mapping shared by objects and query corners
  (Definitions 2-4, mapping functions f and g).
* ``sorted_codes`` + ``quadtree`` -- Algorithm 1 (PR-quadtree construction):
  Morton codes at the finest level, stable sort, level-wise split of every
  quadrant holding more than th objects until no quadrant needs splitting
  or l_max is reached.
* ``split`` -- query splitting into intersecting and covering subqueries
  (mapping function g; indexing of queries).
* ``mix64`` -- SplitMix64's output function, used by the pair-set hash.
* ``knn`` / ``knn_d2`` -- repeated k-nearest-neighbour queries (the
  paper's future work, Section "Conclusions"): the k present objects of
  smallest (binary32 squared distance, id), by brute force.
* ``ug_col`` / ``ug_cells`` / ``ug_split`` -- the uniform grid of the UG
  method (Definition "MBR partitioning into a uniform grid"; UG index
  creation and query indexing): columns and rows of the frame along its
  finest cells, cells numbered by Morton code, query splitting by the
  nested loop over the query's cell range.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "sj_oracle.c"
_LIB = _HERE / "_build" / "libsj_oracle.so"

_lib = None


def build(force: bool = False) -> Path:
    """Compile ``sj_oracle.c`` with gcc into ``oracle/_build``."""
    if _LIB.exists() and not force and _LIB.stat().st_mtime >= _SRC.stat().st_mtime:
        return _LIB
    _LIB.parent.mkdir(parents=True, exist_ok=True)
    tmp = _LIB.with_suffix(".so.tmp%d" % os.getpid())
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-o", str(tmp), str(_SRC), "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    lib = ctypes.CDLL(str(build()))
    P = ctypes.c_void_p
    u32, i32, u64, i64 = ctypes.c_uint32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64
    sig = {
        "or_apply_updates": (i64, [u32, P, P, P, u32, P, P, P]),
        "or_live_queries": (None, [u32, u32, P, P]),
        "or_brute_counts": (i64, [u32, P, P, P, u32, P, P, P, P, P, P]),
        "or_brute_lists": (None, [u32, P, P, P, u32, P, P, P, P, P, P, P]),
        "or_brute_hash": (i64, [u32, P, P, P, u32, P, P, P, P, P, P, P, P]),
        "or_grid_hash": (i64, [u32, P, P, P, u32, P, P, P, P, P, P, P, P]),
        "or_mix64": (u64, [u64]),
        "or_frame": (ctypes.c_int, [u32, P, P, P, P, P, P]),
        "or_cell": (u32, [ctypes.c_float, ctypes.c_float, i32]),
        "or_morton": (u32, [u32, u32, u32]),
        "or_sorted_codes": (u32, [u32, P, P, P, ctypes.c_float, ctypes.c_float, i32, P, P]),
        "or_quadtree": (i64, [u32, P, u32, u32, u64, P, P, P, P, P]),
        "or_split": (None, [u32, P, P, P, P, P, ctypes.c_float, ctypes.c_float, i32,
                            u32, P, P, P, P, P, P, P, P]),
        "or_num_threads": (ctypes.c_int, []),
        "or_set_num_threads": (None, [ctypes.c_int]),
        "or_ug_col": (u32, [u32, u32]),
        "or_ug_bits": (u32, [u32]),
        "or_ug_cells": (None, [u32, P, P, P, ctypes.c_float, ctypes.c_float, i32, u32, P]),
        "or_ug_split": (None, [u32, P, P, P, P, P, ctypes.c_float, ctypes.c_float, i32, u32,
                               P, P, P, P, P, P, P]),
        "or_knn": (None, [u32, P, P, P, u32, P, P, P, u32, P, P]),
        "or_knn_d2": (ctypes.c_float, [ctypes.c_float] * 4),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _u32(a):
    return np.ascontiguousarray(a, dtype=np.uint32)


def num_threads() -> int:
    return int(_load().or_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's loops over queries (1: single core)."""
    _load().or_set_num_threads(int(n))


class State:
    """Last-known positions of N objects indexed by id (``has`` marks objects
    that have received at least one update)."""

    def __init__(self, n_cap: int):
        self.N = int(n_cap)
        self.px = np.zeros(self.N, np.float32)
        self.py = np.zeros(self.N, np.float32)
        self.has = np.zeros(self.N, np.uint8)

    def copy(self) -> "State":
        s = State(self.N)
        s.px[:] = self.px
        s.py[:] = self.py
        s.has[:] = self.has
        return s


def apply_updates(st: State, ids, x, y) -> int:
    ids, x, y = _u32(ids), _f32(x), _f32(y)
    return int(_load().or_apply_updates(st.N, _p(st.px), _p(st.py), _p(st.has),
                                        len(ids), _p(ids), _p(x), _p(y)))


def live_queries(n_cap: int, qid) -> np.ndarray:
    qid = _u32(qid)
    live = np.zeros(len(qid), np.uint8)
    _load().or_live_queries(int(n_cap), len(qid), _p(qid), _p(live))
    return live


def _q(rects):
    xa, ya, xb, yb = (_f32(r) for r in rects)
    return xa, ya, xb, yb


def brute_counts(st: State, live, rects) -> np.ndarray:
    xa, ya, xb, yb = _q(rects)
    live = np.ascontiguousarray(live, np.uint8)
    cnt = np.zeros(len(xa), np.uint64)
    _load().or_brute_counts(st.N, _p(st.px), _p(st.py), _p(st.has), len(xa), _p(live),
                            _p(xa), _p(ya), _p(xb), _p(yb), _p(cnt))
    return cnt


def brute_lists(st: State, live, rects):
    """Per-query result sets, ascending ids: returns (off[nq+1], ids)."""
    xa, ya, xb, yb = _q(rects)
    live = np.ascontiguousarray(live, np.uint8)
    cnt = brute_counts(st, live, (xa, ya, xb, yb))
    off = np.zeros(len(xa) + 1, np.uint64)
    np.cumsum(cnt, out=off[1:])
    ids = np.zeros(int(off[-1]), np.uint32)
    _load().or_brute_lists(st.N, _p(st.px), _p(st.py), _p(st.has), len(xa), _p(live),
                           _p(xa), _p(ya), _p(xb), _p(yb), _p(off), _p(ids))
    return off, ids


def brute_hash(st: State, qid, live, rects):
    """Per-query (count, pair-set hash) by brute force."""
    xa, ya, xb, yb = _q(rects)
    qid = _u32(qid)
    live = np.ascontiguousarray(live, np.uint8)
    cnt = np.zeros(len(xa), np.uint64)
    h = np.zeros(len(xa), np.uint64)
    _load().or_brute_hash(st.N, _p(st.px), _p(st.py), _p(st.has), len(xa), _p(qid), _p(live),
                          _p(xa), _p(ya), _p(xb), _p(yb), _p(cnt), _p(h))
    return cnt, h


def grid_hash(st: State, qid, live, rects):
    """Per-query (count, pair-set hash) through the CPU uniform grid."""
    xa, ya, xb, yb = _q(rects)
    qid = _u32(qid)
    live = np.ascontiguousarray(live, np.uint8)
    cnt = np.zeros(len(xa), np.uint64)
    h = np.zeros(len(xa), np.uint64)
    _load().or_grid_hash(st.N, _p(st.px), _p(st.py), _p(st.has), len(xa), _p(qid), _p(live),
                         _p(xa), _p(ya), _p(xb), _p(yb), _p(cnt), _p(h))
    return cnt, h


def mix64(v: int) -> int:
    return int(_load().or_mix64(ctypes.c_uint64(v & (2**64 - 1))))


def frame(st: State):
    """(x0, y0, e, n_present): frame anchored at the MBR's lower-left corner
    with side 2**e."""
    x0 = np.zeros(1, np.float32)
    y0 = np.zeros(1, np.float32)
    e = np.zeros(1, np.int32)
    n = _load().or_frame(st.N, _p(st.px), _p(st.py), _p(st.has), _p(x0), _p(y0), _p(e))
    return float(x0[0]), float(y0[0]), int(e[0]), int(n)


def cell(v: float, v0: float, e: int) -> int:
    return int(_load().or_cell(ctypes.c_float(v), ctypes.c_float(v0), int(e)))


def morton(i: int, j: int, nbits: int = 16) -> int:
    return int(_load().or_morton(i, j, nbits))


def sorted_codes(st: State, fr):
    x0, y0, e = fr[0], fr[1], fr[2]
    codes = np.zeros(st.N, np.uint32)
    ids = np.zeros(st.N, np.uint32)
    n = _load().or_sorted_codes(st.N, _p(st.px), _p(st.py), _p(st.has),
                                ctypes.c_float(x0), ctypes.c_float(y0), int(e),
                                _p(codes), _p(ids))
    return codes[:n].copy(), ids[:n].copy()


class Leaves:
    """Quadtree leaves in Morton order: level, code at that level and the
    [beg, end) range of the sorted objects they hold."""

    def __init__(self, lvl, z, beg, end, l_deep):
        self.lvl, self.z, self.beg, self.end, self.l_deep = lvl, z, beg, end, l_deep

    def __len__(self):
        return len(self.lvl)

    @property
    def count(self):
        return (self.end.astype(np.int64) - self.beg.astype(np.int64))

    @property
    def start(self):
        """First finest-level (16-bit per axis) Morton code of each leaf."""
        return self.z.astype(np.uint64) << (2 * (16 - self.lvl.astype(np.uint64)))


def quadtree(codes, th: int, l_max: int = 16) -> Leaves:
    codes = _u32(codes)
    cap = 4 * (len(codes) // max(int(th), 1) + 1) * 17 + 64
    lvl = np.zeros(cap, np.uint32)
    z = np.zeros(cap, np.uint32)
    beg = np.zeros(cap, np.uint32)
    end = np.zeros(cap, np.uint32)
    ld = np.zeros(1, np.uint32)
    n = _load().or_quadtree(len(codes), _p(codes), int(th), int(l_max), cap,
                            _p(lvl), _p(z), _p(beg), _p(end), _p(ld))
    if n < 0:
        raise RuntimeError("leaf capacity exceeded")
    return Leaves(lvl[:n].copy(), z[:n].copy(), beg[:n].copy(), end[:n].copy(), int(ld[0]))


def split(live, rects, fr, leaves: Leaves):
    """Query splitting: returns (oi, li, oc, lc): CSR offsets and leaf indices
    of the intersecting and covering subqueries of each query."""
    xa, ya, xb, yb = _q(rects)
    live = np.ascontiguousarray(live, np.uint8)
    nq = len(xa)
    lib = _load()
    ni = np.zeros(nq, np.uint64)
    nc = np.zeros(nq, np.uint64)
    args = (nq, _p(live), _p(xa), _p(ya), _p(xb), _p(yb),
            ctypes.c_float(fr[0]), ctypes.c_float(fr[1]), int(fr[2]),
            len(leaves), _p(leaves.lvl), _p(leaves.z))
    lib.or_split(*args, _p(ni), _p(nc), None, None, None, None)
    oi = np.zeros(nq + 1, np.uint64)
    oc = np.zeros(nq + 1, np.uint64)
    np.cumsum(ni, out=oi[1:])
    np.cumsum(nc, out=oc[1:])
    li = np.zeros(int(oi[-1]), np.uint32)
    lc = np.zeros(int(oc[-1]), np.uint32)
    lib.or_split(*args, None, None, _p(oi), _p(oc), _p(li), _p(lc))
    return oi, li, oc, lc


def ug_col(fine: int, s: int) -> int:
    """Grid column (or row) of a finest-level cell for split factor s."""
    return int(_load().or_ug_col(int(fine), int(s)))


def ug_bits(s: int) -> int:
    return int(_load().or_ug_bits(int(s)))


def ug_cells(st: State, fr, s: int) -> np.ndarray:
    """Grid cell (Morton code over ug_bits(s) bits per axis) of every object
    by id; 0xffffffff for objects without a position."""
    cell = np.zeros(st.N, np.uint32)
    _load().or_ug_cells(st.N, _p(st.px), _p(st.py), _p(st.has), ctypes.c_float(fr[0]),
                        ctypes.c_float(fr[1]), int(fr[2]), int(s), _p(cell))
    return cell


def ug_split(live, rects, fr, s: int, count):
    """Query splitting over the grid: (oi, li, oc, lc) as ``split``, with
    cell Morton codes in place of leaf indices; count[z] = objects of cell z
    (cells without objects are skipped)."""
    xa, ya, xb, yb = _q(rects)
    live = np.ascontiguousarray(live, np.uint8)
    count = _u32(count)
    nq = len(xa)
    lib = _load()
    ni = np.zeros(nq, np.uint64)
    nc = np.zeros(nq, np.uint64)
    args = (nq, _p(live), _p(xa), _p(ya), _p(xb), _p(yb), ctypes.c_float(fr[0]),
            ctypes.c_float(fr[1]), int(fr[2]), int(s), _p(count))
    lib.or_ug_split(*args, _p(ni), _p(nc), None, None, None, None)
    oi = np.zeros(nq + 1, np.uint64)
    oc = np.zeros(nq + 1, np.uint64)
    np.cumsum(ni, out=oi[1:])
    np.cumsum(nc, out=oc[1:])
    li = np.zeros(int(oi[-1]), np.uint32)
    lc = np.zeros(int(oc[-1]), np.uint32)
    lib.or_ug_split(*args, None, None, _p(oi), _p(oc), _p(li), _p(lc))
    return oi, li, oc, lc


def knn(st: State, live, qx, qy, k: int):
    """k nearest present objects of every live query point, ascending by
    (binary32 squared distance, id): returns (ids[nq, k], d2[nq, k]); empty
    slots hold id 0xffffffff and d2 = inf."""
    qx, qy = _f32(qx), _f32(qy)
    live = np.ascontiguousarray(live, np.uint8)
    nq = len(qx)
    ids = np.zeros((nq, max(k, 0)), np.uint32)
    d2 = np.zeros((nq, max(k, 0)), np.float32)
    _load().or_knn(st.N, _p(st.px), _p(st.py), _p(st.has), nq, _p(live), _p(qx), _p(qy),
                   int(k), _p(ids), _p(d2))
    return ids, d2


def knn_d2(px: float, py: float, qx: float, qy: float) -> float:
    """The binary32 squared distance of the kNN definition for one pair."""
    return float(_load().or_knn_d2(px, py, qx, qy))
