"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function include/sj.h declares, and sizes workspaces sensibly."""
import ctypes
import re
from pathlib import Path

import pytest

from paper_1411_3212_amd import binding

HEADER = Path(__file__).resolve().parents[1] / "include" / "sj.h"


def declared_functions():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sj_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    names = declared_functions()
    assert len(names) >= 13
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(binding.EXPORTS)


def test_workspace_bytes_and_config_validation():
    lib = binding.load()
    cfg = binding.SjConfig(1_000_000, 100_000, 0, 0, 0, 64, 0, 16, 3, 0, 32, 0)
    n = lib.sj_workspace_bytes(ctypes.byref(cfg))
    assert n > 1_000_000 * 40 and n % 256 == 0
    cfg2 = binding.SjConfig(1_000_000, 100_000, 0, 0, 0, 64, 16, 16, 3, 0, 32, 0)
    assert lib.sj_workspace_bytes(ctypes.byref(cfg2)) > n  # smaller th_min: larger leaf table
    for bad in [binding.SjConfig(0, 1, 0, 0, 0, 64, 0, 16, 3, 0, 32, 0),
                binding.SjConfig(10, 1, 0, 0, 0, 64, 0, 17, 3, 0, 32, 0),
                binding.SjConfig(10, 1, 0, 0, 0, 8, 16, 16, 3, 0, 32, 0),
                binding.SjConfig(10, 1, 2**32, 0, 0, 64, 0, 16, 3, 0, 32, 0),
                binding.SjConfig(10, 1, 0, 0, 0, 64, 0, 16, 3, 7, 32, 0)]:
        assert lib.sj_workspace_bytes(ctypes.byref(bad)) == 0


def test_create_rejects_bad_workspace_without_touching_the_device():
    lib = binding.load()
    cfg = binding.SjConfig(1000, 100, 0, 0, 0, 64, 0, 16, 3, 0, 32, 0)
    h = ctypes.c_void_p()
    assert lib.sj_scene_create(ctypes.byref(cfg), None, 0, None, ctypes.byref(h)) == binding.SJ_EINVAL
    assert lib.sj_scene_create(ctypes.byref(cfg), ctypes.c_void_p(256), 10, None,
                               ctypes.byref(h)) == binding.SJ_ENOSPACE
    assert b"needs" in lib.sj_last_error(None)
    assert lib.sj_scene_create(ctypes.byref(cfg), ctypes.c_void_p(8), 1 << 30, None,
                               ctypes.byref(h)) == binding.SJ_EINVAL
