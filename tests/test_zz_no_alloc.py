"""The gradient entry point that allocates nothing (its per-block partials
in a fixed array inside the library) against the one that takes a scratch
buffer: the same kernels, so the gradients must be identical bit for bit.
Two calls in a row, the second on fewer samples, so that the second reads
nothing the first left behind."""
import ctypes

import numpy as np
import pytest

from paper_1411_3212_amd import binding

pytestmark = pytest.mark.gpu


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _call(name, *args):
    lib = binding.load()
    rc = getattr(lib, name)(*args)
    assert rc == 0, f"{name} returned {rc}: {lib.sj_last_error(None).decode()}"


def test_grad_noalloc_equals_grad_with_scratch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lib = binding.load()
    P = int(lib.sj_mlp_param_count())
    assert lib.sj_mlp_noalloc_scratch_bytes() >= 256 * (P + 1) * 4
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rng = np.random.default_rng(12)
    master = torch.from_numpy(rng.normal(0, 0.3, P).astype(np.float32)).cuda()
    w = torch.empty(P, dtype=torch.int16, device="cuda")
    _call("sj_mlp_round", _ptr(master), _ptr(w), stream)
    for n in (20000, 777):
        X = torch.from_numpy(rng.random((n, 4)).astype(np.float32)).cuda()
        T = torch.from_numpy(rng.normal(2.0, 1.0, n).astype(np.float32)).cuda()
        want = torch.full((P + 1,), np.nan, dtype=torch.float32, device="cuda")
        got = torch.full((P + 1,), np.nan, dtype=torch.float32, device="cuda")
        nb = int(lib.sj_mlp_scratch_bytes(n))
        scratch = torch.empty(nb, dtype=torch.uint8, device="cuda")
        _call("sj_mlp_grad", _ptr(w), _ptr(X), _ptr(T), n, _ptr(want), _ptr(scratch), nb, stream)
        _call("sj_mlp_grad_noalloc", _ptr(w), _ptr(X), _ptr(T), n, _ptr(got), stream)
        torch.cuda.synchronize()
        a = want.cpu().numpy().view(np.uint32)
        b = got.cpu().numpy().view(np.uint32)
        assert np.isfinite(want.cpu().numpy()).all()
        assert np.array_equal(a, b), f"n={n}: {np.count_nonzero(a != b)} entries differ"
        print(f"n={n}: loss {float(want[-1]):.6f}, {P} gradient entries identical", flush=True)
