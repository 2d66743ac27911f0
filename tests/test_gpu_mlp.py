"""The cost-model MLP kernels against the FP64 oracle: BF16 rounding
bit-exact, forward and gradient within the stated tolerance, Adam, and a
short training run that fits a smooth target."""
import ctypes

import numpy as np
import pytest

from oracle import mlp
from paper_1411_3212_amd import binding

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.synchronize()


def call(name, *args):
    """Calls an sj_mlp_* entry point; a failure raises with the library's
    message (device tensors are never formatted)."""
    rc = getattr(lib(), name)(*args)
    if rc != 0:
        raise RuntimeError(f"{name} returned {rc}: {lib().sj_last_error(None).decode()}")


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def lib():
    return binding.load()


def rounded(master):
    import torch
    w = torch.empty(mlp.P, dtype=torch.int16, device="cuda")
    call("sj_mlp_round", ptr(master), ptr(w), None)
    return w


def test_param_count_and_rounding_bit_exact():
    import torch
    pr = torch.cuda.get_device_properties(0)
    print("device", pr.name, "LDS per block", getattr(pr, "shared_memory_per_block", "?"), flush=True)
    assert lib().sj_mlp_param_count() == mlp.P
    rng = np.random.default_rng(0)
    p = np.concatenate([rng.normal(0, 3, mlp.P - 6), [1 + 2**-8, 1 + 3 * 2**-8, 65504, 2**-130,
                                                      -0.0, 3.14159274]]).astype(np.float32)
    w = rounded(dev(p)).cpu().numpy().view(np.uint16)
    assert np.array_equal(w, mlp.bf16_bits(p))


def forward_gpu(w, X):
    import torch
    y = torch.empty(len(X), dtype=torch.float32, device="cuda")
    dX = dev(X.astype(np.float32))  # held: a freed block would be reused by the next allocation
    call("sj_mlp_forward", ptr(w), ptr(dX), len(X), ptr(y), None)
    return y.cpu().numpy().astype(np.float64)


def grad_gpu(w, X, T):
    import torch
    n = len(X)
    g = torch.empty(mlp.P + 1, dtype=torch.float32, device="cuda")
    nb = lib().sj_mlp_scratch_bytes(n)
    scratch = torch.empty(nb, dtype=torch.uint8, device="cuda")
    dX, dT = dev(X.astype(np.float32)), dev(T.astype(np.float32))
    call("sj_mlp_grad", ptr(w), ptr(dX), ptr(dT), n, ptr(g), ptr(scratch), nb, None)
    out = g.cpu().numpy().astype(np.float64)
    return out[-1], out[:-1]


@pytest.mark.parametrize("n", [1, 63, 64, 1000, 20011])
def test_forward_and_gradient_match_oracle(n):
    rng = np.random.default_rng(n)
    master = (mlp.init_params(3) + rng.normal(0, 0.05, mlp.P)).astype(np.float32)
    w = rounded(dev(master))
    p = mlp.bf16_round(master).astype(np.float64)
    X = np.c_[rng.uniform(0, 7, n), rng.uniform(0, 6, n), rng.uniform(0, 1, n),
              rng.uniform(0, 1, n)].astype(np.float32)
    T = rng.normal(1.0, 0.5, n).astype(np.float32)
    y = forward_gpu(w, X)
    yo = mlp.forward(p, X)
    assert np.allclose(y, yo, rtol=1e-4, atol=1e-4 * np.abs(yo).max())
    L, g = grad_gpu(w, X, T)
    Lo, go = mlp.loss_grad(p, X, T)
    assert abs(L - Lo) <= 1e-4 * Lo + 1e-7
    # |delta| <= 1e-3 (|g| + 1e-3 max|g|)
    assert np.all(np.abs(g - go) <= 1e-3 * (np.abs(go) + 1e-3 * np.abs(go).max()))


def test_adam_step_matches_oracle():
    import torch
    rng = np.random.default_rng(4)
    master = mlp.init_params(5)
    grad = rng.normal(0, 1, mlp.P).astype(np.float32)
    m = rng.normal(0, 0.1, mlp.P).astype(np.float32)
    v = np.abs(rng.normal(0, 0.1, mlp.P)).astype(np.float32)
    dm, dg, dmm, dv = dev(master.copy()), dev(grad), dev(m.copy()), dev(v.copy())
    w = torch.empty(mlp.P, dtype=torch.int16, device="cuda")
    call("sj_mlp_adam", ptr(dm), ptr(dg), ptr(dmm), ptr(dv), ptr(w), 3, ctypes.c_float(1e-3), None)
    wo, mo, vo = mlp.adam_step(master.astype(np.float64), grad, m, v, 3, 1e-3)
    hm, hmm, hv = dm.cpu().numpy(), dmm.cpu().numpy(), dv.cpu().numpy()
    assert np.allclose(hm, wo, rtol=1e-5, atol=1e-7)
    # FP32 moments: a few ulps of their terms (|m|, |g| <= ~5)
    assert np.allclose(hmm, mo, rtol=1e-5, atol=1e-6) and np.allclose(hv, vo, rtol=1e-5, atol=1e-6)
    hw = w.cpu().numpy().view(np.uint16)
    assert np.array_equal(hw, mlp.bf16_bits(hm))


def test_training_fits_a_smooth_target():
    import torch
    rng = np.random.default_rng(6)
    n = 8192
    X = np.c_[rng.uniform(0, 7, n), rng.uniform(0, 6, n), rng.uniform(0, 1, n),
              rng.uniform(0, 1, n)].astype(np.float32)
    T = (0.4 * X[:, 0] + 0.3 * X[:, 1] * X[:, 3] - X[:, 2] + 0.5).astype(np.float32)
    master = dev(mlp.init_params(7))
    m = torch.zeros(mlp.P, device="cuda")
    v = torch.zeros(mlp.P, device="cuda")
    w = rounded(master)
    dX, dT = dev(X), dev(T)
    g = torch.empty(mlp.P + 1, device="cuda")
    nb = lib().sj_mlp_scratch_bytes(n)
    scratch = torch.empty(nb, dtype=torch.uint8, device="cuda")
    losses = []
    for step in range(1, 401):
        call("sj_mlp_grad", ptr(w), ptr(dX), ptr(dT), n, ptr(g), ptr(scratch), nb, None)
        if step in (1, 400):
            losses.append(float(g[-1].item()))
        call("sj_mlp_adam", ptr(master), ptr(g), ptr(m), ptr(v), ptr(w), step, ctypes.c_float(3e-3),
             None)
    assert losses[1] < 0.05 * losses[0], losses
