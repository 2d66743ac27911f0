"""Pins of the cost-model MLP oracle: BF16 rounding closed forms, analytic
gradients against central finite differences, closed-form gradients with a
zero hidden layer, and the first Adam step."""
import numpy as np
import pytest

from oracle import mlp

F32 = np.float32


def test_bf16_round_to_nearest_even_closed_forms():
    v = np.array([1.0, 1 + 2**-8, 1 + 3 * 2**-8, 1 + 2**-8 + 2**-20, -2.5, 3.14159274,
                  65504.0, 2**-130], F32)
    bits = mlp.bf16_bits(v)
    # ties go to the even mantissa; above the tie rounds up; pi truncates to
    # 3.140625; a subnormal keeps its top bits
    assert [int(b) for b in bits[:5]] == [0x3F80, 0x3F80, 0x3F82, 0x3F81, 0xC020]
    assert mlp.bf16_value(bits[5]) == F32(3.140625)
    assert mlp.bf16_value(bits[6]) == F32(65536.0)  # 65504 rounds up to 2^16
    assert bits[7] == (np.array([2**-130], F32).view(np.uint32)[0] >> 16)
    nan = mlp.bf16_bits(np.array([np.nan], F32))
    assert np.isnan(mlp.bf16_value(nan))[0]


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    p = mlp.bf16_round(mlp.init_params(1) + rng.normal(0, 0.05, mlp.P).astype(F32)).astype(np.float64)
    X = rng.normal(0, 1, (40, 4))
    T = rng.normal(0, 1, 40)
    L, g = mlp.loss_grad(p, X, T)
    assert abs(L - np.mean((mlp.forward(p, X) - T) ** 2)) < 1e-12
    h = 1e-4
    idx = np.r_[rng.choice(mlp.P - 1, 60, replace=False), mlp.P - 1, 0, 256, 320, 4416, 4480]
    for i in idx:
        e = np.zeros(mlp.P)
        e[i] = h
        fd = (mlp.loss_grad(p + e, X, T)[0] - mlp.loss_grad(p - e, X, T)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-5 * max(1.0, abs(g[i])) + 1e-7, i


def test_gradient_closed_form_with_zero_hidden_weights():
    rng = np.random.default_rng(2)
    p = np.zeros(mlp.P)
    q = mlp.unpack(p)  # views into p
    q["W1"][:] = rng.normal(0, 1, (64, 4))
    q["b2"][:] = np.abs(rng.normal(0, 1, 64)) + 0.1  # h2 = b2 > 0 whatever h1 is
    q["w3"][:] = rng.normal(0, 1, 64)
    p[-1] = 0.3
    X = rng.normal(0, 1, (25, 4))
    T = rng.normal(0, 1, 25)
    L, g = mlp.loss_grad(p, X, T)
    y = q["w3"] @ q["b2"] + 0.3
    r = y - T
    gq = mlp.unpack(g)
    assert np.allclose(gq["b3"], 2 * r.mean())
    assert np.allclose(gq["w3"], 2 * r.mean() * q["b2"])
    assert np.allclose(gq["b2"], 2 * r.mean() * q["w3"])
    h1 = np.maximum(X @ q["W1"].T, 0)
    assert np.allclose(gq["W2"], 2 * np.outer(q["w3"], (r[:, None] * h1).mean(axis=0)))
    assert np.allclose(gq["W1"], 0) and np.allclose(gq["b1"], 0)


def test_first_adam_step_moves_by_lr_times_sign():
    g = np.array([0.5, -2.0, 1e-3])
    w, m, v = mlp.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(w, -0.01 * np.sign(g), rtol=1e-4)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
