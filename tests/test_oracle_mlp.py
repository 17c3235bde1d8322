"""Pins of the surrogate's FP64 twin: bfloat16 rounding on known values,
gradients against central finite differences (unquantised network), and the
closed-form first Adam step."""

import numpy as np

from oracle import mlp


def test_bf16_rounding_known_values():
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7 -> ties to even (1.0)
    assert mlp.bf16(1.0 + 2.0 ** -8) == 1.0
    # 1 + 3 * 2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6 -> ties to even (1 + 2^-6)
    assert mlp.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    # just above a tie rounds up
    assert mlp.bf16(np.float32(1.0 + 2.0 ** -8 + 2.0 ** -20)) == 1.0 + 2.0 ** -7
    assert mlp.bf16(-2.5) == -2.5 and mlp.bf16(0.0) == 0.0
    # unit roundoff 2^-8 (8 significant bits) for normal numbers
    x = np.random.default_rng(0).standard_normal(10000) * 100
    assert np.all(np.abs(mlp.bf16(x) - x.astype(np.float32)) <= 2.0 ** -8 * np.abs(x) + 1e-30)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    theta = mlp.init_params(3).astype(np.float64)
    n = 7
    inputs = rng.standard_normal((n, mlp.N_IN))
    targets = rng.standard_normal((n, mlp.N_OUT)) * 0.3
    mean, std = np.zeros(mlp.N_IN), np.ones(mlp.N_IN)
    loss, g = mlp.loss_and_grad(theta, inputs, targets, mean, std, quantize=False)
    idx = np.concatenate([rng.choice(np.flatnonzero(g != 0), 40, replace=False), [mlp.N_PARAMS - 5]])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        lp, _ = mlp.loss_and_grad(tp, inputs, targets, mean, std, quantize=False)
        lm, _ = mlp.loss_and_grad(tm, inputs, targets, mean, std, quantize=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_padding_gets_no_gradient():
    rng = np.random.default_rng(2)
    theta = mlp.init_params(4).astype(np.float64)
    _, g = mlp.loss_and_grad(theta, rng.standard_normal((5, mlp.N_IN)),
                             rng.standard_normal((5, mlp.N_OUT)), np.zeros(mlp.N_IN),
                             np.ones(mlp.N_IN))
    p = mlp.unpack(g)
    assert np.all(p["W1"][:, mlp.N_IN:] == 0) and np.all(p["W3"][mlp.N_OUT:] == 0)
    assert np.all(p["b3"][mlp.N_OUT:] == 0)


def test_adam_first_step_closed_form():
    """At t = 1 the bias-corrected moments are g and g^2, so the step is
    -lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    th, m, v = mlp.adam_step(np.zeros(4), np.zeros(4), np.zeros(4), g, 1, lr=0.01)
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
