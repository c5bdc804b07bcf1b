"""Pins of the oracle's surrogate network (FP64): GELU closed forms, the
backward pass against central differences, Adam's closed-form steps, the
bfloat16 rounding rule, and that training fits a known function."""
import math

import numpy as np
import pytest

from oracle import mlp
from workloads import mlp_layer_sizes, mlp_init, minibatch_indices


def test_gelu_closed_forms():
    # GELU(z) = z Phi(z); Phi(1) = 0.8413447460685429, Phi(2) = 0.9772498680518208
    z = np.array([0.0, 1.0, -1.0, 2.0])
    np.testing.assert_allclose(mlp.gelu(z), [0.0, 0.8413447460685429, -0.15865525393145707,
                                             2 * 0.9772498680518208], rtol=1e-15, atol=1e-16)
    # derivative against central differences
    zz = np.linspace(-4, 4, 33)
    h = 1e-5
    fd = (mlp.gelu(zz + h) - mlp.gelu(zz - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_prime(zz), fd, rtol=0, atol=1e-9)


@pytest.mark.parametrize("bf16", [False, True])
def test_backward_matches_central_differences(bf16):
    # a small network (the rounding points of the bf16 mode only perturb the
    # function; the derivative check uses the FP64 pipeline for bf16=False and
    # checks the bf16 pipeline's gradient is the FP64 one to bfloat16 accuracy)
    sizes = mlp_layer_sizes(5, 7, 3, 2)
    p = mlp_init(sizes, seed=3).astype(np.float64)
    rng = np.random.default_rng(0)
    x = rng.standard_normal((11, 5))
    t = rng.standard_normal((11, 2))
    loss, g = mlp.loss_grad(p, sizes, x, t, bf16=bf16)
    if not bf16:
        h = 1e-6
        fd = np.empty_like(p)
        for k in range(p.size):
            e = np.zeros_like(p)
            e[k] = h
            fd[k] = (mlp.loss_grad(p + e, sizes, x, t)[0] - mlp.loss_grad(p - e, sizes, x, t)[0]) / (2 * h)
        np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-9)
    else:
        _, g64 = mlp.loss_grad(p, sizes, x, t)
        assert np.linalg.norm(g - g64) / np.linalg.norm(g64) < 2e-2


def test_loss_is_mean_square():
    sizes = mlp_layer_sizes(3, 4, 1, 2)
    p = np.zeros(mlp.num_params(sizes))
    x = np.ones((5, 3))
    t = np.arange(10.0).reshape(5, 2)
    loss, g = mlp.loss_grad(p, sizes, x, t)
    assert loss == pytest.approx((t ** 2).mean(), rel=1e-15)
    # zero weights: y = 0, and of the last layer only the bias sees a gradient,
    # (2 / (5 rows x 2 outputs)) sum_rows (0 - t) = -(mean over rows of t) / 2 x 2
    np.testing.assert_allclose(g[-2:], -t.mean(axis=0), rtol=1e-15)
    assert np.abs(g[:-2]).max() == 0


def test_adam_closed_form_steps():
    # with a constant gradient g every bias-corrected step is lr g/(|g| + eps)
    g = np.array([0.3, -2.0, 1e-3])
    opt = mlp.Adam(3, lr=0.01)
    p = np.zeros(3)
    for k in range(1, 4):
        p = opt.step(p, g)
        np.testing.assert_allclose(p, -k * 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_bf16_rounding_rule():
    # bfloat16 keeps 8 significant bits: 1 + 2^-8 is a tie and rounds to even
    # (1.0); 1 + 3 2^-8 is a tie and rounds up to 1 + 2^-6; 1 + 2^-7 is exact
    v = np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -7, -3.0, 1.0 + 2.0 ** -8 + 2.0 ** -12])
    np.testing.assert_array_equal(mlp.round_bf16(v), [1.0, 1.0 + 2.0 ** -6, 1.0 + 2.0 ** -7, -3.0,
                                                      1.0 + 2.0 ** -7])


def test_training_fits_a_smooth_function():
    sizes = mlp_layer_sizes(2, 16, 2, 1)
    p = mlp_init(sizes, seed=1).astype(np.float64)
    rng = np.random.default_rng(2)
    x = rng.uniform(-1, 1, (256, 2))
    t = (np.sin(2 * x[:, 0]) * x[:, 1])[:, None]
    idx = minibatch_indices(256, 64, 1500, seed=4)
    p1, losses = mlp.train(p, sizes, x, t, idx, 64, mlp.Adam(p.size, lr=3e-3))
    assert losses[:20].mean() > 20 * losses[-50:].mean()
    assert mlp.loss_grad(p1, sizes, x, t)[0] < 2e-3


def test_minibatches_cover_the_data():
    idx = minibatch_indices(100, 32, 10, seed=0)
    assert idx.dtype == np.int32 and idx.size == 320
    # each consecutive 100 indices (one permutation) hit every row once
    assert sorted(idx[:100].tolist()) == list(range(100))
