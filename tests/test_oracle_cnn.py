"""Pins of the warm-start network oracle."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import cnn


def test_parameter_count():
    assert cnn.n_params() == 19105
    p = cnn.init_params(0)
    assert np.array_equal(cnn.flatten(cnn.unflatten(cnn.flatten(p))), cnn.flatten(p))


def test_conv_matches_library_correlation():
    rng = np.random.default_rng(0)
    a = rng.standard_normal((2, 7, 9, 3))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    out = cnn.conv3x3(a, W, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(correlate2d(a[n, :, :, c], W[o, c], mode="same") for c in range(3))
            assert np.max(np.abs(out[n, :, :, o] - ref)) <= 1e-12


def test_zero_last_layer_is_identity():
    p = cnn.init_params(1)
    p[3] = (np.zeros_like(p[3][0]), np.zeros_like(p[3][1]))
    x = np.random.default_rng(2).random((2, 8, 5))
    out, _ = cnn.forward(p, x)
    assert np.array_equal(out, x)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(3)
    p = cnn.init_params(4)
    p = [(W, rng.standard_normal(b.shape) * 0.1) for W, b in p]
    x = rng.random((1, 6, 7))
    target = rng.random((1, 6, 7))
    loss, grads, _ = cnn.loss_and_grads(p, x, target)
    flat = cnn.flatten(p)
    g = cnn.flatten(grads)
    idx = rng.choice(flat.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(flat)
        e[i] = h
        lp, _, _ = cnn.loss_and_grads(cnn.unflatten(flat + e), x, target)
        lm, _, _ = cnn.loss_and_grads(cnn.unflatten(flat - e), x, target)
        num = (lp - lm) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, num, g[i])


def test_bf16_rounding_is_nearest_even():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    v = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-20, 20, 5000),
                        [1 + 2 ** -8, 1 + 3 * 2 ** -8, -1 - 2 ** -8, 0.0, 1.0]]).astype(np.float32)
    ref = torch.tensor(v).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)
    assert np.array_equal(cnn.round_bf16(v), ref)
    assert cnn.round_bf16(np.float32(1 + 2 ** -8)) == 1.0
    assert cnn.round_bf16(np.float32(1 + 3 * 2 ** -8)) == 1 + 2 ** -6


def test_adam_first_step_is_signed_learning_rate():
    g = np.array([3.0, -0.5, 1e-3])
    p1, m, v = cnn.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0)
    assert np.allclose(p1, -0.01 * np.sign(g), rtol=0, atol=1e-15)


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the bias-corrected moments are exactly g
    and g^2 at every step, so each step moves by lr g / (|g| + eps): this
    pins both bias corrections and where eps enters (outside the root)."""
    g = np.array([2.0, -0.5, 1e-8, -3e-8, 0.0])
    lr, eps = 0.01, 1e-8
    w, m, v = np.zeros(5), np.zeros(5), np.zeros(5)
    for k in range(1, 6):
        w, m, v = cnn.adam_step(w, g, m, v, k, lr, eps=eps)
        ref = -k * lr * g / (np.abs(g) + eps)
        assert np.allclose(w, ref, rtol=1e-12, atol=1e-18), (k, w, ref)
