"""Pins of the reference U-Net (test infrastructure) against independent facts."""
import numpy as np
import pytest
import scipy.signal

from oracle import unet_ref as U


def test_bf16_rounding():
    # exactly representable values stay, ties go to even, 8-bit mantissa spacing
    assert U.to_bf16(1.0) == 1.0
    assert U.to_bf16(1.0 + 2 ** -8) == 1.0            # tie -> even (mantissa 0)
    assert U.to_bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6  # tie -> even (mantissa 2)
    assert U.to_bf16(1.0 + 2 ** -7) == 1.0 + 2 ** -7
    x = np.random.default_rng(0).standard_normal(1000)
    assert np.max(np.abs(U.to_bf16(x) - x) / np.abs(x)) <= 2 ** -8   # half a unit in the 7-bit mantissa


def test_conv3_matches_library_correlation():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((1, 9, 7, 1))
    Wt = rng.standard_normal((9, 1))
    y = U.conv3(X, Wt, np.zeros(1))
    ref = scipy.signal.correlate2d(X[0, :, :, 0], Wt.reshape(3, 3), mode="same", boundary="fill")
    np.testing.assert_allclose(y[0, :, :, 0], ref, rtol=1e-13, atol=1e-13)


def test_parameter_count():
    # 4 levels (16,32,64,128), ~0.6M parameters
    assert U.param_count() == 621776 + 1045   # weights + biases


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(2)
    theta = U.init_params(3) + 0.01 * rng.standard_normal(U.param_count())
    x = rng.standard_normal((1, 16, 16, 8))
    t = rng.standard_normal((1, 16, 16, 5))
    loss, g, _ = U.loss_and_grad(theta, x, t)
    idx = rng.choice(theta.size, 12, replace=False)
    h = 1e-6
    for k in idx:
        e = np.zeros_like(theta)
        e[k] = h
        lp = U.loss_and_grad(theta + e, x, t)[0]
        lm = U.loss_and_grad(theta - e, x, t)[0]
        fd = (lp - lm) / (2 * h)
        assert fd == pytest.approx(g[k], rel=1e-4, abs=1e-9)
