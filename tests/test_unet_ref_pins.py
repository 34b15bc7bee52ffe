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


def test_down_is_a_strided_correlation():
    # a 2x2 stride-2 convolution is the full ("valid") correlation sampled at even
    # offsets: pinned per input/output channel pair against scipy's correlation
    rng = np.random.default_rng(4)
    C, Co = 3, 2
    X = rng.standard_normal((2, 10, 6, C))
    W = rng.standard_normal((4 * C, Co))
    b = rng.standard_normal(Co)
    y = U.down(X, W, b)
    assert y.shape == (2, 5, 3, Co)
    Wk = W.reshape(2, 2, C, Co)
    for bi in range(2):
        for o in range(Co):
            ref = np.full((5, 3), b[o])
            for c in range(C):
                full = scipy.signal.correlate2d(X[bi, :, :, c], Wk[:, :, c, o], mode="valid")
                ref += full[::2, ::2]
            np.testing.assert_allclose(y[bi, :, :, o], ref, rtol=1e-13, atol=1e-13)


def test_up_is_the_adjoint_of_down():
    # the 2x2 stride-2 transposed convolution is the adjoint of the strided
    # convolution with the transposed weight matrix: <down(Y; W), X> = <Y, up(X; W^T)>
    rng = np.random.default_rng(5)
    Cb, Cs = 4, 3
    Y = rng.standard_normal((2, 8, 6, Cb))
    X = rng.standard_normal((2, 4, 3, Cs))
    Wd = rng.standard_normal((4 * Cb, Cs))
    lhs = float(np.sum(U.down(Y, Wd, np.zeros(Cs)) * X))
    up = U.up_place(U.up_prod(X, Wd.T, Cb), np.zeros(Cb))
    assert up.shape == Y.shape
    rhs = float(np.sum(Y * up))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_up_places_each_input_pixel_on_its_own_2x2_block():
    # a one-hot input pixel spreads to exactly the 2x2 output block under it,
    # the four positions taking the four weight slices (dy, dx) in row-major order
    Cs, Cb = 2, 3
    W = np.arange(Cs * 4 * Cb, dtype=float).reshape(Cs, 4 * Cb)
    X = np.zeros((1, 3, 4, Cs))
    X[0, 1, 2, 1] = 1.0
    out = U.up_place(U.up_prod(X, W, Cb), np.zeros(Cb))
    nz = np.argwhere(np.abs(out).sum(-1) > 0)
    assert sorted(map(tuple, nz[:, 1:])) == [(2, 4), (2, 5), (3, 4), (3, 5)]
    for dy in range(2):
        for dx in range(2):
            np.testing.assert_array_equal(out[0, 2 + dy, 4 + dx], W[1, (dy * 2 + dx) * Cb:(dy * 2 + dx + 1) * Cb])


def test_adam_bias_correction_closed_forms():
    # step 1 from zero moments: m_hat = g, v_hat = g^2, so the step is
    # -lr g / (|g| + eps) (Kingma and Ba, Sec. 2 and 3)
    rng = np.random.default_rng(6)
    th = rng.standard_normal(50)
    g = rng.standard_normal(50)
    lr = 1e-3
    t1, m, v = U.adam_step(th, g, np.zeros(50), np.zeros(50), 1, lr)
    np.testing.assert_allclose(t1, th - lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-13)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-13)
    # a constant gradient keeps the bias-corrected moments exact at every step
    th_k, m, v = th, np.zeros(50), np.zeros(50)
    for k in range(1, 40):
        prev = th_k
        th_k, m, v = U.adam_step(th_k, g, m, v, k, lr)
        np.testing.assert_allclose(prev - th_k, lr * g / (np.abs(g) + 1e-8), rtol=1e-11, atol=0)
    # sign flips: the first moment decays by beta1 while the second keeps g^2
    t2, _, _ = U.adam_step(t1, -g, 0.1 * g, 0.001 * g * g, 2, lr)
    mh = (0.9 * 0.1 * g - 0.1 * g) / (1 - 0.81)
    vh = (0.999 * 0.001 + 0.001) * g * g / (1 - 0.999 ** 2)
    np.testing.assert_allclose(t2, t1 - lr * mh / (np.sqrt(vh) + 1e-8), rtol=1e-13, atol=1e-16)
