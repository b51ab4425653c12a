"""Pins of the warm-start network oracle (float64): finite differences of the
loss, convolution against direct summation, up-sampling adjoint identity,
Adam against its closed form on a quadratic."""
import numpy as np
import pytest

from oracle import cnn


def test_conv_matches_direct_sum():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 7, 6))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    for s in (1, 2):
        out = cnn.conv(x, W, b, s)
        ref = np.zeros_like(out)
        for bb in range(2):
            for o in range(4):
                for yy in range(out.shape[2]):
                    for xx in range(out.shape[3]):
                        acc = b[o]
                        for c in range(3):
                            for ky in range(3):
                                for kx in range(3):
                                    iy, ix = s * yy + ky - 1, s * xx + kx - 1
                                    if 0 <= iy < 7 and 0 <= ix < 6:
                                        acc += W[o, c, ky, kx] * x[bb, c, iy, ix]
                        ref[bb, o, yy, xx] = acc
        assert np.allclose(out, ref, atol=1e-12)


def test_conv_and_upsample_adjoints():
    """<conv(x), d> - b-part = <x, conv^T(d)> and <up2(a), d> = <a, up2^T(d)>."""
    rng = np.random.default_rng(1)
    for s in (1, 2):
        x = rng.standard_normal((2, 3, 9, 8))
        W = rng.standard_normal((5, 3, 3, 3))
        y = cnn.conv(x, W, np.zeros(5), s)
        d = rng.standard_normal(y.shape)
        dx, dW, db = cnn.conv_backward(x, W, d, s)
        assert np.sum(y * d) == pytest.approx(np.sum(x * dx), rel=1e-12)
        assert np.sum(y * d) == pytest.approx(np.sum(W * dW), rel=1e-12)
    a = rng.standard_normal((1, 2, 5, 4))
    u = cnn.up2(a, 9, 8)
    d = rng.standard_normal(u.shape)
    assert np.sum(u * d) == pytest.approx(np.sum(a * cnn.up2_backward(d, 5, 4)), rel=1e-12)


def test_gradient_by_finite_differences():
    rng = np.random.default_rng(2)
    nf, H, W = 2, 9, 10
    p = cnn.init_params(nf, seed=3) * 0.5
    p += 0.05 * rng.standard_normal(p.size)           # nonzero biases
    x = rng.standard_normal((2, 6 * nf, H, W))
    t = rng.standard_normal((2, nf, H, W))
    loss, g = cnn.loss_and_grad(p, x, t, nf)
    idx = rng.choice(p.size, 40, replace=False)
    eps = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = eps
        num = (cnn.loss_and_grad(p + e, x, t, nf)[0] - cnn.loss_and_grad(p - e, x, t, nf)[0]) / (2 * eps)
        assert num == pytest.approx(g[i], rel=1e-5, abs=1e-9)


def test_adam_first_step_is_signed_lr():
    """On the first step Adam moves each parameter by lr * g / (|g| + eps)."""
    p = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 1e-3])
    p1, m, v = cnn.adam(p, g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8))


def test_features_layout():
    f = np.zeros((2, 5, 6))
    f[0, 2, 3] = -4.0
    f[1, 1, 1] = 2.0
    ft = cnn.features(f, np.array([3.0, 7.0]))
    assert ft.shape == (12, 5, 6)
    assert ft[0, 2, 3] == -1.0 and ft[1, 1, 1] == 1.0
    assert np.allclose(ft[2, :, 0], 0.0) and np.allclose(ft[4, :, 0], 1.0)
    assert np.allclose(ft[11], 7.0 / 50)
