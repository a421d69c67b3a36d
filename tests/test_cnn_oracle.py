"""Pins of the FP64 reference network (CPU only): layer adjoint identities, a
brute-force convolution, and finite differences of the whole-network gradient."""
import numpy as np
import pytest

from oracle import cnn


def test_conv3x3_bruteforce_periodic_x_zero_y():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 5, 7))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = cnn.conv(x, W, b)
    N, C, H, Wd = x.shape
    for n in range(N):
        for o in range(4):
            for i in range(H):
                for j in range(Wd):
                    s = b[o]
                    for c in range(C):
                        for ky in range(3):
                            for kx in range(3):
                                yy, xx = i + ky - 1, (j + kx - 1) % Wd
                                if 0 <= yy < H:
                                    s += W[o, c, ky, kx] * x[n, c, yy, xx]
                    assert abs(y[n, o, i, j] - s) < 1e-12


@pytest.mark.parametrize("k", [1, 3])
def test_conv_backward_is_adjoint(k):
    rng = np.random.default_rng(k)
    x = rng.standard_normal((2, 3, 6, 8))
    W = rng.standard_normal((5, 3, k, k))
    b = np.zeros(5)
    dy = rng.standard_normal((2, 5, 6, 8))
    dx, dW, db = cnn.conv_backward(x, W, dy)
    # <conv(x), dy> = <x, dx> (linear in x); and = <W, dW> (linear in W)
    lhs = (cnn.conv(x, W, b) * dy).sum()
    assert abs(lhs - (x * dx).sum()) < 1e-10 * abs(lhs)
    assert abs(lhs - (W * dW).sum()) < 1e-10 * abs(lhs)
    assert np.allclose(db, dy.sum(axis=(0, 2, 3)))


def test_pool_and_upsample_adjoints():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 3, 8, 12))
    y = rng.standard_normal((2, 3, 4, 6))
    assert abs((cnn.pool(x) * y).sum() - (x * cnn.pool_backward(y)).sum()) < 1e-12
    assert abs((cnn.up(y) * x).sum() - (y * cnn.up_backward(x)).sum()) < 1e-12
    np.testing.assert_allclose(cnn.pool(cnn.up(y)), y)


def test_whole_network_gradient_finite_differences():
    specs = cnn.layer_specs(chans=(3, 4, 4, 5))
    theta = cnn.init_params(specs, seed=1)
    rng = np.random.default_rng(2)
    N, H, W = 2, 8, 16
    x = rng.standard_normal((N, 3, H, W))
    t = rng.standard_normal((N, 3, H, W))
    fluid = rng.random((N, H, W)) > 0.2
    L, g = cnn.backward(theta, specs, x, t, fluid)
    assert abs(L - cnn.loss(cnn.forward(theta, specs, x), t, fluid)) < 1e-14
    idx = rng.choice(theta.size, 60, replace=False)
    eps = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd = (cnn.loss(cnn.forward(tp, specs, x), t, fluid) -
              cnn.loss(cnn.forward(tm, specs, x), t, fluid)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(fd)), (i, fd, g[i])


def test_adam_first_step_is_sign_step():
    """With bias correction the first Adam step is lr * g / (|g| + eps)."""
    rng = np.random.default_rng(4)
    th = rng.standard_normal(10)
    g = rng.standard_normal(10)
    new, m, v = cnn.adam(th, g, np.zeros(10), np.zeros(10), 1, lr=0.01)
    np.testing.assert_allclose(th - new, 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
