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


def test_round_bf16_fixed_values():
    """8 significant bits, ties to even, sign symmetric."""
    r = cnn.round_bf16
    assert r(1.0) == 1.0 and r(0.0) == 0.0
    assert r(1 + 2.0 ** -8) == 1.0                      # tie -> even (1.0)
    assert r(1 + 3 * 2.0 ** -8) == 1 + 2.0 ** -6        # tie -> even (1 + 4 * 2^-8)
    assert r(1 + 2.0 ** -8 + 2.0 ** -20) == 1 + 2.0 ** -7
    assert r(-(1 + 3 * 2.0 ** -8)) == -(1 + 2.0 ** -6)
    assert r(3.0) == 3.0 and r(255.0) == 255.0 and r(257.0) == 256.0 and r(259.0) == 260.0
    assert r(2.0 ** -100 * 1.00390625) == 2.0 ** -100     # scale invariance


def test_round_bf16_matches_library_conversion():
    """Against torch's float32 -> bfloat16 conversion (round to nearest even) on
    values exactly representable in float32."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(9)
    a = (rng.standard_normal(20000) * np.exp(rng.uniform(-20, 20, 20000))).astype(np.float32)
    lib = torch.from_numpy(a).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(cnn.round_bf16(a.astype(np.float64)), lib)


def test_rounded_network_is_close_and_identity_is_default():
    specs = cnn.layer_specs(chans=(3, 4, 4, 5))
    theta = cnn.init_params(specs, seed=4)
    x = np.random.default_rng(5).standard_normal((1, 3, 8, 16))
    y = cnn.forward(theta, specs, x)
    assert np.array_equal(y, cnn.forward(theta, specs, x, act=lambda a: a))
    yb = cnn.forward(theta, specs, x, act=cnn.round_bf16)
    err = np.linalg.norm(yb - y) / np.linalg.norm(y)
    assert 1e-5 < err < 5e-2          # rounding is applied, and it is a small perturbation


def test_weight_rounding_applies_to_the_inner_3x3_layers_only():
    """wround rounds exactly the forward 3x3 convolutions after the first:
    the same as pre-rounding those weights by hand."""
    specs = cnn.layer_specs(chans=(3, 4, 4, 5))
    theta = cnn.init_params(specs, seed=6)
    x = np.random.default_rng(7).standard_normal((1, 3, 8, 16))
    y0 = cnn.forward(theta, specs, x)
    assert np.array_equal(y0, cnn.forward(theta, specs, x, wround=lambda w: w))
    manual, o = theta.copy(), 0
    for i, (name, ci, co, k) in enumerate(specs):
        n = co * ci * k * k
        if i > 0 and k == 3:
            manual[o:o + n] = cnn.round_bf16(theta[o:o + n])
        o += n + co
    y1 = cnn.forward(theta, specs, x, wround=cnn.round_bf16)
    np.testing.assert_array_equal(y1, cnn.forward(manual, specs, x))
    assert not np.array_equal(y1, y0)
    # the backward pass differentiates with the unrounded weights
    t = np.zeros_like(y0)
    fluid = np.ones((1, 8, 16), bool)
    _, g1 = cnn.backward(theta, specs, x, t, fluid, wround=cnn.round_bf16)
    _, g2 = cnn.backward(manual, specs, x, t, fluid)
    rel = np.linalg.norm(g1 - g2) / np.linalg.norm(g2)
    assert 0 < rel < 2e-2          # differs only through the 2^-9 weight rounding in dx


def test_backward_rounding_hook():
    """ground rounds the layer gradient in the 3x3 layers' weight- and
    input-gradient contractions and the weights in the input gradient:
    identity leaves the gradient unchanged; rounding keeps the output layer's
    gradients and every bias gradient of the last 3x3 layer (their inputs are
    not rounded), and moves the other gradients by about the bf16 rounding;
    the last 3x3 layer's weight gradient equals the one formed by hand from
    the rounded layer gradient."""
    specs = cnn.layer_specs(chans=(3, 4, 4, 5))
    theta = cnn.init_params(specs, seed=8)
    rng = np.random.default_rng(9)
    x = rng.standard_normal((2, 3, 8, 16))
    t = rng.standard_normal((2, 3, 8, 16))
    fluid = rng.random((2, 8, 16)) > 0.2
    _, g0 = cnn.backward(theta, specs, x, t, fluid)
    _, gi = cnn.backward(theta, specs, x, t, fluid, ground=lambda a: a)
    assert np.array_equal(g0, gi)
    _, g1 = cnn.backward(theta, specs, x, t, fluid, ground=cnn.round_bf16)
    o = 0
    for name, ci, co, k in specs:
        nw = co * ci * k * k
        aw, bw = g0[o:o + nw], g1[o:o + nw]
        ab, bb = g0[o + nw:o + nw + co], g1[o + nw:o + nw + co]
        if name == "out":
            assert np.array_equal(aw, bw) and np.array_equal(ab, bb)
        else:
            rel = np.linalg.norm(aw - bw) / np.linalg.norm(aw)
            assert 0 < rel < 2e-2, (name, rel)
        if name == "d1b":
            assert np.array_equal(ab, bb)
        o += nw + co
    # d1b by hand: its layer gradient is (dL/d output of d1b) * relu'(z)
    y, cache = cnn.forward(theta, specs, x, keep=True)
    P = cnn.unpack(theta, specs)
    dd1, _, _ = cnn.conv_backward(cache["out"][0], P["out"][0], cnn.loss_grad(y, t, fluid))
    ya, zb = cache["d1b"]
    _, dW, _ = cnn.conv_backward(ya, P["d1b"][0], cnn.round_bf16(dd1 * (zb > 0)))
    names = [nm for nm, *_ in specs]
    o = sum(co_ * ci_ * k_ * k_ + co_ for _, ci_, co_, k_ in specs[:names.index("d1b")])
    np.testing.assert_allclose(g1[o:o + dW.size], dW.ravel(), rtol=0, atol=1e-15)
