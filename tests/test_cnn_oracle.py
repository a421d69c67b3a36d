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


def test_layer_gradient_hook():
    """gact acts on the layer gradient that enters each layer's contractions:
    identity leaves the gradient unchanged; with rounding, the last 3x3 layer's
    weight and bias gradients equal those formed by hand from the rounded layer
    gradient, and every block moves by about the bf16 rounding."""
    specs = cnn.layer_specs(chans=(3, 4, 4, 5))
    theta = cnn.init_params(specs, seed=8)
    rng = np.random.default_rng(9)
    x = rng.standard_normal((2, 3, 8, 16))
    t = rng.standard_normal((2, 3, 8, 16))
    fluid = rng.random((2, 8, 16)) > 0.2
    _, g0 = cnn.backward(theta, specs, x, t, fluid)
    _, gi = cnn.backward(theta, specs, x, t, fluid, gact=lambda a: a)
    assert np.array_equal(g0, gi)
    _, g1 = cnn.backward(theta, specs, x, t, fluid, gact=cnn.round_bf16)
    o = 0
    for name, ci, co, k in specs:
        n = co * ci * k * k + co
        rel = np.linalg.norm(g0[o:o + n] - g1[o:o + n]) / np.linalg.norm(g0[o:o + n])
        assert 0 < rel < 5e-2, (name, rel)
        o += n
    # d1b by hand: its layer gradient is (dL/d output of d1b) * relu'(z), where
    # dL/d output comes from the output layer fed the rounded loss gradient
    y, cache = cnn.forward(theta, specs, x, keep=True)
    P = cnn.unpack(theta, specs)
    dd1, _, _ = cnn.conv_backward(cache["out"][0], P["out"][0], cnn.round_bf16(cnn.loss_grad(y, t, fluid)))
    ya, zb = cache["d1b"]
    _, dW, db = cnn.conv_backward(ya, P["d1b"][0], cnn.round_bf16(dd1 * (zb > 0)))
    names = [nm for nm, *_ in specs]
    o = sum(co_ * ci_ * k_ * k_ + co_ for _, ci_, co_, k_ in specs[:names.index("d1b")])
    np.testing.assert_array_equal(g1[o:o + dW.size], dW.ravel())
    np.testing.assert_array_equal(g1[o + dW.size:o + dW.size + db.size], db)


def test_mca_sample_is_the_network_at_u0_and_scales_with_u():
    """Monte Carlo arithmetic: u = 0 is the FP64 network exactly; the spread
    of the perturbed outputs is linear in u (first-order error propagation),
    so halving u halves their rms error.  The gradient is not continuous where
    a perturbation moves a pre-activation across zero (its ReLU branch flips),
    which happens at u = 2^-8 in a network this small, so for the gradient
    only the size of the spread is checked."""
    specs = cnn.layer_specs(chans=(3, 4, 4, 5))
    theta = cnn.init_params(specs, seed=10)
    rng = np.random.default_rng(11)
    x = rng.standard_normal((2, 3, 8, 16))
    t = rng.standard_normal((2, 3, 8, 16))
    fluid = rng.random((2, 8, 16)) > 0.2
    L0, g0, y0 = cnn.backward(theta, specs, x, t, fluid, with_output=True)
    y, L, g = cnn.mca_gradient(theta, specs, x, t, fluid, np.random.default_rng(0), u=0.0)
    assert np.array_equal(y, y0) and L == L0 and np.array_equal(g, g0)

    def rms(u, n=8):
        r = np.random.default_rng(1)
        ey, eg = [], []
        for _ in range(n):
            y, _, g = cnn.mca_gradient(theta, specs, x, t, fluid, r, u=u)
            ey.append(np.linalg.norm(y - y0) / np.linalg.norm(y0))
            eg.append(np.linalg.norm(g - g0) / np.linalg.norm(g0))
        return np.sqrt(np.mean(np.square(ey))), np.sqrt(np.mean(np.square(eg)))

    ya, ga = rms(2.0 ** -8)
    yb, gb = rms(2.0 ** -9)
    assert 1e-4 < ya < 5e-2 and 1e-4 < ga < 2e-1
    assert 1.6 < ya / yb < 2.5


def test_mca_perturbation_is_relative_and_uniform():
    """Each perturbed value is a (1 + d) with |d| <= u, d of mean 0 and
    variance u^2 / 3 (uniform on [-u, u]); weights are perturbed, biases not."""
    specs = cnn.layer_specs(chans=(3, 4, 4, 5))
    theta = cnn.init_params(specs, seed=12)
    b = ~cnn.weight_mask(specs)
    theta[b] = 0.1
    u = 2.0 ** -8
    seen = []

    def spy(th, sp, xx, tt, ff, act, gact, with_output):
        seen.append(th.copy())
        a = np.linspace(1.0, 2.0, 200001)
        d = act(a) / a - 1.0
        assert np.abs(d).max() <= u
        assert abs(d.mean()) < 4 * u / np.sqrt(3 * a.size)
        assert abs(d.var() / (u * u / 3) - 1) < 0.02
        return 0.0, np.zeros_like(th), np.zeros((1,))

    orig = cnn.backward
    try:
        cnn.backward = spy
        cnn.mca_gradient(theta, specs, None, None, None, np.random.default_rng(3), u=u)
    finally:
        cnn.backward = orig
    th = seen[0]
    w = cnn.weight_mask(specs)
    d = th[w] / theta[w] - 1.0
    assert np.abs(d).max() <= u and np.abs(d).max() > 0.5 * u
    assert np.array_equal(th[b], theta[b])
