"""FP64 numpy reference of the warm-start network.  TEST INFRASTRUCTURE ONLY.

The network maps three input planes of a channel (wall mask, electric force
f, interaction strength G) to three output planes (density and the two
velocity components, normalised) on an H x W lattice:

    level 1 (H, W)       conv3x3 cin->c1, ReLU, conv3x3 c1->c1, ReLU    -> e1
    level 2 (H/2, W/2)   avgpool(e1), conv c1->c2, ReLU, conv c2->c2, ReLU -> e2
    level 3 (H/4, W/4)   avgpool(e2), conv c2->c3 ... -> e3
    bottom  (H/8, W/8)   avgpool(e3), conv c3->c4, ReLU, conv c4->c4, ReLU -> b
    decoder              upsample(b) ++ e3 -> conv (c4+c3)->c3, ReLU, conv c3->c3, ReLU -> d3
                         upsample(d3) ++ e2 -> conv (c3+c2)->c2 ... -> d2
                         upsample(d2) ++ e1 -> conv (c2+c1)->c1 ... -> d1
    output               conv1x1 c1->cout (linear)

conv3x3 is periodic along x (the channel is periodic) and zero-padded along y;
avgpool is 2x2 averaging, upsample repeats each value 2x2, "++" concatenates
channels (the upsampled tensor first).  Loss: mean over fluid nodes and
output channels of (y - t)^2.  Parameters are one flat vector: for every layer
in the order above, W[cout][cin][kh][kw] then b[cout].

A 3x3 convolution is written as its definition, a sum over the nine taps
(ky, kx) of channel contractions of the shifted input, each contraction a
numpy einsum; every other layer is a numpy expression of its formula.  FP64
throughout.  The gradients are checked against finite differences and a
brute-force convolution in tests/test_cnn_oracle.py.

Stored activations in bf16 (the production setting: FP32 weights, bf16
activations) are defined as the same network with every stored activation
(each conv + ReLU output and each pooled tensor; upsampling and concatenation
only move stored values) rounded to the nearest bf16 value, ties to even, and
the gradient passed through the rounding unchanged: ``act=round_bf16``.

Error model of a bf16 build (``mca_gradient``): Monte Carlo arithmetic
(D. S. Parker, "Monte Carlo Arithmetic", 1997).  Every tensor such a build may
hold in 16 bits -- the weights, every stored activation and every layer
gradient that enters a contraction -- is multiplied elementwise by 1 + d with
d independent and uniform on [-u, u], u = 2^-8 (the unit roundoff of an 8-bit
significand), and the network is evaluated in FP64.  The spread of a few such
samples around the FP64 network estimates the size of the error that bf16
storage causes, without reference to where a particular implementation rounds.
The model is wider than round-to-nearest: its relative variance u^2/3 is about
1.8 times that of rounding values whose significands are spread uniformly in
log scale.
"""
from __future__ import annotations

import numpy as np


def layer_specs(cin=3, cout=3, chans=(32, 64, 128, 128)):
    """[(name, cin, cout, k)] in parameter order."""
    c1, c2, c3, c4 = chans
    return [("e1a", cin, c1, 3), ("e1b", c1, c1, 3),
            ("e2a", c1, c2, 3), ("e2b", c2, c2, 3),
            ("e3a", c2, c3, 3), ("e3b", c3, c3, 3),
            ("b_a", c3, c4, 3), ("b_b", c4, c4, 3),
            ("d3a", c4 + c3, c3, 3), ("d3b", c3, c3, 3),
            ("d2a", c3 + c2, c2, 3), ("d2b", c2, c2, 3),
            ("d1a", c2 + c1, c1, 3), ("d1b", c1, c1, 3),
            ("out", c1, cout, 1)]


def param_count(specs) -> int:
    return sum(co * ci * k * k + co for _, ci, co, k in specs)


def unpack(theta, specs):
    out, o = {}, 0
    for name, ci, co, k in specs:
        n = co * ci * k * k
        out[name] = (theta[o:o + n].reshape(co, ci, k, k), theta[o + n:o + n + co])
        o += n + co
    return out


def init_params(specs, seed=0):
    """He-normal weights, zero biases (FP64)."""
    rng = np.random.default_rng(seed)
    parts = []
    for _, ci, co, k in specs:
        parts.append(rng.standard_normal(co * ci * k * k) * np.sqrt(2.0 / (ci * k * k)))
        parts.append(np.zeros(co))
    return np.concatenate(parts)


def round_bf16(a):
    """Nearest value with 8 significant bits (bf16), ties to even; exponent range
    of the values met here is far inside bf16's."""
    m, e = np.frexp(np.asarray(a, np.float64))     # a = m 2^e, 1/2 <= |m| < 1
    return np.ldexp(np.round(np.ldexp(m, 8)), e - 8)


def _identity(a):
    return a


# ------------------------------------------------------------------ layers
def _pad(x):
    """One-node halo: periodic along x (columns), zero along y (rows)."""
    N, ci, H, Wd = x.shape
    xp = np.zeros((N, ci, H + 2, Wd + 2))
    xp[:, :, 1:-1, 1:-1] = x
    xp[:, :, 1:-1, 0] = x[:, :, :, -1]
    xp[:, :, 1:-1, -1] = x[:, :, :, 0]
    return xp


def conv(x, W, b):
    """x [N][ci][H][W] -> [N][co][H][W]; 3x3 periodic in x, zero in y, or 1x1:
    y[n,o,i,j] = b[o] + sum over c, ky, kx of W[o,c,ky,kx] x[n,c,i+ky-1,j+kx-1]."""
    N, ci, H, Wd = x.shape
    co, _, k, _ = W.shape
    y = np.empty((N, co, H, Wd))
    y[:] = b[None, :, None, None]
    if k == 1:
        y += np.einsum("oc,nchw->nohw", W[:, :, 0, 0], x, optimize=True)
        return y
    xp = _pad(x)
    for ky in range(3):
        for kx in range(3):
            y += np.einsum("oc,nchw->nohw", W[:, :, ky, kx], xp[:, :, ky:ky + H, kx:kx + Wd], optimize=True)
    return y


def conv_backward(x, W, dy):
    """Gradients (dx, dW, db) of conv for the upstream gradient dy:
    db[o] = sum dy[n,o,i,j]; dW[o,c,ky,kx] = sum dy[n,o,i,j] x[n,c,i+ky-1,j+kx-1];
    dx is the adjoint of the tap sum (scattered back through the halo)."""
    N, ci, H, Wd = x.shape
    co, _, k, _ = W.shape
    db = dy.sum(axis=(0, 2, 3))
    if k == 1:
        dW = np.einsum("nohw,nchw->oc", dy, x, optimize=True)[:, :, None, None]
        dx = np.einsum("oc,nohw->nchw", W[:, :, 0, 0], dy, optimize=True)
        return dx, dW, db
    xp = _pad(x)
    dW = np.empty_like(W)
    dxp = np.zeros_like(xp)
    for ky in range(3):
        for kx in range(3):
            dW[:, :, ky, kx] = np.einsum("nohw,nchw->oc", dy, xp[:, :, ky:ky + H, kx:kx + Wd], optimize=True)
            dxp[:, :, ky:ky + H, kx:kx + Wd] += np.einsum("oc,nohw->nchw", W[:, :, ky, kx], dy, optimize=True)
    dx = dxp[:, :, 1:-1, 1:-1].copy()
    dx[:, :, :, -1] += dxp[:, :, 1:-1, 0]      # the left pad was column W-1
    dx[:, :, :, 0] += dxp[:, :, 1:-1, -1]      # the right pad was column 0
    return dx, dW, db


def relu(z):
    return np.maximum(z, 0.0)


def pool(x):
    N, C, H, W = x.shape
    return x.reshape(N, C, H // 2, 2, W // 2, 2).mean(axis=(3, 5))


def pool_backward(dy):
    return np.repeat(np.repeat(dy, 2, axis=2), 2, axis=3) / 4.0


def up(x):
    return np.repeat(np.repeat(x, 2, axis=2), 2, axis=3)


def up_backward(dy):
    N, C, H, W = dy.shape
    return dy.reshape(N, C, H // 2, 2, W // 2, 2).sum(axis=(3, 5))


# ----------------------------------------------------------------- network
def forward(theta, specs, x, keep=False, act=_identity):
    """Network output; ``act`` is applied to every stored activation (identity:
    FP64 throughout; ``round_bf16``: bf16 activations)."""
    P = unpack(theta, specs)
    cache = {}

    def block(name_a, name_b, inp):
        za = conv(inp, *P[name_a]); ya = act(relu(za))
        zb = conv(ya, *P[name_b]); yb = act(relu(zb))
        cache[name_a] = (inp, za); cache[name_b] = (ya, zb)
        return yb

    e1 = block("e1a", "e1b", x)
    e2 = block("e2a", "e2b", act(pool(e1)))
    e3 = block("e3a", "e3b", act(pool(e2)))
    bt = block("b_a", "b_b", act(pool(e3)))
    d3 = block("d3a", "d3b", np.concatenate([up(bt), e3], 1))
    d2 = block("d2a", "d2b", np.concatenate([up(d3), e2], 1))
    d1 = block("d1a", "d1b", np.concatenate([up(d2), e1], 1))
    y = conv(d1, *P["out"])
    cache["out"] = (d1, None)
    cache["acts"] = (e1, e2, e3, bt, d3, d2, d1)
    return (y, cache) if keep else y


def loss(y, t, fluid):
    """Mean over fluid nodes and channels of (y - t)^2; fluid [N][H][W] bool."""
    m = fluid[:, None, :, :].astype(np.float64)
    cnt = m.sum() * y.shape[1]
    return float(((y - t) ** 2 * m).sum() / cnt)


def loss_grad(y, t, fluid):
    m = fluid[:, None, :, :].astype(np.float64)
    cnt = m.sum() * y.shape[1]
    return 2.0 * (y - t) * m / cnt


def backward(theta, specs, x, t, fluid, act=_identity, gact=_identity, with_output=False):
    """(loss, gradient of the loss with respect to theta), and the network
    output as a third item with ``with_output``.  The gradient passes ``act``
    unchanged; ``gact`` is applied to the layer gradient (dL/dz of a layer,
    after the ReLU mask) that enters each layer's weight-, bias- and
    input-gradient contractions (identity: FP64 throughout)."""
    y, cache = forward(theta, specs, x, keep=True, act=act)
    P = unpack(theta, specs)
    grads = {}
    dy = gact(loss_grad(y, t, fluid))
    d1_in, _ = cache["out"]
    dd1, dW, db = conv_backward(d1_in, P["out"][0], dy)
    grads["out"] = (dW, db)

    def block_back(name_a, name_b, dout):
        ya, zb = cache[name_b]
        dzb = gact(dout * (zb > 0))
        dya, dW, db = conv_backward(ya, P[name_b][0], dzb)
        grads[name_b] = (dW, db)
        inp, za = cache[name_a]
        dza = gact(dya * (za > 0))
        dinp, dW, db = conv_backward(inp, P[name_a][0], dza)
        grads[name_a] = (dW, db)
        return dinp

    e1, e2, e3, bt, d3, d2, d1 = cache["acts"]
    c1, c2, c3 = e1.shape[1], e2.shape[1], e3.shape[1]
    dcat = block_back("d1a", "d1b", dd1)
    dd2, de1 = up_backward(dcat[:, :-c1]), dcat[:, -c1:]
    dcat = block_back("d2a", "d2b", dd2)
    dd3, de2 = up_backward(dcat[:, :-c2]), dcat[:, -c2:]
    dcat = block_back("d3a", "d3b", dd3)
    dbt, de3 = up_backward(dcat[:, :-c3]), dcat[:, -c3:]
    dp3 = block_back("b_a", "b_b", dbt)
    de3 = de3 + pool_backward(dp3)
    dp2 = block_back("e3a", "e3b", de3)
    de2 = de2 + pool_backward(dp2)
    dp1 = block_back("e2a", "e2b", de2)
    de1 = de1 + pool_backward(dp1)
    block_back("e1a", "e1b", de1)
    flat = []
    for name, *_ in specs:
        flat.append(grads[name][0].ravel())
        flat.append(grads[name][1].ravel())
    if with_output:
        return loss(y, t, fluid), np.concatenate(flat), y
    return loss(y, t, fluid), np.concatenate(flat)


def weight_mask(specs):
    """Boolean mask over theta: True on weights, False on biases."""
    parts = []
    for _, ci, co, k in specs:
        parts.append(np.ones(co * ci * k * k, bool))
        parts.append(np.zeros(co, bool))
    return np.concatenate(parts)


def mca_gradient(theta, specs, x, t, fluid, rng, u=2.0 ** -8):
    """One Monte Carlo arithmetic sample of a bf16 build (module docstring):
    returns (output, loss, gradient) of the FP64 network whose weights, stored
    activations and layer gradients each carry an independent relative error
    uniform on [-u, u].  u = 0 gives the FP64 network exactly."""
    def perturb(a):
        a = np.asarray(a, np.float64)
        return a * (1.0 + rng.uniform(-u, u, a.shape))

    th = theta.copy()
    w = weight_mask(specs)
    th[w] = perturb(theta[w])
    L, g, y = backward(th, specs, x, t, fluid, act=perturb, gact=perturb, with_output=True)
    return y, L, g


def adam(theta, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, with bias correction); returns new arrays."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
