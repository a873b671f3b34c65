"""Pins of the FP64 U-Net oracle (CPU only).

Each layer is checked against an independent definition (scipy's 2-D
cross-correlation, a Kronecker-product form of the transposed convolution,
reshape-max pooling, torch's bfloat16 conversion, the closed form of Adam
under a constant gradient) and the whole backward pass against central finite
differences of the FP64 loss, so a dropped term, a flipped kernel, a
transposed operand or a wrong skip/pool routing fails here."""
import math

import numpy as np
import pytest
import scipy.signal
import torch

import synth
from oracle import unet as U


def test_bf16_matches_torch_round_to_nearest_even():
    rng = np.random.default_rng(0)
    x = rng.normal(0, 10, 20000).astype(np.float32)
    # exact ties: 1 + 2^-8 (ties to 1), 1 + 3*2^-8 (ties up), and their negatives
    ties = np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 2 ** -130, 0.0], np.float32)
    x = np.concatenate([x, ties])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(U.bf16(x.astype(np.float64)), ref)
    assert U.bf16(np.array([1 + 2 ** -8]))[0] == 1.0
    assert U.bf16(np.array([1 + 3 * 2 ** -8]))[0] == 1 + 2 ** -6


@pytest.mark.parametrize("K", [1, 3])
def test_conv_forward_is_zero_padded_cross_correlation(K):
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 7, 9, 3))
    W = rng.normal(size=(4, K, K, 3))
    b = rng.normal(size=4)
    out = U.conv_fwd(x, W, b)
    ref = np.zeros_like(out)
    for n in range(2):
        for co in range(4):
            acc = b[co]
            for ci in range(3):
                acc = acc + scipy.signal.correlate2d(x[n, :, :, ci], W[co, :, :, ci], mode="same",
                                                     boundary="fill")
            ref[n, :, :, co] = acc
    assert np.allclose(out, ref, rtol=0, atol=1e-12)


def test_transposed_conv_is_kronecker_product():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 3, 5, 1))
    W = rng.normal(size=(2, 2, 1, 1))
    b = rng.normal(size=1)
    out = U.up_fwd(x, W, b)
    for n in range(2):
        assert np.allclose(out[n, :, :, 0], np.kron(x[n, :, :, 0], W[:, :, 0, 0]) + b[0], atol=1e-14)


def test_pool_is_block_max_and_routes_ties_to_first():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(2, 6, 8, 3))
    y, arg = U.pool_fwd(x)
    assert np.array_equal(y, x.reshape(2, 3, 2, 4, 2, 3).max(axis=(2, 4)))
    # a window of equal values: the gradient goes to (0,0); (0,1)=(1,1) tie -> (0,1)
    t = np.zeros((1, 2, 4, 1))
    t[0, 0, 2, 0], t[0, 0, 3, 0], t[0, 1, 2, 0], t[0, 1, 3, 0] = 1.0, 5.0, 2.0, 5.0
    _, arg = U.pool_fwd(t)
    g = U.pool_bwd(np.ones((1, 1, 2, 1)), arg, t.shape)
    assert g[0, 0, 0, 0] == 1 and g[0, :, :2, 0].sum() == 1
    assert g[0, 0, 3, 0] == 1 and g[0, 1, 3, 0] == 0


def test_adam_constant_gradient_closed_form():
    # with a constant gradient g the bias-corrected moments are g and g^2, so
    # each step moves w by lr * g / (|g| + eps)
    w0 = np.array([0.5, -1.0, 2.0])
    g = np.array([0.3, -2e-3, 5.0])
    w, m, v = w0.copy(), np.zeros(3), np.zeros(3)
    lr, eps, T = 1e-3, 1e-8, 25
    for t in range(1, T + 1):
        w, m, v = U.adam(w, g, m, v, t, lr, eps=eps)
    assert np.allclose(w, w0 - T * lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)


def test_layout_roundtrip_and_independent_count():
    for L, C0 in [(2, 8), (3, 16), (4, 32)]:
        cfg = U.Config(levels=L, base=C0)
        n = sum(a + c for a, _, c in synth.unet_segments(L, C0))
        assert U.num_params(cfg) == n
        p = np.arange(n, dtype=np.float64)
        d = U.unpack(cfg, p)
        assert np.array_equal(U.pack(cfg, {k: v for k, v in d.items()}), p)


@pytest.mark.parametrize("levels,H,W", [(2, 8, 8), (3, 8, 12)])
def test_backward_matches_finite_differences(levels, H, W):
    cfg = U.Config(levels=levels, base=8, cin=3, cout=3, H=H, W=W)
    params = synth.unet_params(levels, 8, seed=5).astype(np.float64)
    x, t = synth.unet_batch(2, H, W, 3, 3, seed=6)
    x, t = x.astype(np.float64), t.astype(np.float64)
    loss, g = U.loss_and_grads(cfg, params, x, t, rounding=False)
    y, _ = U.forward(cfg, params, x, rounding=False)
    assert loss == pytest.approx(np.mean((y - t) ** 2), rel=1e-14)
    rng = np.random.default_rng(7)
    # every layer: a few weights and a few biases
    idx, off = [], 0
    for name, _, ws, nb in U.layer_shapes(cfg):
        nw = int(np.prod(ws))
        if name == "head":  # only the first cout outputs carry loss
            idx += [off + co * 8 + ci for co in range(3) for ci in (0, 5)] + [off + nw, off + nw + 2]
        else:
            idx += list(off + rng.choice(nw, 4, replace=False)) + list(off + nw + rng.choice(nb, 2, replace=False))
        off += nw + nb
    h = 1e-6
    err = 0.0
    for i in idx:
        pp, pm = params.copy(), params.copy()
        pp[i] += h
        pm[i] -= h
        fd = (U.loss_and_grads(cfg, pp, x, t, rounding=False)[0]
              - U.loss_and_grads(cfg, pm, x, t, rounding=False)[0]) / (2 * h)
        err = max(err, abs(fd - g[i]))
    scale = np.abs(g).max()
    assert err <= 1e-7 * scale, (err, scale)
    # padding outputs of the head receive no gradient
    off = U.num_params(cfg) - 8 * 8 - 8
    Wh = g[off:off + 64].reshape(8, 8)
    assert np.all(Wh[3:] == 0) and np.all(g[-5:] == 0)


def test_rounded_forward_is_close_to_exact():
    """The BF16 rounding points change the output by O(2^-8) relative."""
    cfg = U.Config(levels=3, base=8, cin=3, cout=3, H=16, W=16)
    params = synth.unet_params(3, 8, seed=8).astype(np.float64)
    x, _ = synth.unet_batch(2, 16, 16, 3, 3, seed=9)
    y0, _ = U.forward(cfg, params, x.astype(np.float64), rounding=False)
    y1, _ = U.forward(cfg, params, x.astype(np.float64), rounding=True)
    rel = np.abs(y1 - y0).max() / np.abs(y0).max()
    assert 1e-5 < rel < 16 * 2 ** -8
