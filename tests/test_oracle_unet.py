"""Pins of the denoiser oracle: parameter layout and tap order against a
direct loop, pooling / upsampling / concatenation semantics, and its
gradient against central finite differences."""
import numpy as np
import pytest
import torch

from oracle import unet


def _n_params():
    return sum(co * k * k * ci + co for ci, co, k in zip(unet.CIN, unet.COUT, unet.KS))


def test_conv_layout_matches_a_direct_loop():
    """Weight [co][t][ci] with t = 3 (dy + 1) + (dx + 1) applied to the
    neighbour (y + dy, x + dx), zero outside the image."""
    rng = np.random.default_rng(0)
    ci, co, H, W = 16, 32, 5, 7
    wflat = rng.normal(size=(co, 9, ci))
    bias = rng.normal(size=co)
    x = rng.normal(size=(H, W, ci))
    params = np.zeros(_n_params())
    params[:co * 9 * ci] = wflat.ravel()
    params[co * 9 * ci:co * 9 * ci + co] = bias
    w, b = unet.unpack(params)[0]
    got = torch.nn.functional.conv2d(torch.tensor(x).permute(2, 0, 1)[None], w, b, padding=1)[0].permute(1, 2, 0).numpy()
    want = np.zeros((H, W, co))
    for y in range(H):
        for xx in range(W):
            acc = bias.copy()
            for t in range(9):
                sy, sx = y + t // 3 - 1, xx + t % 3 - 1
                if 0 <= sy < H and 0 <= sx < W:
                    acc += wflat[:, t, :] @ x[sy, sx]
            want[y, xx] = acc
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)


def test_pool_upsample_concat_semantics():
    t = torch.arange(16.0, dtype=torch.float64).reshape(1, 1, 4, 4)
    pooled = torch.nn.functional.avg_pool2d(t, 2)
    np.testing.assert_allclose(pooled[0, 0].numpy(), [[2.5, 4.5], [10.5, 12.5]])
    up = torch.nn.functional.interpolate(pooled, scale_factor=2, mode="nearest")
    np.testing.assert_allclose(up[0, 0, :2, :2].numpy(), [[2.5, 2.5], [2.5, 2.5]])
    np.testing.assert_allclose(up[0, 0, 2:, 2:].numpy(), [[12.5, 12.5], [12.5, 12.5]])


def test_input_packing():
    rgb = np.full((8, 8, 3), (np.e - 1) / unet.EXPOSURE)
    aux = np.arange(7.0)[None, None, :] * np.ones((8, 8, 1))
    x = unet.pack_input(rgb, aux)
    assert x.shape == (1, 16, 8, 8)
    np.testing.assert_allclose(x[0, :3].numpy(), 1.0)
    np.testing.assert_allclose(x[0, 3:10, 0, 0].numpy(), np.arange(7.0))
    assert float(x[0, 10:].abs().max()) == 0.0


@pytest.mark.parametrize("which", [0, 7, 12, 14])
def test_gradient_matches_finite_differences(which):
    rng = np.random.default_rng(which)
    params = rng.normal(size=_n_params()) * 0.05
    rgb = rng.uniform(0, 1, (8, 8, 3))
    aux = rng.uniform(-1, 1, (8, 8, 7))
    tgt = rng.uniform(0, 1, (8, 8, 3))
    _, g = unet.loss_and_grad(params, rgb, aux, tgt)
    off = 0
    for i, (ci, co, k) in enumerate(zip(unet.CIN, unet.COUT, unet.KS)):
        if i == which:
            break
        off += co * k * k * ci + co
    idx = [off, off + 5, off + co * k * k * ci]          # two weights and the first bias
    h = 1e-6
    for j in idx:
        pp, pm = params.copy(), params.copy()
        pp[j] += h
        pm[j] -= h
        fd = (unet.loss_and_grad(pp, rgb, aux, tgt)[0] - unet.loss_and_grad(pm, rgb, aux, tgt)[0]) / (2 * h)
        assert fd == pytest.approx(g[j], rel=1e-5, abs=1e-10)


def test_single_layer_gradients_are_the_adjoints_of_the_layer():
    """The single-layer references: the input and weight gradients satisfy
    <conv(x, w), g> = <x, input_grad(g, w)> = <w, weight_grad(x, g)>, and
    the bias gradient is the sum of g; the layer itself is the direct-loop
    layout (test_conv_layout_matches_a_direct_loop) through conv3x3_layer."""
    rng = np.random.default_rng(4)
    H, W, ci, co = 6, 9, 16, 24
    x, w, g = rng.normal(size=(H, W, ci)), rng.normal(size=(co, 9, ci)), rng.normal(size=(H, W, co))
    b = rng.normal(size=co)
    y = unet.conv3x3_layer(x, w)
    dx = unet.conv3x3_input_grad(g, w)
    dw, db = unet.conv3x3_weight_grad(x, g)
    lhs = float(np.sum(y * g))
    assert abs(lhs - float(np.sum(x * dx))) <= 1e-10 * abs(lhs)
    assert abs(lhs - float(np.sum(w * dw))) <= 1e-10 * abs(lhs)
    np.testing.assert_allclose(db, g.sum(axis=(0, 1)), rtol=1e-12)
    yb = unet.conv3x3_layer(x, w, b, relu=True)
    pre = y + b
    np.testing.assert_allclose(yb, np.where(pre > 0, pre, unet.SLOPE * pre), rtol=1e-12, atol=1e-12)
    # the direct loop of the layout pin, once more through conv3x3_layer
    want = np.zeros((H, W, co))
    for yy in range(H):
        for xx in range(W):
            for t in range(9):
                sy, sx = yy + t // 3 - 1, xx + t % 3 - 1
                if 0 <= sy < H and 0 <= sx < W:
                    want[yy, xx] += w[:, t, :] @ x[sy, sx]
    np.testing.assert_allclose(y, want, rtol=1e-11, atol=1e-11)
