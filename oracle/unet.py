"""Oracle of the denoiser network (test infrastructure only).

The same U-Net as the GPU library, written with plain PyTorch CPU operations
in float64, from the flat parameter vector in the library's layout (for
each layer: weights [Cout][k*k][Cin], tap t = 3 (dy + 1) + (dx + 1), then
bias [Cout]).  Only the test suite imports it.

With bf16=True the same computation rounds to bfloat16 (nearest even, from
the float32 value) at the points where the GPU library stores or feeds
bfloat16: the packed input, the 3x3 weights, every 3x3 convolution's
output after its activation, every pooled value, and, in the backward pass,
the gradient of each 3x3 convolution's pre-activation where it enters the
weight-gradient and input-gradient products (its bias gradient and all other
gradients stay unrounded).  Sums are exact (float64) in both modes.  This
is the network at the precision the library computes in, so the library can
be held to it tightly; the float64 mode bounds what bfloat16 costs.

Network: input channels log(1 + 16 rgb), albedo, normal, depth, zero-padded
to 16; per level two 3x3 convolutions (zero padding) with leaky ReLU (slope
0.01), channels 32, 64, 128, 256; 2x2 average pooling down; nearest 2x
upsampling, then concatenation [upsampled, skip] up; a 1x1 output
convolution gives a correction added to the input's log(1 + 16 rgb).
Output radiance expm1(pred) / 16.  Loss: mean of (pred - log(1 + 16
target))^2.  input_grad is the gradient of a loss on the output with
respect to the rgb input (the packed input's rounding passed straight
through, as the library does).
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

SLOPE = 0.01
EXPOSURE = 16.0
CIN = [16, 32, 32, 64, 64, 128, 128, 256, 384, 128, 192, 64, 96, 32, 32]
COUT = [32, 32, 64, 64, 128, 128, 256, 256, 128, 128, 64, 64, 32, 32, 3]
KS = [3] * 14 + [1]


def unpack(params):
    """Flat vector -> list of (weight [Cout][Cin][k][k], bias) tensors."""
    p = torch.as_tensor(np.asarray(params, np.float64))
    out, off = [], 0
    for ci, co, k in zip(CIN, COUT, KS):
        n = co * k * k * ci
        w = p[off:off + n].reshape(co, k, k, ci).permute(0, 3, 1, 2).contiguous()   # [co][ci][ky][kx]
        off += n
        b = p[off:off + co]
        off += co
        out.append((w, b))
    assert off == p.numel()
    return out


def pack_input(rgb, aux):
    """[H][W][3], [H][W][7] -> [1][16][H][W] float64."""
    rgb = torch.as_tensor(np.asarray(rgb, np.float64))
    aux = torch.as_tensor(np.asarray(aux, np.float64))
    H, W = rgb.shape[:2]
    x = torch.zeros(1, 16, H, W, dtype=torch.float64)
    x[0, :3] = torch.log1p(EXPOSURE * rgb.clamp(min=0)).permute(2, 0, 1)
    x[0, 3:10] = aux.permute(2, 0, 1)
    return x


def bf16_round(t):
    """Round to bfloat16 (nearest even) through float32, kept in float64."""
    f = t.detach().to(torch.float32).contiguous().numpy()
    u = f.view(np.uint32).astype(np.uint64)
    u = (((u + 0x7fff + ((u >> 16) & 1)) >> 16) << 16).astype(np.uint32)
    return torch.from_numpy(u.view(np.float32).astype(np.float64)).reshape(t.shape)


class _ConvBF16(torch.autograd.Function):
    """3x3 convolution + leaky ReLU with the library's bfloat16 rounding."""

    @staticmethod
    def forward(ctx, x, w, b):
        wr = bf16_round(w)
        y = bf16_round(F.leaky_relu(F.conv2d(x, wr, b, padding=1), SLOPE))
        ctx.save_for_backward(x, wr, y)
        return y

    @staticmethod
    def backward(ctx, gy):
        x, wr, y = ctx.saved_tensors
        gpre = torch.where(y > 0, gy, SLOPE * gy)
        gr = bf16_round(gpre)
        dw = torch.nn.grad.conv2d_weight(x, wr.shape, gr, padding=1)
        dx = torch.nn.grad.conv2d_input(x.shape, wr, gr, padding=1)
        return dx, dw, gpre.sum(dim=(0, 2, 3))


class _PoolBF16(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x):
        return bf16_round(F.avg_pool2d(x, 2))

    @staticmethod
    def backward(ctx, g):
        return F.interpolate(g, scale_factor=2, mode="nearest") * 0.25


def forward(layers, x, bf16=False):
    """log-radiance [1][3][H][W] for input x [1][16][H][W] (its first three
    channels, unrounded, are the log-radiance the output corrects)."""
    x_log = x[:, :3]
    def conv(i, t, act=True):
        w, b = layers[i]
        if bf16 and act:
            return _ConvBF16.apply(t, w, b)
        y = F.conv2d(t, w, b, padding=w.shape[-1] // 2)
        return F.leaky_relu(y, SLOPE) if act else y

    pool = _PoolBF16.apply if bf16 else (lambda t: F.avg_pool2d(t, 2))
    if bf16:
        x = x + (bf16_round(x) - x).detach()     # rounded value, gradient passed straight through
    e0 = conv(1, conv(0, x))
    e1 = conv(3, conv(2, pool(e0)))
    e2 = conv(5, conv(4, pool(e1)))
    e3 = conv(7, conv(6, pool(e2)))
    up = lambda t: F.interpolate(t, scale_factor=2, mode="nearest")
    d2 = conv(9, conv(8, torch.cat([up(e3), e2], 1)))
    d1 = conv(11, conv(10, torch.cat([up(d2), e1], 1)))
    d0 = conv(13, conv(12, torch.cat([up(d1), e0], 1)))
    return x_log + conv(14, d0, act=False)


def denoise(params, rgb, aux, bf16=False):
    """Radiance [H][W][3] (numpy float64)."""
    with torch.no_grad():
        pred = forward(unpack(params), pack_input(rgb, aux), bf16)
    return (torch.expm1(pred) / EXPOSURE)[0].permute(1, 2, 0).numpy()


def loss_and_grad(params, rgb, aux, target, bf16=False):
    """(loss, d loss / d params as a flat float64 numpy vector)."""
    p = torch.tensor(np.asarray(params, np.float64), requires_grad=True)
    layers, off = [], 0
    for ci, co, k in zip(CIN, COUT, KS):
        n = co * k * k * ci
        w = p[off:off + n].reshape(co, k, k, ci).permute(0, 3, 1, 2)
        off += n
        layers.append((w, p[off:off + co]))
        off += co
    pred = forward(layers, pack_input(rgb, aux), bf16)
    tgt = torch.log1p(EXPOSURE * torch.as_tensor(np.asarray(target, np.float64)).clamp(min=0)).permute(2, 0, 1)[None]
    loss = ((pred - tgt) ** 2).mean()
    loss.backward()
    return float(loss), p.grad.numpy().copy()


def input_grad(params, rgb, aux, dL_dout, bf16=False):
    """d/d rgb of sum(dL_dout * denoised radiance), [H][W][3] float64."""
    rgb_t = torch.tensor(np.asarray(rgb, np.float64), requires_grad=True)
    x = torch.zeros(1, 16, *rgb_t.shape[:2], dtype=torch.float64)
    x = torch.cat([torch.log1p(EXPOSURE * rgb_t.clamp(min=0)).permute(2, 0, 1)[None],
                   torch.as_tensor(np.asarray(aux, np.float64)).permute(2, 0, 1)[None], x[:, 10:]], 1)
    pred = forward(unpack(params), x, bf16)
    out = (torch.expm1(pred) / EXPOSURE)[0].permute(1, 2, 0)
    (out * torch.as_tensor(np.asarray(dL_dout, np.float64))).sum().backward()
    return rgb_t.grad.numpy().copy()


# ------------------------------------------------------------ single layers
# One 3x3 convolution and its two gradients in float64, [H][W][C] layouts,
# weights [Cout][9][Cin] with tap t = 3 (dy + 1) + (dx + 1) (the layout the
# direct-loop pin checks).  Inputs are taken as given (a caller that models
# bfloat16 storage rounds them first with bf16_round).

def _w4(w):
    w = torch.as_tensor(np.asarray(w, np.float64))
    co, _, ci = w.shape
    return w.reshape(co, 3, 3, ci).permute(0, 3, 1, 2).contiguous()      # [co][ci][ky][kx]


def conv3x3_layer(x, w, bias=None, relu=False):
    """act(bias + conv(x, w)), [H][W][Cout] float64."""
    xt = torch.as_tensor(np.asarray(x, np.float64)).permute(2, 0, 1)[None]
    b = None if bias is None else torch.as_tensor(np.asarray(bias, np.float64))
    y = F.conv2d(xt, _w4(w), b, padding=1)
    if relu:
        y = F.leaky_relu(y, SLOPE)
    return y[0].permute(1, 2, 0).numpy()


def conv3x3_input_grad(g, w):
    """d/dx of sum(g * conv(x, w)), [H][W][Cin] float64."""
    gt = torch.as_tensor(np.asarray(g, np.float64)).permute(2, 0, 1)[None]
    w4 = _w4(w)
    H, W = gt.shape[2:]
    dx = torch.nn.grad.conv2d_input((1, w4.shape[1], H, W), w4, gt, padding=1)
    return dx[0].permute(1, 2, 0).numpy()


def conv3x3_weight_grad(x, g):
    """(d/dw [Cout][9][Cin], d/dbias [Cout]) of sum(g * (bias + conv(x, w))), float64."""
    xt = torch.as_tensor(np.asarray(x, np.float64)).permute(2, 0, 1)[None]
    gt = torch.as_tensor(np.asarray(g, np.float64)).permute(2, 0, 1)[None]
    co, ci = gt.shape[1], xt.shape[1]
    dw = torch.nn.grad.conv2d_weight(xt, (co, ci, 3, 3), gt, padding=1)       # [co][ci][ky][kx]
    return dw.permute(0, 2, 3, 1).reshape(co, 9, ci).numpy(), gt.sum(dim=(0, 2, 3)).numpy()
