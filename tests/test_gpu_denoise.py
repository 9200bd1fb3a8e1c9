"""Denoiser on the GPU (libfadenoise through its C-ABI) against the oracle
network.

Two references.  The oracle in its bfloat16 mode rounds where the library
rounds, so the two differ only in the order and precision of fp32 sums;
such a difference can move a stored value across a bfloat16 rounding
boundary (one ulp, 2^-8 relative) now and then, and the change travels on.
Forward: the bar against it is BAR_EMU of the largest output magnitude,
element by element.  Gradients are more sensitive: perturbing the oracle's
own parameters by 1e-7 relative (fp32-level noise) moves its bfloat16-mode
gradients by up to about 10% in the deepest layers.  So the bar for each
layer's gradient is relative L2 error <= 3 x that measured self-sensitivity
+ 1e-2.  Against the float64 oracle the bar is BAR_F64: what bfloat16
storage costs in all.
"""
import numpy as np
import pytest

from oracle import unet

pytestmark = pytest.mark.gpu
BAR_EMU = 1e-2
BAR_F64 = 2e-1


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no HIP device")
    return T


def _inputs(H, W, seed):
    rng = np.random.default_rng(seed)
    rgb = rng.gamma(0.6, 0.3, (H, W, 3)).astype(np.float32)
    aux = np.concatenate([rng.uniform(0.2, 0.7, (H, W, 3)), rng.normal(size=(H, W, 3)) * 0.5,
                          rng.uniform(0.4, 0.6, (H, W, 1))], axis=2).astype(np.float32)
    tgt = np.clip(rgb + rng.normal(0, 0.05, rgb.shape), 0, None).astype(np.float32)
    return rgb, aux, tgt


def _net(torch, H, W, seed=0):
    from paper_1910_05200_amd import denoise
    dn = denoise.Denoiser(H, W)
    p = denoise.init_params(dn.layer_shapes(), seed)
    # nonzero biases so that the bias paths are exercised
    p = p + np.random.default_rng(seed + 1).normal(0, 0.02, p.shape).astype(np.float32)
    dn.set_params(torch.from_numpy(p).cuda())
    return dn, p


def _rel(got, want):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    return float(np.abs(got - want).max() / max(np.abs(want).max(), 1e-30))


@pytest.mark.parametrize("H,W", [(32, 32), (40, 24), (64, 128)])
def test_forward_parity(torch, H, W):
    dn, p = _net(torch, H, W)
    rgb, aux, _ = _inputs(H, W, H + W)
    out = dn.forward(torch.from_numpy(rgb).cuda(), torch.from_numpy(aux).cuda())
    torch.cuda.synchronize()
    got = np.log1p(out.cpu().numpy())
    r_emu = _rel(got, np.log1p(unet.denoise(p, rgb, aux, bf16=True)))
    r_f64 = _rel(got, np.log1p(unet.denoise(p, rgb, aux)))
    print(f"forward {H}x{W}: max error / max |ref|: bf16 oracle {r_emu:.2e}, fp64 oracle {r_f64:.2e}")
    assert r_emu <= BAR_EMU and r_f64 <= BAR_F64


def _layers():
    off = 0
    for i, (ci, co, k) in enumerate(zip(unet.CIN, unet.COUT, unet.KS)):
        n = co * k * k * ci
        yield f"{i}w", slice(off, off + n)
        yield f"{i}b", slice(off + n, off + n + co)
        off += n + co


def _l2(got, want):
    return float(np.linalg.norm(np.asarray(got, np.float64) - want) / max(np.linalg.norm(want), 1e-30))


def test_gradient_parity(torch):
    H, W = 32, 32
    dn, p = _net(torch, H, W, seed=3)
    rgb, aux, tgt = _inputs(H, W, 9)
    T = lambda a: torch.from_numpy(a).cuda()
    loss, g = dn.train_step(T(rgb), T(aux), T(tgt), 0.0, want_grads=True)
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    l_emu, g_emu = unet.loss_and_grad(p, rgb, aux, tgt, bf16=True)
    noise = np.random.default_rng(1).normal(size=p.shape) * 1e-7
    _, g_pert = unet.loss_and_grad(p.astype(np.float64) * (1 + noise), rgb, aux, tgt, bf16=True)
    l_f64, g_f64 = unet.loss_and_grad(p, rgb, aux, tgt)
    assert abs(float(loss) - l_emu) <= BAR_EMU * l_emu and abs(float(loss) - l_f64) <= BAR_F64 * l_f64
    rows, bad = [], []
    for name, sl in _layers():
        sens = _l2(g_pert[sl], g_emu[sl])
        e_emu, e_f64 = _l2(g[sl], g_emu[sl]), _l2(g[sl], g_f64[sl])
        rows.append(f"{name}:{e_emu:.1e}/{sens:.1e}/{e_f64:.1e}")
        if e_emu > 3 * sens + 1e-2 or e_f64 > BAR_F64:
            bad.append(rows[-1])
    print("relative L2 error per layer (vs bf16 oracle / oracle self-sensitivity / vs fp64):", " ".join(rows))
    assert not bad, bad


def test_training_reduces_the_loss(torch):
    """40 steps toward a learnable target (a 3x3 box blur of the input): the
    loss falls well below that of the untrained network, which passes the
    input through."""
    H, W = 64, 64
    dn, _ = _net(torch, H, W, seed=5)
    rgb, aux, _ = _inputs(H, W, 11)
    pad = np.pad(rgb, ((1, 1), (1, 1), (0, 0)), mode="edge")
    tgt = sum(pad[dy:dy + H, dx:dx + W] for dy in range(3) for dx in range(3)) / 9.0
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    losses = [float(dn.train_step(T(rgb), T(aux), T(tgt), 1e-3)) for _ in range(40)]
    assert losses[-1] < 0.8 * losses[0] and losses[-1] < min(losses[:10]), losses[::8]


def test_input_gradient_parity(torch):
    """fd_backward_input against the oracle's gradient with respect to the
    rgb input (relative L2; the chain runs through every layer)."""
    H, W = 32, 32
    dn, p = _net(torch, H, W, seed=7)
    rgb, aux, _ = _inputs(H, W, 13)
    gout = np.random.default_rng(2).normal(size=(H, W, 3)).astype(np.float32)
    T = lambda a: torch.from_numpy(a).cuda()
    dn.forward(T(rgb), T(aux))
    g = dn.backward_input(T(rgb), T(gout)).cpu().numpy()
    e_emu = _l2(g, unet.input_grad(p, rgb, aux, gout, bf16=True))
    e_f64 = _l2(g, unet.input_grad(p, rgb, aux, gout))
    print(f"input gradient relative L2: bf16 oracle {e_emu:.2e}, fp64 oracle {e_f64:.2e}")
    assert e_emu <= 5e-2 and e_f64 <= BAR_F64


def test_bad_arguments(torch):
    from paper_1910_05200_amd import denoise
    import ctypes as C
    lib = denoise.load()
    out = C.c_void_p()
    assert lib.fd_create(30, 32, C.byref(out)) == -1 and not out.value       # not a multiple of 8
    dn = denoise.Denoiser(16, 16)
    with pytest.raises(denoise.FdError):
        dn.train_step(torch.zeros(16, 16, 3, device="cuda"), torch.zeros(16, 16, 7, device="cuda"),
                      torch.zeros(16, 16, 3, device="cuda"), float("nan"))
    with pytest.raises(denoise.FdError) as e:            # no fd_forward yet
        dn.backward_input(torch.zeros(16, 16, 3, device="cuda"), torch.zeros(16, 16, 3, device="cuda"))
    assert e.value.code == -4


# ---------------------------------------------------------------------------
# Single layers, element by element.  Each kernel of the network (the 3x3
# convolution, its input-gradient form on fp32 gradients, the weight and
# bias gradients) against the float64 oracle on bfloat16-representable
# inputs: the only differences left are the order and precision of the fp32
# sums, so the renderer's parity rule applies, |gpu - ref| <= 1e-4 *
# max(|ref|, 1e-2 * max|ref|).  Sizes cover ragged pixel tiles (8 x 16) and
# channel counts that are not multiples of the channel tile.

LAYER_CASES = [(8, 16, 16, 32), (24, 40, 32, 64), (17, 23, 96, 32), (13, 31, 64, 128), (32, 32, 384, 128),
               (16, 16, 256, 256), (9, 33, 32, 16), (64, 64, 32, 32)]


def _bf16_bits(t64):
    """bfloat16 bit patterns (int16 tensor) of the bfloat16-rounded values."""
    import torch
    r = unet.bf16_round(torch.as_tensor(t64))
    u = r.to(torch.float32).contiguous().numpy().view(np.uint32) >> 16
    return torch.from_numpy(u.astype(np.uint16).view(np.int16)), r.numpy()


def _floor_rule(got, ref, name):
    from parity import assert_group_parity
    return assert_group_parity(got, ref, name)


@pytest.mark.parametrize("H,W,cin,cout", LAYER_CASES)
def test_conv3x3_layer_elementwise(torch, H, W, cin, cout):
    from paper_1910_05200_amd import denoise
    rng = np.random.default_rng(H * 1000 + cin)
    xb, x = _bf16_bits(rng.normal(size=(H, W, cin)))
    wb, w = _bf16_bits(rng.normal(0, 1 / np.sqrt(9 * cin), size=(cout, 9, cin)))
    bias = rng.normal(0, 0.1, size=cout).astype(np.float32)
    y = denoise.conv3x3(xb.cuda(), wb.cuda(), torch.from_numpy(bias).cuda(), relu=True)
    torch.cuda.synchronize()
    ref = unet.conv3x3_layer(x, w, bias.astype(np.float64), relu=True)
    print(_floor_rule(y.cpu().numpy(), ref, f"conv {H}x{W} {cin}->{cout}"))


@pytest.mark.parametrize("H,W,cin,cout", LAYER_CASES[:5])
def test_conv3x3_input_gradient_elementwise(torch, H, W, cin, cout):
    """The input-gradient pass: fp32 gradients (rounded to bfloat16 as read)
    through the flipped, transposed weights equal the oracle's input
    gradient of the layer."""
    from paper_1910_05200_amd import denoise
    rng = np.random.default_rng(W * 100 + cout)
    g = rng.normal(size=(H, W, cout)).astype(np.float32)
    _, g_r = _bf16_bits(g.astype(np.float64))
    wb, w = _bf16_bits(rng.normal(0, 1 / np.sqrt(9 * cin), size=(cout, 9, cin)))
    # flipped, transposed weights: wf[ci][t][co] = w[co][8 - t][ci]
    wf = np.ascontiguousarray(w[:, ::-1, :].transpose(2, 1, 0))
    wfb, _ = _bf16_bits(wf)
    dx = denoise.conv3x3(torch.from_numpy(g).cuda(), wfb.cuda(), x_is_f32=True)
    torch.cuda.synchronize()
    print(_floor_rule(dx.cpu().numpy(), unet.conv3x3_input_grad(g_r, w), f"input grad {H}x{W} {cin}<-{cout}"))


@pytest.mark.parametrize("H,W,cin,cout", LAYER_CASES)
def test_conv3x3_weight_gradient_elementwise(torch, H, W, cin, cout):
    from paper_1910_05200_amd import denoise
    rng = np.random.default_rng(H + W + cin + cout)
    xb, x = _bf16_bits(rng.normal(size=(H, W, cin)))
    g = rng.normal(size=(H, W, cout)).astype(np.float32)
    _, g_r = _bf16_bits(g.astype(np.float64))
    dw, db = denoise.conv3x3_wgrad(xb.cuda(), torch.from_numpy(g).cuda())
    torch.cuda.synchronize()
    ref_w, ref_b = unet.conv3x3_weight_grad(x, g_r)
    print(_floor_rule(dw.cpu().numpy(), ref_w, f"weight grad {H}x{W} {cin}->{cout}"))
    # the bias gradient sums the unrounded fp32 gradient
    print(_floor_rule(db.cpu().numpy(), g.astype(np.float64).sum(axis=(0, 1)), "bias grad"))


def test_single_layer_argument_errors(torch):
    from paper_1910_05200_amd import denoise
    lib = denoise.load()
    z = torch.zeros(64, device="cuda")
    assert lib.fd_conv3x3(None, 4, 4, 24, 8, z.data_ptr(), 0, z.data_ptr(), None, 0, z.data_ptr()) == -1  # cin % 16
    assert lib.fd_conv3x3(None, 0, 4, 16, 8, z.data_ptr(), 0, z.data_ptr(), None, 0, z.data_ptr()) == -1
    assert lib.fd_conv3x3(None, 4, 4, 16, 8, None, 0, z.data_ptr(), None, 0, z.data_ptr()) == -1
    assert lib.fd_conv3x3_wgrad(None, 4, 4, 12, 8, z.data_ptr(), z.data_ptr(), z.data_ptr(), None) == -1


def test_batched_network_equals_single_image_networks(torch):
    """A network made for n images per call (fd_create_batch) against a
    one-image network with the same weights: the forward and the input
    gradient of every image bit for bit (the same kernels, per-pixel sums in
    the same order; no image reads another's pixels across the stack), the
    training gradient equal to the mean of the single images' gradients up
    to fp32 summation order (the batched loss is the mean over all images'
    pixels), at the renderer's per-component bar with each layer's floor.
    n is a power of two: the batched loss gradient is the single image's
    divided by n, and only then does that scaling commute with the bfloat16
    rounding of the gradients where they enter a product (with n = 3 the
    two roundings differ by up to 2^-8 per element, and the weight
    gradients by about 1%, as for any two equally valid bf16 evaluations)."""
    from paper_1910_05200_amd import denoise
    from parity import assert_group_parity
    H, W, n = 64, 96, 4
    one, p = _net(torch, H, W, seed=4)
    many = denoise.Denoiser(H, W, n=n)
    many.set_params(torch.from_numpy(p).cuda())
    ins = [_inputs(H, W, 40 + i) for i in range(n)]
    rgb = torch.from_numpy(np.stack([a[0] for a in ins])).cuda()
    aux = torch.from_numpy(np.stack([a[1] for a in ins])).cuda()
    tgt = torch.from_numpy(np.stack([a[2] for a in ins])).cuda()
    out = many.forward(rgb, aux).clone()
    rng = np.random.default_rng(8)
    gout = torch.from_numpy(rng.normal(size=(n, H, W, 3)).astype(np.float32)).cuda()
    gin = many.backward_input(rgb, gout).clone()
    for i in range(n):
        o1 = one.forward(rgb[i], aux[i])
        assert torch.equal(o1, out[i]), i
        assert torch.equal(one.backward_input(rgb[i], gout[i]), gin[i]), i
    # gradients of a training step (the step's update itself is not compared)
    many.set_params(torch.from_numpy(p).cuda())
    _, g_many = many.train_step(rgb, aux, tgt, 0.0, want_grads=True)
    g_ref = np.zeros(p.shape, np.float64)
    for i in range(n):
        one.set_params(torch.from_numpy(p).cuda())
        _, g1 = one.train_step(rgb[i], aux[i], tgt[i], 0.0, want_grads=True)
        g_ref += g1.cpu().numpy().astype(np.float64) / n
    g_many = g_many.cpu().numpy()
    off = 0
    for li, (ci, co, k) in enumerate(many.layer_shapes()):
        nw = co * k * k * ci
        assert_group_parity(g_many[off:off + nw], g_ref[off:off + nw], f"layer {li} weights")
        assert_group_parity(g_many[off + nw:off + nw + co], g_ref[off + nw:off + nw + co], f"layer {li} bias")
        off += nw + co
    assert off == p.size
