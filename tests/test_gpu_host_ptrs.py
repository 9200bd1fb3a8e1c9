"""Host-pointer mode of the C-ABI: a context created without FR_DEVICE_PTRS
takes host arrays in every compute call (fr_blend, fr_render, fr_backward,
fr_loss_l2, fr_aov, fr_light_reg, fr_adam), copies them to its own device
buffers and back, and waits.  Its results must equal a device-pointer
context's: images, blends, AOV buffers, the loss, E_light and Adam bitwise;
gradients up to the summation order of their atomics (1e-5 of the largest
component).  fr_backward must read the parameters that fr_render copied,
not the caller's arrays, which may have changed in between.  A batch refuses
host-pointer contexts."""
import ctypes as C

import numpy as np
import pytest

from paper_1910_05200_amd import synth

pytestmark = pytest.mark.gpu
SEED, SPP = 1000, 4


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no HIP device")
    return T


@pytest.fixture(scope="module")
def pair(torch):
    from paper_1910_05200_amd import facert
    model, scene, params, _ = synth.workload("tiny")
    dev = facert.Renderer(model, scene)
    host = facert.Renderer(model, scene, host_ptrs=True)
    return model, scene, params, dev, host


def _host_params(params):
    return {k: np.ascontiguousarray(getattr(params, k), np.float32).copy()
            for k in ("alpha", "beta", "delta", "pose", "lights", "spec")}


def _close_grads(a, b, what):
    for k in a:
        x, y = np.asarray(a[k], np.float64), np.asarray(b[k], np.float64)
        tol = 1e-5 * max(np.abs(y).max(), 1e-30)
        assert np.all(np.abs(x - y) <= tol), (what, k, float(np.abs(x - y).max()), tol)


def test_blend_render_aov_loss_match_device_mode(torch, pair):
    from paper_1910_05200_amd import facert
    _, _, params, dev, host = pair
    pd, ph = facert.params_to_device(params), _host_params(params)
    v_d, a_d = dev.blend(pd["alpha"], pd["beta"], pd["delta"], pd["pose"])
    v_h, a_h = host.blend(ph["alpha"], ph["beta"], ph["delta"], ph["pose"])
    assert isinstance(v_h, np.ndarray)
    assert np.array_equal(v_h, v_d.cpu().numpy()) and np.array_equal(a_h, a_d.cpu().numpy())
    img_d = dev.render(pd, SEED, SPP).clone()
    img_h = host.render(ph, SEED, SPP)
    torch.cuda.synchronize()
    assert np.array_equal(img_h, img_d.cpu().numpy())
    assert np.array_equal(host.aov(), dev.aov().cpu().numpy())
    target = (img_h * 0.7 + 0.01).astype(np.float32)
    dl_d, loss_d = dev.loss_l2(img_d, torch.from_numpy(target).cuda())
    dl_h, loss_h = host.loss_l2(img_h, target)
    assert np.array_equal(dl_h, dl_d.cpu().numpy()) and float(loss_h) == float(loss_d)


def test_backward_reads_the_rendered_parameters(torch, pair):
    """The host arrays given to fr_render are overwritten before
    fr_backward: the gradients must still be those of the render."""
    from paper_1910_05200_amd import facert
    _, _, params, dev, host = pair
    pd, ph = facert.params_to_device(params), _host_params(params)
    img_d = dev.render(pd, SEED + 1, SPP).clone()
    img_h = host.render(ph, SEED + 1, SPP)
    assert np.array_equal(img_h, img_d.cpu().numpy())
    for k in ("alpha", "beta", "delta", "lights", "spec"):
        ph[k][...] = np.float32(7.0)
    rng = np.random.default_rng(3)
    dl = rng.normal(size=img_h.shape).astype(np.float32)
    g_d = {k: v.cpu().numpy() for k, v in dev.backward(torch.from_numpy(dl).cuda()).items()}
    g_h = host.backward(dl)
    assert set(g_h) == set(g_d)
    _close_grads(g_h, g_d, "backward")


def test_light_reg_and_adam_match_device_mode(torch, pair):
    _, _, params, dev, host = pair
    rng = np.random.default_rng(9)
    L = rng.uniform(0, 1, (dev.n_lights, 3)).astype(np.float32)
    g0 = rng.normal(size=L.shape).astype(np.float32)
    gd = torch.from_numpy(g0.copy()).cuda()
    gh = g0.copy()
    loss_d = dev.light_reg(torch.from_numpy(L).cuda(), 1e-3, gd)
    loss_h = host.light_reg(L, 1e-3, gh)
    assert float(loss_h) == float(loss_d) and np.array_equal(gh, gd.cpu().numpy())
    n = 1000
    p0 = rng.normal(size=n).astype(np.float32)
    grads = [rng.normal(size=n).astype(np.float32) for _ in range(3)]
    pdv, mdv, vdv = (torch.from_numpy(x).cuda() for x in (p0.copy(), np.zeros(n, np.float32), np.zeros(n, np.float32)))
    ph, mh, vh = p0.copy(), np.zeros(n, np.float32), np.zeros(n, np.float32)
    for t, g in enumerate(grads, start=1):
        dev.adam(pdv, torch.from_numpy(g).cuda(), mdv, vdv, t, 0.01)
        host.adam(ph, g, mh, vh, t, 0.01)
    torch.cuda.synchronize()
    assert np.array_equal(ph, pdv.cpu().numpy()) and np.array_equal(mh, mdv.cpu().numpy())
    assert np.array_equal(vh, vdv.cpu().numpy())


def test_host_mode_errors_and_batch_refusal(torch, pair):
    from paper_1910_05200_amd import facert
    _, _, params, dev, host = pair
    ph = _host_params(params)
    with pytest.raises(facert.FrError):
        host.render(ph, SEED, 0)                    # spp out of range: nothing is rendered
    lib = facert.load()
    out = C.c_void_p()
    arr = (C.c_void_p * 1)(host.ctx.value)
    assert lib.fr_batch_create(1, arr, 0, C.byref(out)) == -1 and not out.value
    arr = (C.c_void_p * 1)(dev.ctx.value)
    assert lib.fr_batch_create(1, arr, 0, C.byref(out)) == 0
    lib.fr_batch_destroy(out)
