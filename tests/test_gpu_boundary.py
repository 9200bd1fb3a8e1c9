"""GPU parity of the boundary's smaller calls against the oracle, and of the
torch.autograd wrapper against the call it wraps.

* fr_loss_l2: E_data of Eq. 1 and its image gradient 2 (I - T), element by
  element against the oracle's definition, on oracle renders (tiny, a
  ragged image, paper scale).  Pixel bar: 1e-4 relative; the loss: 1e-4
  relative (an fp32 sum).
* fr_aov: the denoiser's input buffers (mean albedo, shading normal and
  depth of the first hits) against orc_aov: albedo and depth 1e-4
  relative, normal components by the group floor rule.
* face_render (FaceRender): loss.backward() through it gives Renderer.backward's
  gradients, also when another render ran in between; an in-place change
  to a saved input raises.
"""
import numpy as np
import pytest

from paper_1910_05200_amd import synth
from parity import assert_group_parity, assert_image_parity

pytestmark = pytest.mark.gpu
SEED = 1000


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no HIP device")
    return T


def _scene(name):
    if name == "ragged":
        return synth.make_model(7, 11), synth.make_scene(37, 23), synth.make_params(5), 3
    return synth.workload(name)


@pytest.mark.parametrize("name", ["tiny", "ragged", "paper"])
def test_loss_l2_parity(torch, orc, name):
    from paper_1910_05200_amd import facert
    model, scene, params, spp = _scene(name)
    spp = 1 if name == "paper" else spp
    osc, _, _ = orc.scene_from_model(model, scene, params)
    tosc, _, _ = orc.scene_from_model(model, scene, synth.make_params(synth.TARGET_SCENE_SEED))
    I = orc.render(osc, SEED, spp).astype(np.float32)
    T = orc.render(tosc, synth.TARGET_RENDER_SEED, spp).astype(np.float32)
    L_ref, g_ref = orc.loss_l2(I, T)
    r = facert.Renderer(model, scene)
    dL, loss = r.loss_l2(torch.from_numpy(I).cuda(), torch.from_numpy(T).cuda())
    torch.cuda.synchronize()
    assert_image_parity(dL.cpu().numpy(), g_ref, what="dL/dI")
    assert abs(float(loss) - L_ref) <= 1e-4 * L_ref, (float(loss), L_ref)
    assert L_ref > 0


def _aov_compare(got, ref):
    got = np.asarray(got, np.float64).reshape(-1, 7)
    ref = np.asarray(ref, np.float64).reshape(-1, 7)
    assert_image_parity(got[:, :3], ref[:, :3], what="aov albedo")
    assert_image_parity(got[:, 6], ref[:, 6], what="aov depth")
    assert_group_parity(got[:, 3:6], ref[:, 3:6], "aov normal")


@pytest.mark.parametrize("name", ["tiny", "ragged"])
def test_aov_parity(torch, orc, name):
    from paper_1910_05200_amd import facert
    model, scene, params, spp = _scene(name)
    r = facert.Renderer(model, scene)
    r.render(facert.params_to_device(params), SEED, spp)
    got = r.aov().cpu().numpy()
    osc, _, _ = orc.scene_from_model(model, scene, params)
    ref = orc.aov(osc, SEED, spp)
    assert (ref[..., 6] > 0).mean() > 0.2 and (ref[..., 6] == 0).any()
    _aov_compare(got, ref)


def test_aov_parity_paper_sampled(torch, orc):
    from paper_1910_05200_amd import facert
    model, scene, params, spp = synth.workload("paper")
    r = facert.Renderer(model, scene)
    r.render(facert.params_to_device(params), SEED, spp)
    got = r.aov().cpu().numpy().reshape(-1, 7)
    osc, _, _ = orc.scene_from_model(model, scene, params)
    rng = np.random.default_rng(1)
    hit = np.flatnonzero(got[:, 6] > 0)
    pix = np.concatenate([rng.choice(hit, 384, replace=False), rng.integers(0, 256 * 256, 128)])
    _aov_compare(got[pix], orc.aov(osc, SEED, spp, pixels=pix))


def test_aov_needs_the_kept_records(torch):
    from paper_1910_05200_amd import facert
    model, scene, params, spp = synth.workload("tiny")
    r = facert.Renderer(model, scene)
    with pytest.raises(facert.FrError) as e:            # no render yet
        r.aov()
    assert e.value.code == -4
    r.set_chunk(5000)                                   # 16,384 samples: more than one chunk
    r.render(facert.params_to_device(params), SEED, spp)
    with pytest.raises(facert.FrError) as e:
        r.aov()
    assert e.value.code == -4


def _leaves(torch, params):
    out = {}
    for k in ("alpha", "beta", "delta", "pose", "lights", "spec"):
        dev = "cpu" if k == "pose" else "cuda"
        out[k] = torch.tensor(np.asarray(getattr(params, k), np.float32), device=dev, requires_grad=True)
    return out


@pytest.mark.parametrize("between", [False, True])
def test_autograd_matches_backward(torch, between):
    """loss = sum (face_render(...) - T)^2; loss.backward() must give what
    fr_backward gives for dL/dI = 2 (I - T), every group, also when another
    render used the renderer between the forward and the backward (the
    wrapper then replays the forward)."""
    from paper_1910_05200_amd import facert
    model, scene, params, spp = synth.workload("tiny")
    r = facert.Renderer(model, scene)
    T = torch.from_numpy(np.random.default_rng(3).uniform(0, 0.05, (scene.height, scene.width, 3))
                         .astype(np.float32)).cuda()
    x = _leaves(torch, params)
    img = facert.face_render(r, SEED, spp, x["alpha"], x["beta"], x["delta"], x["pose"], x["lights"], x["spec"])
    ref_img = img.detach().clone()
    if between:
        other = synth.make_params(9)
        r.render(facert.params_to_device(other), SEED + 5, 2)
    loss = ((img - T) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    # reference: the plain calls on a fresh renderer
    r2 = facert.Renderer(model, scene)
    img2 = r2.render(facert.params_to_device(params), SEED, spp)
    assert torch.equal(img2, ref_img)
    g = r2.backward((2 * (img2 - T)).contiguous())
    torch.cuda.synchronize()
    names = {"alpha": "d_alpha", "beta": "d_beta", "delta": "d_delta", "pose": "d_pose",
             "lights": "d_lights", "spec": "d_spec"}
    for k, gk in names.items():
        got = x[k].grad.detach().cpu().numpy().reshape(-1)
        want = g[gk].cpu().numpy().reshape(-1)
        scale = max(float(np.abs(want).max()), 1e-30)
        # the same kernels: equal up to the order of their float atomics
        assert np.abs(got - want).max() <= 2e-5 * scale, (k, np.abs(got - want).max() / scale)
        assert np.abs(want).max() > 0, k


def test_autograd_refuses_inputs_changed_in_place(torch):
    from paper_1910_05200_amd import facert
    model, scene, params, spp = synth.workload("tiny")
    r = facert.Renderer(model, scene)
    x = _leaves(torch, params)
    img = facert.face_render(r, SEED, spp, x["alpha"], x["beta"], x["delta"], x["pose"], x["lights"], x["spec"])
    loss = img.sum()
    with torch.no_grad():
        x["lights"].mul_(1.1)                        # an optimiser step before backward
    with pytest.raises(RuntimeError):
        loss.backward()
