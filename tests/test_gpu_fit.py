"""Fitting loop on the GPU: fr_adam and fr_light_reg against the oracle's
plain float64 definitions, and a short fit that must reduce the error."""
import numpy as np
import pytest

from oracle import fitting
from paper_1910_05200_amd import synth
from parity import assert_group_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no HIP device")
    return T


@pytest.fixture(scope="module")
def renderer(torch):
    from paper_1910_05200_amd import facert
    model, scene, _, _ = synth.workload("tiny")
    return facert.Renderer(model, scene)


@pytest.mark.parametrize("n", [1, 255, 1000, 4099])
def test_adam_parity(torch, renderer, n):
    rng = np.random.default_rng(n)
    p0 = rng.normal(size=n).astype(np.float32)
    scales = [1e-3, 1.0, 30.0, 0.0, 1e-6, 2.0, 0.5]
    grads = [(rng.normal(size=n) * s).astype(np.float32) for s in scales]
    p = torch.from_numpy(p0.copy()).cuda()
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    rp, rm, rv = p0.astype(np.float64), np.zeros(n), np.zeros(n)
    for t, g in enumerate(grads, start=1):
        renderer.adam(p, torch.from_numpy(g).cuda(), m, v, t, 0.01, 0.9, 0.999, 1e-8)
        rp, rm, rv = fitting.adam(rp, g.astype(np.float64), rm, rv, t, 0.01, 0.9, 0.999, 1e-8)
    torch.cuda.synchronize()
    # The updates carry the test: compare p - p0 at the 1e-4 bar.  The GPU
    # stores p in fp32 after each step, which adds up to half an ulp of |p|
    # per step on top of that bar.
    got = p.cpu().numpy().astype(np.float64)
    ulp = np.spacing(np.abs(rp).astype(np.float32)).astype(np.float64)
    ref_d = rp - p0
    floor = 1e-2 * np.abs(ref_d).max()
    tol = 1e-4 * np.maximum(np.abs(ref_d), floor) + 0.5 * len(grads) * ulp
    assert np.all(np.abs(got - rp) <= tol), float(np.max(np.abs(got - rp) / tol))
    assert_group_parity(m.cpu().numpy(), rm, "adam m")
    assert_group_parity(v.cpu().numpy(), rv, "adam v")


def test_adam_rejects_bad_arguments(torch, renderer):
    from paper_1910_05200_amd import facert
    p = torch.zeros(4, device="cuda")
    with pytest.raises(facert.FrError):
        renderer.adam(p, p.clone(), p.clone(), p.clone(), 0, 0.1)        # step counts from 1
    with pytest.raises(facert.FrError):
        renderer.adam(p, p.clone(), p.clone(), p.clone(), 1, 0.1, beta1=1.0)


def test_light_reg_parity(torch, renderer):
    rng = np.random.default_rng(5)
    L = rng.uniform(0, 1, (20, 3)).astype(np.float32)
    L[3] = 0.0
    lights = torch.from_numpy(L).cuda()
    grad = torch.zeros((20, 3), device="cuda")
    loss = renderer.light_reg(lights, 1e-3, grad)
    # the gradient is added to what the buffer holds: one fp32 rounding
    g0 = rng.normal(size=(20, 3)).astype(np.float32)
    acc = torch.from_numpy(g0.copy()).cuda()
    renderer.light_reg(lights, 1e-3, acc)
    torch.cuda.synchronize()
    e, ge = fitting.light_reg(L.astype(np.float64), 1e-3)
    assert abs(float(loss) - e) <= 1e-4 * abs(e)
    assert_group_parity(grad.cpu().numpy(), ge, "E_light gradient")
    want = g0.astype(np.float64) + ge
    assert np.all(np.abs(acc.cpu().numpy() - want) <= 1e-4 * np.abs(ge) + np.spacing(np.abs(want).astype(np.float32)))


def test_short_fit_reduces_error(torch, renderer):
    """40 iterations from the perturbed start on the tiny workload: the data
    term falls, the fitted render moves toward the target (PSNR) and so does
    the pose.  Lights, albedo and texels are not checked one by one: light
    colour times albedo is ambiguous in the image, E_light only tilts it."""
    from paper_1910_05200_amd import facert, fit
    truth = synth.make_params(synth.TARGET_SCENE_SEED)
    start = synth.perturb(truth, fit.START_SEED)
    target = renderer.render(facert.params_to_device(truth), synth.TARGET_RENDER_SEED, 64).clone()
    tgt = target.cpu().numpy()
    psnr0 = fit.psnr(renderer.render(facert.params_to_device(start), 99, 64).cpu().numpy(), tgt)
    p, losses, _ = fit.fit(renderer, target, start, 40, 4)
    psnr1 = fit.psnr(renderer.render(p, 99, 64).cpu().numpy(), tgt)
    e0 = fit.param_errors(facert.params_to_device(start), truth)
    e1 = fit.param_errors(p, truth)
    print({k: (round(e0[k], 4), round(e1[k], 4)) for k in e0}, losses[0], np.mean(losses[-5:]), psnr0, psnr1)
    assert np.mean(losses[-5:]) < 0.5 * losses[0]
    assert psnr1 > psnr0 + 2.0
    assert e1["rot_deg"] < e0["rot_deg"]


def test_sequence_fit_runs_every_mode(torch):
    """Two frames with shared identity/albedo/lights, 12 iterations on the
    tiny workload, plain and both denoised modes: the frames' PSNR rises."""
    from paper_1910_05200_amd import denoise, facert, sequence
    model, scene, _, _ = synth.workload("tiny")
    r = facert.Renderer(model, scene)
    base, frames = sequence.make_truth(2)
    start, start_frames = sequence.make_start(base, frames)
    targets = [r.render(facert.params_to_device(sequence.frame_params_np(base, b, p)), 7 + f, 64).clone()
               for f, (b, p) in enumerate(frames)]
    dn = denoise.Denoiser(scene.height, scene.width)
    denoise.train(r, dn, 8, 1, log=None)
    rs = sequence.frame_renderers(model, scene, 2)
    for mode, spp in (("plain", 4), ("denoised", 2), ("denoised-st", 2)):
        out = sequence.run(r, targets, base, frames, start, start_frames, 12, mode, spp, dn, eval_spp=16,
                           log_every=12, rs=rs)
        first, last = out["log"][0]["psnr_db"], out["log"][-1]["psnr_db"]
        print(mode, spp, first, last)
        assert out["batched"] and last > first + 1.0, (mode, first, last)
    # a denoiser made for both frames (one call for the stack) gives each
    # frame's denoised image and input gradient bit for bit: the same fit
    # up to the renderer's atomics order
    dn2 = denoise.Denoiser(scene.height, scene.width, n=2)
    dn2.set_params(dn.get_params())
    for mode in ("denoised", "denoised-st"):
        one = sequence.run(r, targets, base, frames, start, start_frames, 6, mode, 2, dn, eval_spp=16,
                           log_every=6, rs=rs)
        two = sequence.run(r, targets, base, frames, start, start_frames, 6, mode, 2, dn2, eval_spp=16,
                           log_every=6, rs=rs)
        assert abs(one["log"][-1]["psnr_db"] - two["log"][-1]["psnr_db"]) < 0.05, (mode, one["log"][-1], two["log"][-1])
    # frame by frame: the same images and, up to atomics order, the same gradients: the same fit
    a = sequence.run(r, targets, base, frames, start, start_frames, 6, "plain", 4, dn, eval_spp=16, log_every=6,
                     rs=rs)
    b = sequence.run(r, targets, base, frames, start, start_frames, 6, "plain", 4, dn, eval_spp=16, log_every=6)
    assert a["batched"] and not b["batched"]
    assert abs(a["log"][-1]["psnr_db"] - b["log"][-1]["psnr_db"]) < 0.05, (a["log"][-1], b["log"][-1])


def test_sequence_fit_resumes_from_a_checkpoint(torch, tmp_path):
    """A fit stopped after its first iteration, written to a checkpoint file
    and resumed, ends where the uninterrupted fit ends (up to the atomics
    order of the adjoint's light and texel sums)."""
    from paper_1910_05200_amd import facert, sequence
    model, scene, _, _ = synth.workload("tiny")
    r = facert.Renderer(model, scene)
    base, frames = sequence.make_truth(2)
    start, start_frames = sequence.make_start(base, frames, seed=7)
    targets = [r.render(facert.params_to_device(sequence.frame_params_np(base, b, p)), 7 + f, 64).clone()
               for f, (b, p) in enumerate(frames)]
    rs = sequence.frame_renderers(model, scene, 2)
    whole = sequence.run(r, targets, base, frames, start, start_frames, 6, "plain", 4, eval_spp=16, log_every=3,
                         rs=rs, seed=3)
    part = sequence.run(r, targets, base, frames, start, start_frames, 6, "plain", 4, eval_spp=16, log_every=3,
                        rs=rs, seed=3, stop_after_s=0.0)
    assert part["iters_done"] == 1 and "state" in part
    path = tmp_path / "seq.npz"
    np.savez(path, **part["state"])
    with np.load(path, allow_pickle=False) as z:
        st = {k: z[k] for k in z.files}
    rest = sequence.run(r, targets, base, frames, start, start_frames, 6, "plain", 4, eval_spp=16, log_every=3,
                        rs=rs, seed=3, state=st)
    assert rest["iters_done"] == 6 and "state" not in rest
    assert [e["iter"] for e in rest["log"]] == [0, 3, 6]
    assert abs(rest["log"][-1]["psnr_db"] - whole["log"][-1]["psnr_db"]) < 0.05, (rest["log"][-1], whole["log"][-1])
    for k in ("alpha", "delta", "lights", "spec", "beta", "rot_deg", "trans_mm"):
        a, b = rest["log"][-1]["errors"][k], whole["log"][-1]["errors"][k]
        assert abs(a - b) <= 2e-3 * max(abs(b), 1e-3), (k, a, b)
