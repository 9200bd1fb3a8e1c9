"""Batched evaluation (fr_batch_*) through the C-ABI.

A batch must give, for every instance, what fr_render / fr_backward give on
that instance's context alone (themselves held to the oracle by
test_gpu_parity): images bitwise, in every launch mode and tile size;
gradients up to the order of their atomic sums.  Bars, of the group's
largest magnitude: 1e-6 for the groups summed in fp64; 2e-5 for the light
and texel adjoints, which each block first sums in fp32 LDS atomics (their
rounding changes with the order in which lanes arrive, from one run to the
next even on one context).  One instance is also held to the oracle
directly, and the full batched workload (32 faces of 5k-40k vertices at
128^2-512^2 and 4-16 spp) to the single-context path after autotuning.
"""
import ctypes as C

import numpy as np
import pytest

from paper_1910_05200_amd import synth
from parity import assert_group_parity, assert_image_parity

pytestmark = pytest.mark.gpu

# (nx, ny, W, H, spp, lights): meshes of 6 to 360 vertices, ragged image
# sizes down to one pixel, 1 to 4 spp, two light-stage sizes; the last face
# is moved out of view (an empty image: no hits, no silhouettes)
SMALL = [(12, 14, 32, 32, 2, 20), (16, 16, 40, 24, 3, 12), (20, 18, 48, 48, 4, 20), (9, 11, 24, 40, 1, 20),
         (3, 2, 1, 1, 1, 12), (10, 10, 24, 24, 2, 20)]
OUT_OF_VIEW = len(SMALL) - 1
GRAD_BAR = 1e-6
GRAD_BAR_LDS32 = 2e-5
LDS32 = ("d_lights", "d_spec")
# A persistent work-queue mode (a fixed grid taking tiles from an atomic
# counter; its run also used tile size 1024) hung on its first GPU run, and
# again after a change that did not find its cause; it is switched off in the
# library (the mode and that tile size are refused) and its cases stay here,
# skipped, until it is back.
_NO_PERSISTENT = pytest.mark.skip(reason="persistent launches hung on the GPU; switched off (FR_EINVAL)")
MODES = [("flat", 0, 512), ("xcd", 1, 256), ("xcd512", 1, 512), ("flat256", 0, 256),
         pytest.param("persistent2", 2, 1024, marks=_NO_PERSISTENT),
         pytest.param("persistent8", 2, 512, marks=_NO_PERSISTENT)]


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no HIP device")
    return T


def _small():
    out = []
    for i, (nx, ny, W, H, spp, nl) in enumerate(SMALL):
        model = synth.make_model(nx, ny, seed=10 + i)
        scene = synth.make_scene(W, H)
        scene.light_geom = synth.light_stage(nl)
        params = synth.make_params(50 + i, n_lights=nl)
        if i == OUT_OF_VIEW:
            params.pose[3] = 5.0
        out.append((model, scene, params, spp))
    return out


def _setup(torch, inst, timing=False):
    from paper_1910_05200_amd import facert
    rs = [facert.Renderer(m, sc) for m, sc, _, _ in inst]
    ps = [facert.params_to_device(p) for _, _, p, _ in inst]
    return rs, ps, facert.Batch(rs, timing=timing)


def _set_mode(batch, mode, tile):
    for k in batch.kinds:
        tiled = k == "edge_secondary"
        batch.set_launch(k, mode, tile if tiled else 0)


def _dls(torch, inst, seed=3):
    rng = np.random.default_rng(seed)
    return [torch.from_numpy(rng.normal(size=(sc.height, sc.width, 3)).astype(np.float32)).cuda()
            for _, sc, _, _ in inst]


def _np(d):
    return {k: v.cpu().numpy() for k, v in d.items()}


@pytest.mark.parametrize("name,mode,tile", MODES)
def test_batch_render_bitwise_matches_single(torch, name, mode, tile):
    inst = _small()
    rs, ps, batch = _setup(torch, inst)
    _set_mode(batch, mode, tile)
    seeds = [1000 + 17 * i for i in range(len(inst))]
    spps = [spp for *_, spp in inst]
    imgs = [x.cpu().numpy() for x in batch.render(ps, seeds, spps)]
    for i, r in enumerate(rs):
        ref = r.render(ps[i], seeds[i], spps[i]).cpu().numpy()
        if i == OUT_OF_VIEW:
            assert not ref.any()
        else:
            assert imgs[i].shape == ref.shape and (ref.size < 64 * 3 or (ref.sum(-1) > 0).mean() > 0.1)
        assert np.array_equal(imgs[i], ref), f"instance {i}: max diff {np.abs(imgs[i] - ref).max()}"


def _assert_grads_close(gb, gs, where):
    for k in gs:
        scale = float(np.abs(gs[k]).max())
        err = float(np.abs(gb[k].astype(np.float64) - gs[k]).max())
        bar = GRAD_BAR_LDS32 if k in LDS32 else GRAD_BAR
        assert err <= bar * scale + 1e-30, f"{where} {k}: max err {err:.3g}, scale {scale:.3g}"


@pytest.mark.parametrize("name,mode,tile", [MODES[0], MODES[1], MODES[4]])
def test_batch_backward_matches_single(torch, name, mode, tile):
    inst = _small()
    rs, ps, batch = _setup(torch, inst)
    _set_mode(batch, mode, tile)
    seeds = [2000 + i for i in range(len(inst))]
    spps = [spp for *_, spp in inst]
    dls = _dls(torch, inst)
    batch.render(ps, seeds, spps)
    gb = [_np(g) for g in batch.backward(dls)]
    for i, r in enumerate(rs):
        r.render(ps[i], seeds[i], spps[i])
        gs = _np(r.backward(dls[i]))
        if i == OUT_OF_VIEW:
            assert not any(np.abs(v).max() > 0 for k, v in gs.items() if k != "d_lights")
        else:
            assert rs[i].W * rs[i].H < 64 or any(np.abs(v).max() > 0 for v in gs.values())
        _assert_grads_close(gb[i], gs, f"instance {i}")


def test_batch_instance_matches_oracle(torch, orc):
    """Instance 2 of a batch against the CPU oracle (pixels 1e-4 relative,
    gradients 1e-4 relative with the group floor of test_gpu_parity)."""
    inst = _small()
    rs, ps, batch = _setup(torch, inst)
    k = 2
    model, scene, params, spp = inst[k]
    seed = 4242
    osc, vm, R = orc.scene_from_model(model, scene, params)
    ref_img = orc.render(osc, seed, spp)
    tosc, _, _ = orc.scene_from_model(model, scene, synth.make_params(77, n_lights=scene.light_geom.shape[0]))
    target = orc.render(tosc, 5, 8)
    dL = (2 * (ref_img - target)).astype(np.float32)
    dls = _dls(torch, inst)
    dls[k] = torch.from_numpy(dL).cuda()
    seeds = [seed + 100 * (i != k) * (i + 1) for i in range(len(inst))]
    imgs = batch.render(ps, seeds, [s for *_, s in inst])
    g = _np(batch.backward(dls)[k])
    worst = assert_image_parity(imgs[k].cpu().numpy().astype(np.float64), ref_img)
    ref = orc.backward(osc, seed, spp, dL.astype(np.float64), flags=7)
    pg = orc.parameter_grads(model, params, vm, R, ref["d_pos"], ref["d_alb"])
    assert_group_parity(g["d_lights"], ref["d_light"], "d_lights")
    assert_group_parity(g["d_spec"], ref["d_spec"], "d_spec")
    assert_group_parity(g["d_albedo"], ref["d_alb"], "d_albedo")
    assert_group_parity(g["d_vertices"], ref["d_pos"], "d_vertices")
    for name in ("d_alpha", "d_beta", "d_delta", "d_pose"):
        assert_group_parity(g[name], pg[name], name)
    print(f"batched instance vs oracle: worst pixel rel {worst:.3g}")


def test_batch_graph_replays_match_eager(torch):
    """One iteration (batched render, per-instance loss, batched adjoint)
    captured in a HIP graph and replayed three times, with eager work and
    synchronisation between replays: every replay equals the eager run."""
    from paper_1910_05200_amd import facert
    inst = _small()
    lib = facert.load()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        rs, ps, batch = _setup(torch, inst)
        seeds = [3000 + i for i in range(len(inst))]
        spps = [spp for *_, spp in inst]
        tgts = [torch.rand((sc.height, sc.width, 3), device="cuda") * 0.05 for _, sc, _, _ in inst]
        imgs = [torch.empty((sc.height, sc.width, 3), device="cuda") for _, sc, _, _ in inst]
        dls = [torch.empty_like(x) for x in imgs]
        losses = [torch.empty((), device="cuda") for _ in inst]
        shapes = lambda r: {"d_lights": (r.n_lights, 3), "d_spec": (r.spec_res ** 2,), "d_vertices": (3, r.V),
                            "d_albedo": (3, r.V), "d_alpha": (r.n_id,), "d_beta": (r.n_exp,),
                            "d_delta": (r.n_alb,), "d_pose": (6,)}
        grads = [{k: torch.empty(v, device="cuda") for k, v in shapes(r).items()} for r in rs]

        def iteration():
            batch.render(ps, seeds, spps, outs=imgs)
            for r, im, t, d, l in zip(rs, imgs, tgts, dls, losses):
                assert lib.fr_loss_l2(r.ctx, im.data_ptr(), t.data_ptr(), d.data_ptr(), l.data_ptr()) == 0
            batch.backward(dls, outs=grads)

        iteration()
        s.synchronize()
        eager_img = [x.cpu().numpy() for x in imgs]
        eager_g = [_np(g) for g in grads]
        eager_l = [float(x) for x in losses]
        batch.capture_begin()
        iteration()
        batch.capture_end()
        for rep in range(3):
            for x in imgs:
                x.zero_()
            for g in grads:
                for v in g.values():
                    v.fill_(7.0)
            junk = torch.randn(1 << 16, device="cuda")
            junk.mul_(2.0)
            s.synchronize()
            batch.graph_launch()
            s.synchronize()
            for i in range(len(inst)):
                assert np.array_equal(imgs[i].cpu().numpy(), eager_img[i]), f"replay {rep} image {i}"
                assert float(losses[i]) == eager_l[i]
                _assert_grads_close(_np(grads[i]), eager_g[i], f"replay {rep} instance {i}")
        # a second capture of the same iteration with other seeds updates the graph in place
        seeds[:] = [x + 1 for x in seeds]
        batch.capture_begin()
        iteration()
        batch.capture_end()
        batch.graph_launch()
        s.synchronize()
        for i, r in enumerate(rs):
            ref = r.render(ps[i], seeds[i], spps[i]).cpu().numpy()
            assert np.array_equal(imgs[i].cpu().numpy(), ref)


def test_batch_tune_keeps_results(torch):
    inst = _small()
    rs, ps, batch = _setup(torch, inst, timing=True)
    seeds = [5000 + i for i in range(len(inst))]
    spps = [spp for *_, spp in inst]
    dls = _dls(torch, inst, seed=9)
    batch.render(ps, seeds, spps)
    batch.backward(dls)
    chosen = batch.tune(trials=1)
    assert "sh_propose" in chosen and "render_adj" in chosen
    t = batch.timing()
    assert t["render"] > 0 and t["backward"] > 0
    imgs = [x.cpu().numpy() for x in batch.render(ps, seeds, spps)]
    gb = [_np(g) for g in batch.backward(dls)]
    for i, r in enumerate(rs):
        assert np.array_equal(imgs[i], r.render(ps[i], seeds[i], spps[i]).cpu().numpy())
        _assert_grads_close(gb[i], _np(r.backward(dls[i])), f"tuned instance {i}")


def test_batch_relaunch_does_not_disturb_enqueued_work(torch):
    """New launch modes and tile sizes while batched work is still queued
    (behind a long matrix product on the same stream), then new sample
    counts: each queued render and backward keeps the tile maps and
    descriptors it was enqueued with.  (The
    first change must not rewrite the tile maps under the queued render: the
    sample counts stay, so no reallocation synchronises the device.)"""
    inst = _small()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        rs, ps, batch = _setup(torch, inst)
        seeds = [6000 + i for i in range(len(inst))]
        spps = [spp for *_, spp in inst]
        batch.render(ps, seeds, spps)                    # configure once
        s.synchronize()
        a = torch.randn(6144, 6144, device="cuda")
        for _ in range(4):
            a = a @ a * 1e-3                             # keeps the stream busy
        first = batch.render(ps, seeds, spps)
        dls = _dls(torch, inst)
        g_first = batch.backward(dls)
        batch.set_launch("sh_propose", 1, 0)
        batch.set_launch("edge_secondary", 0, 512)
        batch.set_launch("pv_propose", 1, 0)
        second = batch.render(ps, [x + 1 for x in seeds], spps)
        for _ in range(4):
            a = a @ a * 1e-3
        batch.set_launch("sh_propose", 0, 0)
        third = batch.render(ps, [x + 2 for x in seeds], [x + 1 for x in spps])
        s.synchronize()
        g_first = [_np(g) for g in g_first]
        for i, r in enumerate(rs):
            r.render(ps[i], seeds[i], spps[i])
            _assert_grads_close(g_first[i], _np(r.backward(dls[i])), f"first backward, instance {i}")
        for i, r in enumerate(rs):
            assert torch.equal(first[i], r.render(ps[i], seeds[i], spps[i])), f"first render, instance {i}"
            assert torch.equal(second[i], r.render(ps[i], seeds[i] + 1, spps[i])), f"second render, instance {i}"
            assert torch.equal(third[i], r.render(ps[i], seeds[i] + 2, spps[i] + 1)), f"third render, instance {i}"


def test_batch_launch_beyond_32bit_work_items(torch):
    """25 instances of 256 x 256 at 64 spp with 42 lights: the shadow-ray and
    shadow-boundary kinds have 25 x 16,384 x 42 tiles of 256 lanes, 4.4e9
    work-items, more than one dispatch dimension holds.  The batched launch
    splits its grid into rows; sampled instances equal their single-context
    renders bit for bit and their gradients as the other batch tests
    require.  (A one-dimensional grid ran only part of the tiles.)"""
    from paper_1910_05200_amd import facert
    n, nl, spp = 25, 42, 64
    model = synth.make_model(6, 6, seed=21)
    scene = synth.make_scene(256, 256)
    scene.light_geom = synth.light_stage(nl)
    params = [synth.make_params(300 + i, n_lights=nl) for i in range(n)]
    rs = [facert.Renderer(model, scene) for _ in range(n)]
    ps = [facert.params_to_device(p) for p in params]
    batch = facert.Batch(rs)
    assert 256 * 256 * spp == facert.FR_CHUNK_MAX
    tiles = n * (256 * 256 * spp // 256) * nl
    assert tiles * 256 > 2 ** 32
    seeds = [7000 + i for i in range(n)]
    imgs = batch.render(ps, seeds, [spp] * n)
    rng = np.random.default_rng(8)
    dls = [torch.from_numpy(rng.normal(size=(256, 256, 3)).astype(np.float32)).cuda() for _ in range(n)]
    gb = batch.backward(dls)
    torch.cuda.synchronize()
    imgs = [x.cpu().numpy() for x in imgs]
    gb = [_np(g) for g in gb]
    batch.close()
    for i in (0, 12, n - 1):
        ref = rs[i].render(ps[i], seeds[i], spp).cpu().numpy()
        assert (ref.sum(-1) > 0).mean() > 0.05
        assert np.array_equal(imgs[i], ref), f"instance {i}: max diff {np.abs(imgs[i] - ref).max()}"
        _assert_grads_close(gb[i], _np(rs[i].backward(dls[i])), f"instance {i}")
    for r in rs:
        r.close()


def test_batch_errors(torch):
    from paper_1910_05200_amd import facert
    inst = _small()
    rs, ps, batch = _setup(torch, inst)
    seeds = [1, 2, 3, 4, 5, 6]
    spps = [spp for *_, spp in inst]
    with pytest.raises(facert.FrError) as e:
        batch.backward(_dls(torch, inst))
    assert e.value.code == -4
    with pytest.raises(facert.FrError) as e:
        facert.Batch([rs[0], rs[0]])
    assert e.value.code == -1
    rr = facert.Renderer(inst[0][0], inst[0][1], refit=True)
    with pytest.raises(facert.FrError):
        facert.Batch([rr, rs[1]])
    with pytest.raises(facert.FrError) as e:
        batch.render(ps, seeds, [1, 1, 1, 1, 1, 4097])
    assert e.value.code == -1
    for bad in [(0, 300), (0, 1024), (2, 512), (-1, 256)]:
        with pytest.raises(facert.FrError):
            batch.set_launch("edge_secondary", *bad)
    with pytest.raises(facert.FrError):             # only edge_secondary takes a tile size
        batch.set_launch("pv_propose", 1, 256)
    batch.render(ps, seeds, spps)
    rs[1].render(ps[1], 9, spps[1])           # instance 1 rendered on its own since
    with pytest.raises(facert.FrError) as e:
        batch.backward(_dls(torch, inst))
    assert e.value.code == -4
    with pytest.raises(facert.FrError) as e:   # the null stream cannot be captured
        batch.capture_begin()
    assert e.value.code == -4
    with pytest.raises(facert.FrError) as e:
        batch.capture_end()
    assert e.value.code == -4
    with pytest.raises(facert.FrError) as e:
        batch.graph_launch()
    assert e.value.code == -4
    lib = facert.load()
    assert lib.fr_batch_render(batch.b, None, None, None, None) == -1


def _with_big(torch):
    """Three small instances and one of 64 x 64 at 1,100 spp (4,505,600
    camera samples, above one chunk)."""
    inst = _small()[:3]
    model = synth.make_model(14, 12, seed=31)
    scene = synth.make_scene(64, 64)
    scene.light_geom = synth.light_stage(20)
    inst.insert(1, (model, scene, synth.make_params(91, n_lights=20), 1100))
    return inst


def test_batch_instance_above_one_chunk(torch):
    """An instance with more camera samples than one chunk goes through its
    context's own chunked render and recomputing adjoint inside the batch:
    its image equals fr_render's bit for bit and its gradients
    fr_backward's; the batched instances beside it are unaffected, also
    after autotuning (which leaves it out)."""
    from paper_1910_05200_amd import facert
    inst = _with_big(torch)
    assert 64 * 64 * 1100 > facert.FR_CHUNK_MAX
    rs, ps, batch = _setup(torch, inst, timing=True)
    seeds = [8000 + i for i in range(len(inst))]
    spps = [spp for *_, spp in inst]
    dls = _dls(torch, inst, seed=5)
    for tuned in (False, True):
        imgs = [x.cpu().numpy() for x in batch.render(ps, seeds, spps)]
        gb = [_np(g) for g in batch.backward(dls)]
        t = batch.timing()
        assert t["render"] > 0 and t["backward"] > 0
        for i, r in enumerate(rs):
            ref = r.render(ps[i], seeds[i], spps[i]).cpu().numpy()
            assert (ref.sum(-1) > 0).mean() > 0.1
            assert np.array_equal(imgs[i], ref), f"tuned={tuned} instance {i}"
            _assert_grads_close(gb[i], _np(r.backward(dls[i])), f"tuned={tuned} instance {i}")
        if not tuned:
            batch.render(ps, seeds, spps)
            batch.backward(dls)
            batch.tune(trials=1)


def test_batch_graph_with_instance_above_one_chunk(torch):
    """The same batch captured in a HIP graph (the large instance's chunk
    loop and its second-stream silhouette work included) and replayed
    twice with eager work in between: each replay equals the eager run.
    The large instance's context keeps timing events, which a capture must
    leave out."""
    from paper_1910_05200_amd import facert
    inst = _with_big(torch)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        rs = [facert.Renderer(m, sc, timing=(spp > 64)) for m, sc, _, spp in inst]
        ps = [facert.params_to_device(p) for _, _, p, _ in inst]
        batch = facert.Batch(rs, timing=True)
        seeds = [8100 + i for i in range(len(inst))]
        spps = [spp for *_, spp in inst]
        dls = _dls(torch, inst, seed=6)
        imgs = [torch.empty((sc.height, sc.width, 3), device="cuda") for _, sc, _, _ in inst]
        shapes = lambda r: {"d_lights": (r.n_lights, 3), "d_spec": (r.spec_res ** 2,), "d_vertices": (3, r.V),
                            "d_albedo": (3, r.V), "d_alpha": (r.n_id,), "d_beta": (r.n_exp,),
                            "d_delta": (r.n_alb,), "d_pose": (6,)}
        grads = [{k: torch.empty(v, device="cuda") for k, v in shapes(r).items()} for r in rs]

        def iteration():
            batch.render(ps, seeds, spps, outs=imgs)
            batch.backward(dls, outs=grads)

        iteration()
        s.synchronize()
        eager_img = [x.cpu().numpy() for x in imgs]
        eager_g = [_np(g) for g in grads]
        batch.capture_begin()
        iteration()
        batch.capture_end()
        for rep in range(2):
            for x in imgs:
                x.zero_()
            for g in grads:
                for v in g.values():
                    v.fill_(7.0)
            junk = torch.randn(1 << 16, device="cuda")
            junk.mul_(2.0)
            s.synchronize()
            batch.graph_launch()
            s.synchronize()
            for i in range(len(inst)):
                assert np.array_equal(imgs[i].cpu().numpy(), eager_img[i]), f"replay {rep} image {i}"
                _assert_grads_close(_np(grads[i]), eager_g[i], f"replay {rep} instance {i}")


def test_batch_full_workload_matches_single(torch):
    """The full batched workload (32 instances, the configuration bench.py
    times with --workload batch, after autotuning): every image bitwise equal
    to its single-context render, every gradient within the atomics-order bar."""
    inst = synth.batch_workload()
    rs, ps, batch = _setup(torch, inst, timing=True)
    seeds = [7000 + i for i in range(len(inst))]
    spps = [spp for *_, spp in inst]
    dls = _dls(torch, inst, seed=11)
    batch.render(ps, seeds, spps)
    batch.backward(dls)
    print({k: v for k, v in batch.tune(trials=1).items()})
    imgs = [x.cpu().numpy() for x in batch.render(ps, seeds, spps)]
    gb = [_np(g) for g in batch.backward(dls)]
    torch.cuda.synchronize()
    for i, r in enumerate(rs):
        ref = r.render(ps[i], seeds[i], spps[i]).cpu().numpy()
        assert np.array_equal(imgs[i], ref), f"instance {i}"
        _assert_grads_close(gb[i], _np(r.backward(dls[i])), f"instance {i}")
    batch.close()
    for r in rs:
        r.close()
