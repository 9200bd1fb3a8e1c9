"""GPU (libfacert through the C-ABI) against the CPU oracle.

Bars: positions and albedo bit-exact (fp64 sums in a fixed order, rounded
once); pixels within 1e-4 relative; gradient components within 1e-4
relative to max(|ref|, 1e-2 * max|ref| of the group).
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


def _case(name):
    model, scene, params, spp = synth.workload(name)
    return model, scene, params, spp


def _renderer(torch, model, scene, refit=False):
    from paper_1910_05200_amd import facert
    return facert.Renderer(model, scene, timing=True, refit=refit)


def _gpu_render(torch, r, params, seed, spp):
    from paper_1910_05200_amd import facert
    p = facert.params_to_device(params)
    img = r.render(p, seed, spp)
    torch.cuda.synchronize()
    return img.cpu().numpy().astype(np.float64), p


@pytest.mark.parametrize("name", ["tiny", "paper"])
def test_blend_bitwise(torch, orc, name):
    model, scene, params, spp = _case(name)
    r = _renderer(torch, model, scene)
    p = {k: torch.from_numpy(getattr(params, k)).cuda() for k in ("alpha", "beta", "delta")}
    v, a = r.blend(p["alpha"], p["beta"], p["delta"], params.pose)
    torch.cuda.synchronize()
    vm, vo, Ao, R = orc.blend(model, params)
    assert np.array_equal(v.cpu().numpy(), vo.astype(np.float32))
    assert np.array_equal(a.cpu().numpy(), Ao.astype(np.float32))


@pytest.mark.parametrize("refit", [False, True])
def test_render_parity_tiny(torch, orc, refit):
    model, scene, params, spp = _case("tiny")
    r = _renderer(torch, model, scene, refit)
    img, _ = _gpu_render(torch, r, params, SEED, spp)
    osc, _, _ = orc.scene_from_model(model, scene, params)
    ref, cnt = orc.render(osc, SEED, spp, counts=True)
    assert (ref.sum(-1) > 0).mean() > 0.2
    worst = assert_image_parity(img, ref)
    st = r.stats()
    assert st["rays_camera"] == cnt.camera and st["rays_shadow"] == cnt.shadow
    print(f"tiny render worst rel {worst:.3g}")


def test_render_deterministic(torch):
    model, scene, params, spp = _case("tiny")
    r = _renderer(torch, model, scene)
    a, _ = _gpu_render(torch, r, params, SEED, spp)
    b, _ = _gpu_render(torch, r, params, SEED, spp)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("nx,ny,W,H,spp", [(7, 11, 37, 23, 3), (20, 9, 1, 1, 1), (16, 16, 300, 5, 2)])
@pytest.mark.parametrize("refit", [False, True])
def test_render_parity_ragged(torch, orc, nx, ny, W, H, spp, refit):
    model = synth.make_model(nx, ny)
    scene = synth.make_scene(W, H)
    params = synth.make_params(5)
    r = _renderer(torch, model, scene, refit)
    img, _ = _gpu_render(torch, r, params, 77, spp)
    osc, _, _ = orc.scene_from_model(model, scene, params)
    assert_image_parity(img, orc.render(osc, 77, spp))


@pytest.mark.parametrize("refit", [False, True])
def test_render_parity_paper_sampled(torch, orc, refit):
    model, scene, params, spp = _case("paper")
    r = _renderer(torch, model, scene, refit)
    img, _ = _gpu_render(torch, r, params, SEED, spp)
    osc, _, _ = orc.scene_from_model(model, scene, params)
    rng = np.random.default_rng(0)
    lit = np.flatnonzero(img.reshape(-1, 3).sum(-1) > 0)
    pix = np.concatenate([rng.choice(lit, 384, replace=False), rng.integers(0, 256 * 256, 128)])
    ref = orc.render_pixels(osc, SEED, spp, pix)
    assert_image_parity(img.reshape(-1, 3)[pix], ref)


def test_lbvh_and_refit_trees_render_identically(torch):
    """The per-evaluation Morton-code tree (default) and the refitted SAH
    tree (FR_REFIT) give the same hits and shadow decisions, hence
    bit-identical images."""
    model, scene, params, spp = _case("paper")
    a, _ = _gpu_render(torch, _renderer(torch, model, scene, False), params, SEED, spp)
    b, _ = _gpu_render(torch, _renderer(torch, model, scene, True), params, SEED, spp)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("nx,ny", [(240, 250), (400, 400)])
def test_large_mesh_trees_match_oracle(torch, orc, nx, ny):
    """Meshes whose per-evaluation tree has 1,298 and 3,569 nodes spanning
    the box pass's 1024-leaf tiles (119k and 318k triangles): the first
    climbs those nodes in LDS, the second, past 2,048, through global
    memory.  Both images equal the refitted tree's bit for bit and the
    oracle's at the pixel bar."""
    model = synth.make_model(nx, ny, seed=5)
    scene = synth.make_scene(48, 40)
    params = synth.make_params(1)
    a, _ = _gpu_render(torch, _renderer(torch, model, scene, False), params, SEED, 2)
    b, _ = _gpu_render(torch, _renderer(torch, model, scene, True), params, SEED, 2)
    assert (a.sum(-1) > 0).mean() > 0.2
    assert np.array_equal(a, b)
    osc, _, _ = orc.scene_from_model(model, scene, params)
    assert_image_parity(a, orc.render(osc, SEED, 2))


def _grad_case(torch, orc, name, terms, chunk=None, refit=False, size=None, n_lights=None):
    from paper_1910_05200_amd import facert
    model, scene, params, spp = _case(name)
    if size:
        scene = synth.make_scene(*size)
    nl = synth.N_LIGHTS
    if n_lights:
        nl = n_lights
        scene.light_geom = synth.light_stage(nl)
        params = synth.make_params(synth.EVAL_SCENE_SEED, n_lights=nl, n_off=min(5, nl // 3))
    tosc, _, _ = orc.scene_from_model(model, scene, synth.make_params(synth.TARGET_SCENE_SEED, n_lights=nl,
                                                                      n_off=min(5, nl // 3)))
    target = orc.render(tosc, synth.TARGET_RENDER_SEED, 16)
    osc, vm, R = orc.scene_from_model(model, scene, params)
    ref_img = orc.render(osc, SEED, spp)
    dL = (2 * (ref_img - target)).astype(np.float32)
    r = _renderer(torch, model, scene, refit)
    r.set_terms(terms)
    if chunk:
        r.set_chunk(chunk)
    img, p = _gpu_render(torch, r, params, SEED, spp)
    g = r.backward(torch.from_numpy(dL).cuda())
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in g.items()}
    flags = (1 if terms & facert.FR_TERM_INTERIOR else 0) | (2 if terms & facert.FR_TERM_PRIMARY else 0) \
        | (4 if terms & facert.FR_TERM_SECONDARY else 0)
    ref = orc.backward(osc, SEED, spp, dL.astype(np.float64), flags=flags)
    pg = orc.parameter_grads(model, params, vm, R, ref["d_pos"], ref["d_alb"])
    return g, ref, pg, r


def _compare(g, ref, pg):
    out = {}
    out["lights"] = assert_group_parity(g["d_lights"], ref["d_light"], "d_lights")
    out["spec"] = assert_group_parity(g["d_spec"], ref["d_spec"], "d_spec")
    out["albedo"] = assert_group_parity(g["d_albedo"], ref["d_alb"], "d_albedo")
    out["vertices"] = assert_group_parity(g["d_vertices"], ref["d_pos"], "d_vertices")
    out["alpha"] = assert_group_parity(g["d_alpha"], pg["d_alpha"], "d_alpha")
    out["beta"] = assert_group_parity(g["d_beta"], pg["d_beta"], "d_beta")
    out["delta"] = assert_group_parity(g["d_delta"], pg["d_delta"], "d_delta")
    out["pose"] = assert_group_parity(g["d_pose"], pg["d_pose"], "d_pose")
    print({k: f"{a:.2g}/{b:.2g}" for k, (a, b) in out.items()})


def test_backward_interior_tiny(torch, orc):
    from paper_1910_05200_amd import facert
    g, ref, pg, _ = _grad_case(torch, orc, "tiny", facert.FR_TERM_INTERIOR)
    _compare(g, ref, pg)


def test_backward_all_terms_tiny(torch, orc):
    g, ref, pg, r = _grad_case(torch, orc, "tiny", 7)
    st = r.stats()
    assert st["rays_edge_secondary"] > 0 and st["rays_edge_primary"] > 0
    _compare(g, ref, pg)


@pytest.mark.parametrize("n_lights", [12, 3])
def test_backward_all_terms_light_groups(torch, orc, n_lights):
    """Light counts that are not a multiple of the shadow-boundary kernel's
    lights per block (a short last group, and a single short group)."""
    g, ref, pg, r = _grad_case(torch, orc, "tiny", 7, n_lights=n_lights)
    assert g["d_lights"].shape[0] == n_lights
    if n_lights >= 12:
        assert r.stats()["rays_edge_secondary"] > 0
    _compare(g, ref, pg)


def test_backward_all_terms_ragged_image(torch, orc):
    """An image whose sides are not multiples of the silhouette sort's
    8x8-pixel tiles or of the screen grid's cells."""
    g, ref, pg, r = _grad_case(torch, orc, "tiny", 7, size=(53, 37))
    assert r.stats()["rays_edge_primary"] > 0
    _compare(g, ref, pg)


def test_backward_on_a_busy_user_stream(torch):
    """The silhouette term runs on the context's second stream, forked from
    and joined back into the caller's stream: on a busy user stream, two
    backward calls queued back to back give the default stream's gradients."""
    model, scene, params, spp = _case("tiny")
    r = _renderer(torch, model, scene)
    dL = torch.from_numpy(np.random.default_rng(5).normal(0, 1, (scene.height, scene.width, 3)).astype(np.float32)).cuda()
    _gpu_render(torch, r, params, SEED, spp)
    g0 = {k: v.cpu().numpy() for k, v in r.backward(dL).items()}
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        a = torch.randn(4096, 4096, device="cuda")
        for _ in range(4):
            a = a @ a * 1e-3                            # keeps the stream busy
        dL2 = dL * 1.0                                  # written on s, read by the backward calls
        g1 = r.backward(dL2)
        g2 = r.backward(dL2)
    s.synchronize()
    for g in (g1, g2):
        for k, v in g0.items():
            got = g[k].cpu().numpy()
            scale = max(float(np.abs(v).max()), 1e-30)
            assert np.abs(got - v).max() <= 1e-6 * scale, k


def test_backward_all_terms_tiny_refit(torch, orc):
    g, ref, pg, _ = _grad_case(torch, orc, "tiny", 7, refit=True)
    _compare(g, ref, pg)


def test_backward_all_terms_tiny_chunked(torch, orc):
    """Render larger than a chunk: no records are kept, the backward
    recomputes hits and visibility chunk by chunk (ragged last chunk)."""
    g, ref, pg, r = _grad_case(torch, orc, "tiny", 7, chunk=5000)
    _compare(g, ref, pg)
    with pytest.raises(Exception):
        r.set_chunk(0)


def test_chunks_that_end_inside_a_pixel(torch, orc):
    """Chunks of 4,999 samples at 4 spp end inside pixels and inside rows:
    the chunked camera step, forward and backward recomputation give the
    unchunked image bit for bit and the oracle's gradients."""
    model, scene, params, spp = _case("tiny")
    assert 4999 % spp != 0
    whole, _ = _gpu_render(torch, _renderer(torch, model, scene), params, SEED, spp)
    g, ref, pg, r = _grad_case(torch, orc, "tiny", 7, chunk=4999)
    _compare(g, ref, pg)
    part, _ = _gpu_render(torch, r, params, SEED, spp)
    assert np.array_equal(whole, part)


def _footprint_cells(osc, faces, W, H, cell=2):
    """Screen cells (cell x cell pixels, a one-pixel border around the
    image) that the triangles' projected bounding boxes cover, summed over
    the triangles: a lower bound of the silhouette setup's cell records."""
    pos = np.asarray(osc.pos, np.float64).T
    cam = np.asarray(osc.cam, np.float64)
    depth = cam[2] - pos[:, 2]
    assert (depth > 0).all()
    qx = W / 2 + (pos[:, 0] - cam[0]) / (depth * osc.pix_scale)
    qy = H / 2 - (pos[:, 1] - cam[1]) / (depth * osc.pix_scale)
    c = lambda p: (p // cell if p >= 0 else -1) + 1
    total = 0
    for f in np.asarray(faces):
        x0, x1 = max(-1, int(np.floor(qx[f].min()))), min(W, int(np.floor(qx[f].max())))
        y0, y1 = max(-1, int(np.floor(qy[f].min()))), min(H, int(np.floor(qy[f].max())))
        total += max(0, c(x1) - c(x0) + 1) * max(0, c(y1) - c(y0) + 1)
    return total


def test_silhouette_sides_walk_the_tree_when_cell_records_overflow(torch, orc):
    """One quad (two triangles) close to the camera, rolled so that a
    boundary edge crosses the image: the triangles' screen footprints need
    more cell records than the store holds (16 per triangle plus one per
    cell), so the silhouette sides are traced through the tree instead.
    Image and gradients still match the oracle."""
    W, H, spp = 40, 36, 2
    model, scene = synth.make_model(2, 2, seed=3), synth.make_scene(W, H)
    params = synth.make_params(5)
    params.pose = np.array([0.0, 0.0, 0.8, -0.02, -0.03, 0.3], np.float32)
    osc, vm, R = orc.scene_from_model(model, scene, params)
    cells = (W // 2 + 2) * (H // 2 + 2)
    assert _footprint_cells(osc, model.faces, W, H) > 16 * model.n_faces + cells
    r = _renderer(torch, model, scene)
    img, _ = _gpu_render(torch, r, params, SEED, spp)
    ref_img = orc.render(osc, SEED, spp)
    assert_image_parity(img, ref_img)
    dL = np.random.default_rng(4).normal(size=ref_img.shape).astype(np.float32)
    g = r.backward(torch.from_numpy(dL).cuda())
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in g.items()}
    ref = orc.backward(osc, SEED, spp, dL.astype(np.float64), flags=7)
    pg = orc.parameter_grads(model, params, vm, R, ref["d_pos"], ref["d_alb"])
    assert r.stats()["rays_edge_primary"] > 0
    _compare(g, ref, pg)


def test_backward_all_terms_paper(torch, orc):
    g, ref, pg, _ = _grad_case(torch, orc, "paper", 7)
    _compare(g, ref, pg)


def test_error_codes(torch):
    from paper_1910_05200_amd import facert
    model, scene, params, spp = _case("tiny")
    r = _renderer(torch, model, scene)
    with pytest.raises(facert.FrError) as e:
        r.backward(torch.zeros((64, 64, 3), device="cuda"))
    assert e.value.code == -4
    p = facert.params_to_device(params)
    with pytest.raises(facert.FrError) as e:
        r.render(p, 1, 0)
    assert e.value.code == -1
    bad = dict(p)
    bad["pose"] = np.array([np.nan, 0, 0, 0, 0, 0], np.float32)
    with pytest.raises(facert.FrError) as e:
        r.render(bad, 1, 4)
    assert e.value.code == -1
    # the context is still usable
    img = r.render(p, 1, 2)
    torch.cuda.synchronize()
    assert float(img.sum()) > 0
