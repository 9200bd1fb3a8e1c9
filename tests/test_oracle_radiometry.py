"""Pins of the oracle's forward estimator against closed forms.

* diffuse, unshadowed: Lambert's polygon formula integrated over each pixel;
* diffuse, shadowed by one triangle: visible light polygon = quad minus the
  triangle's central projection, then Lambert's formula;
* furnace: a closed box of unit emitters around a white plane gives
  radiance exactly 1;
* specular: tiny light and narrow pixel in mirror / off-mirror geometry
  against the textbook Beckmann-tangent form of the microfacet lobe;
* linearity in the light intensities (same seed).
"""
import math

import numpy as np
import pytest

from paper_1910_05200_amd import synth
import closed_forms as cf

SPEC0 = np.zeros(32 * 32)


def _mc_stats(orc, osc, spp, seeds):
    """Mean and standard error over independent seeds (32 seeds keep the
    Student-t tails of the error estimate close to normal)."""
    imgs = np.stack([orc.render(osc, s, spp) for s in seeds])
    return imgs.mean(0), imgs.std(0, ddof=1) / math.sqrt(len(seeds))


def _flat_scene(orc, W, ps, lights, rgb, albedo=1.0, extra_tris=None, spec=SPEC0):
    mesh = synth.flat_grid(9, 0.6, z=0.0, albedo=(albedo,) * 3)
    if extra_tris is not None:
        V = mesh.pos.shape[1]
        tri = np.asarray(extra_tris, np.float32)          # [k][3][3]
        pos = np.concatenate([mesh.pos, tri.reshape(-1, 3).T], axis=1)
        faces = np.concatenate([mesh.faces, V + np.arange(tri.shape[0] * 3, dtype=np.int32).reshape(-1, 3)])
        alb = np.ones((3, pos.shape[1]), np.float32) * albedo
        uv = np.zeros((2, pos.shape[1]), np.float32)
        mesh = synth.Mesh(np.ascontiguousarray(pos), faces, alb, uv)
    return orc.scene_from_mesh(mesh, W, W, [0, 0, 0.5], ps, lights, rgb, spec)


def test_lambert_polygon_unshadowed(orc):
    W, ps = 12, np.float32(0.01)
    lights = np.stack([synth.quad_light([0.15, 0.05, 0.45], [0.2, 0, 0], [0, -0.2, 0]),
                       synth.quad_light([-0.2, -0.1, 0.3], [0.1, 0, 0.05], [0, -0.15, 0])])
    rgb = np.array([[1.0, 0.5, 0.25], [0.3, 0.9, 0.6]])
    osc = _flat_scene(orc, W, ps, lights, rgb, albedo=0.8)
    mean, sem = _mc_stats(orc, osc, 32, range(101, 133))
    nrm = np.array([0, 0, 1.0])
    worst = 0.0
    for py in range(W):
        for px in range(W):
            val = np.zeros(3)
            for qx, qy, w in cf.gauss_pixel(px, py):
                x = cf.camera_plane_point(qx, qy, W, W, osc.cam, float(ps), 0.0)
                for j in range(2):
                    phi = cf.projected_solid_angle(x, nrm, cf.quad_corners(lights[j]))
                    val += w * 0.8 / math.pi * rgb[j] * phi
            z = np.abs(mean[py, px] - val) / np.maximum(sem[py, px], 1e-12)
            worst = max(worst, z.max())
            assert np.all(z < 5.0), (px, py, mean[py, px], val, sem[py, px])
    assert worst > 0.1           # the estimator is noisy, not a copy of the formula


def test_lambert_with_triangle_shadow(orc):
    W, ps = 10, np.float32(0.012)
    light = synth.quad_light([0.35, 0.0, 0.6], [0.15, 0, 0], [0, -0.15, 0])
    # occluder outside the camera frustum, casting a shadow across the view
    tri = [[[0.15, -0.12, 0.3], [0.2, 0.1, 0.3], [0.12, 0.05, 0.32]]]
    osc = _flat_scene(orc, W, ps, light[None], np.array([[1.0, 1.0, 1.0]]), albedo=1.0, extra_tris=tri)
    mean, sem = _mc_stats(orc, osc, 64, range(201, 233))
    corners = cf.quad_corners(light)
    lp, ln = np.asarray(light[:3], float), np.asarray(light[9:12], float)
    nrm = np.array([0, 0, 1.0])
    shaded = 0
    for py in range(W):
        for px in range(W):
            val = 0.0
            for qx, qy, w in cf.gauss_pixel(px, py, 12):
                x = cf.camera_plane_point(qx, qy, W, W, osc.cam, float(ps), 0.0)
                phi = cf.projected_solid_angle(x, nrm, corners)
                shadow = cf.clip_convex(cf.project_to_plane(x, tri[0], lp, ln), corners)
                if len(shadow) >= 3:
                    phi -= cf.projected_solid_angle(x, nrm, shadow)
                val += w * phi / math.pi
            full = sum(w * cf.projected_solid_angle(cf.camera_plane_point(qx, qy, W, W, osc.cam, float(ps), 0.0),
                                                     nrm, corners) / math.pi
                       for qx, qy, w in cf.gauss_pixel(px, py, 4))
            shaded += val < 0.98 * full
            z = abs(mean[py, px, 0] - val) / max(sem[py, px, 0], 1e-12)
            assert z < 5.0, (px, py, mean[py, px, 0], val)
    assert shaded >= 10          # the shadow really crosses the view


def _box_lights(h=1.0):
    """Six inward-facing unit quads forming the cube [-h, h]^3."""
    out = []
    for axis in range(3):
        for s in (-1, 1):
            c = np.zeros(3); c[axis] = s * h
            a = np.zeros(3); a[(axis + 1) % 3] = 2 * h
            b = np.zeros(3); b[(axis + 2) % 3] = 2 * h
            if np.cross(a, b) @ (-c) < 0:
                b = -b
            out.append(synth.quad_light(c, a, b))
    return np.stack(out)


def test_furnace_box(orc):
    W, ps = 8, np.float32(0.05)
    osc = _flat_scene(orc, W, ps, _box_lights(), np.ones((6, 3)), albedo=1.0)
    mean, sem = _mc_stats(orc, osc, 64, range(301, 333))
    z = np.abs(mean - 1.0) / sem
    assert z.max() < 5.0, z.max()
    assert abs(mean.mean() - 1.0) < 5 * sem.mean() / W


def _beckmann_textbook(theta_h, m):
    return math.exp(-math.tan(theta_h) ** 2 / m ** 2) / (math.pi * m ** 2 * math.cos(theta_h) ** 4)


def _vcavity_textbook(n, wo, wi):
    """Cook-Torrance V-cavity masking-shadowing (Cook and Torrance 1982):
    min(1, 2 (n.h)(n.wo)/(wo.h), 2 (n.h)(n.wi)/(wo.h))."""
    h = (wo + wi) / np.linalg.norm(wo + wi)
    nh, oh = float(n @ h), float(wo @ h)
    g1, g2 = 2 * nh * float(n @ wo) / oh, 2 * nh * float(n @ wi) / oh
    return min(1.0, g1, g2), g1, g2


def _point_geometry(orc, view_deg, light_deg, rho, spec, uv_of_pos=None, side=1e-4, spp=4,
                    seed=5):
    """One narrow pixel looking at the centre of a flat receiver, one tiny
    light; camera and light directions in the receiver's x-z plane at the
    given angles from its normal.  The scene is rotated so that the camera
    axis is -z, as the estimator's pinhole model has it.  Returns the pixel
    value (red channel) and the textbook integrand's ingredients at the
    receiver centre."""
    dist_c, dist_l = 0.5, 0.8
    vc, vl = math.radians(view_deg), math.radians(light_deg)
    cam = np.array([math.sin(vc), 0.0, math.cos(vc)]) * dist_c
    lc = np.array([math.sin(vl), 0.0, math.cos(vl)]) * dist_l
    n_l = -lc / np.linalg.norm(lc)
    a = np.cross([0, 1.0, 0], n_l); a /= np.linalg.norm(a)
    b = np.cross(n_l, a)
    light = synth.quad_light(lc, side * a, side * b)
    R = np.array([[math.cos(vc), 0, -math.sin(vc)], [0, 1, 0], [math.sin(vc), 0, math.cos(vc)]])
    cam_r = R @ cam
    assert np.allclose(cam_r, [0, 0, dist_c])
    lg = light.astype(np.float64)
    lg_r = np.concatenate([R @ lg[0:3], R @ lg[3:6], R @ lg[6:9], R @ lg[9:12]])
    mesh = synth.flat_grid(5, 0.2, z=0.0, albedo=(rho,) * 3)
    # the viewed point (the origin) inside a triangle, away from the grid's
    # vertices and edges: a ray through a shared vertex may slip between the
    # triangles' fp32 tests, which would only add noise here
    mesh.pos[0] += np.float32(0.0137)
    mesh.pos[1] += np.float32(0.0071)
    uv = np.full_like(mesh.uv, 0.5) if uv_of_pos is None else uv_of_pos(mesh.pos).astype(np.float32)
    pos = (R @ mesh.pos.astype(np.float64)).astype(np.float32)
    mesh = synth.Mesh(np.ascontiguousarray(pos), mesh.faces, mesh.albedo, np.ascontiguousarray(uv))
    osc = orc.scene_from_mesh(mesh, 1, 1, cam_r, 1e-6, lg_r, [[1.0, 1.0, 1.0]], spec)
    got = orc.render(osc, seed, spp)[0, 0, 0]
    wo = cam / np.linalg.norm(cam)
    wi = lc / np.linalg.norm(lc)
    n = np.array([0, 0, 1.0])
    h = (wo + wi) / np.linalg.norm(wo + wi)
    geo = {"wo": wo, "wi": wi, "n": n, "th": math.acos(min(1.0, float(n @ h))),
           "co": float(n @ wo), "ci": float(n @ wi), "cos_l": float(-n_l @ wi),
           "area": side * side, "d2": dist_l ** 2}
    return got, geo


def _textbook_pixel(geo, rho, ks, m=0.35):
    D = _beckmann_textbook(geo["th"], m)
    G, _, _ = _vcavity_textbook(geo["n"], geo["wo"], geo["wi"])
    irr = geo["cos_l"] * geo["area"] / geo["d2"]
    return rho / math.pi * geo["ci"] * irr + ks * D * G / (4 * geo["co"]) * irr


@pytest.mark.parametrize("view_deg,light_deg", [(0.0, 0.0), (30.0, -30.0), (0.0, 40.0), (20.0, 35.0)])
def test_specular_lobe_point_geometry(orc, view_deg, light_deg):
    """Tiny light, narrow pixel: the pixel value is the integrand at one
    point.  Reference: f_s cos = ks D G / (4 cos_o) with the textbook
    Beckmann form D = exp(-tan^2 th_h / m^2) / (pi m^2 cos^4 th_h)."""
    ks, rho = 0.3, 0.4
    got, geo = _point_geometry(orc, view_deg, light_deg, rho, np.full(1024, ks))
    want = _textbook_pixel(geo, rho, ks)
    assert abs(got - want) < 1e-4 * want, (got, want)


# (view, light, branch): the V-cavity term below 1.  G1 < 1 when the viewer
# grazes, G2 < 1 when the light grazes; in the last two rows both are below
# 1 and the smaller one decides.
VCAVITY_CASES = [(80.0, -40.0, 1), (40.0, -80.0, 2), (70.0, 60.0, 1), (60.0, 70.0, 2), (75.0, -25.0, 1)]


@pytest.mark.parametrize("view_deg,light_deg,branch", VCAVITY_CASES)
def test_specular_vcavity_below_one(orc, view_deg, light_deg, branch):
    """Geometries where the V-cavity term is below 1, specular only (zero
    albedo), against the textbook Cook-Torrance form.  The light is small
    enough that the lobe varies by less than 1e-5 across it.  A V-cavity
    term divided by n.wo instead of wo.h, or G1 and G2 swapped, or G
    dropped, fails here (each is checked to move the value by more than
    the tolerance)."""
    ks = 0.3
    got, geo = _point_geometry(orc, view_deg, light_deg, 0.0, np.full(1024, ks), side=1e-5, spp=64)
    G, g1, g2 = _vcavity_textbook(geo["n"], geo["wo"], geo["wi"])
    assert G < 0.8 and G == (g1 if branch == 1 else g2), (G, g1, g2)
    want = _textbook_pixel(geo, 0.0, ks)
    assert want > 0
    assert abs(got - want) < 1e-4 * want, (got, want, got / want)
    # the test's power: plausible mistakes move the value well outside it
    h = (geo["wo"] + geo["wi"]) / np.linalg.norm(geo["wo"] + geo["wi"])
    nh = float(geo["n"] @ h)
    wrong = [min(1.0, 2 * nh * geo["co"] / geo["co"], 2 * nh * geo["ci"] / geo["co"]),   # / n.wo
             min(1.0, g2 if branch == 1 else g1),                                      # branches swapped
             1.0]                                                                      # G dropped
    for Gw in wrong:
        assert abs(Gw - G) > 1e-2 * G, (Gw, G)


def _ramp_texture(a, bx, by, res=32):
    """Texels of a linear ramp: T[ty][tx] = a + bx (tx + 1/2)/res + by (ty + 1/2)/res.
    Bilinear interpolation between texel centres reproduces it exactly."""
    tx, ty = np.meshgrid(np.arange(res), np.arange(res), indexing="xy")
    return (a + bx * (tx + 0.5) / res + by * (ty + 0.5) / res).ravel()


@pytest.mark.parametrize("u0,v0", [(0.3, 0.6), (0.5 + 1 / 64, 0.27), (0.123, 0.877), (0.01, 0.995),
                                   (0.999, 0.004), (16 / 32, 13 / 32)])
def test_specular_texture_bilinear_lookup(orc, u0, v0):
    """Textured specular map: a linear ramp in both texture directions
    (different slopes) is interpolated exactly by a bilinear lookup between
    texel centres at (i + 1/2)/32, and held at the edge texels' values
    outside [1/64, 63/64] (clamp to edge).  The pixel sees one receiver
    point whose uv is (u0, v0); its value must equal the specular lobe with
    ks = a + bx clamp(u0) + by clamp(v0).  A half-texel shift, swapped
    texture axes, or a wrap instead of a clamp each fail (checked below)."""
    a, bx, by = 0.1, 0.3, 0.15
    tex = _ramp_texture(a, bx, by)
    uv_of_pos = lambda p: np.stack([u0 + 1.5 * p[0].astype(np.float64), v0 + 2.0 * p[1].astype(np.float64)])
    got, geo = _point_geometry(orc, 10.0, -15.0, 0.0, tex, uv_of_pos=uv_of_pos, side=1e-4, spp=16)
    lo, hi = 0.5 / 32, 31.5 / 32
    cl = lambda x: min(max(x, lo), hi)
    ks = a + bx * cl(u0) + by * cl(v0)
    want = _textbook_pixel(geo, 0.0, ks)
    assert abs(got - want) < 1e-4 * want, (got, want, got / want)
    if lo + 0.5 / 32 <= min(u0, v0) and max(u0, v0) <= hi - 0.5 / 32:
        for ks_wrong in (a + bx * (u0 - 0.5 / 32) + by * (v0 - 0.5 / 32),   # half-texel shift
                         a + bx * v0 + by * u0):                            # axes swapped
            assert abs(ks_wrong - ks) > 2e-3 * ks
    if not lo <= u0 <= hi:
        # a wrapping lookup would blend in the opposite edge's texels
        wrap = a + bx * ((u0 * 32 - 0.5) % 32 + 0.5) / 32 + by * cl(v0)
        assert abs(wrap - ks) > 1e-3 * ks


def test_linearity_in_lights(orc):
    model, scene, params, spp = synth.workload("tiny")
    osc, _, _ = orc.scene_from_model(model, scene, params)
    full = orc.render(osc, 42, spp)
    acc = np.zeros_like(full)
    base = osc.light_rgb.copy()
    for j in range(base.shape[0]):
        osc.light_rgb[:] = 0
        osc.light_rgb[j] = base[j]
        acc += orc.render(osc, 42, spp)
    osc.light_rgb[:] = base
    assert np.allclose(acc, full, rtol=1e-12, atol=1e-15)
    assert full.max() > 0
